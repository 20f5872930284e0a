"""CPU oracle for the colour-ordered single-spin-flip descent -- TEST
INFRASTRUCTURE ONLY.

A plain, slow, sequential C implementation (``sg_oracle.c``) driven through
ctypes.  Only the test suite, the smoke check and the benchmark's CPU
baseline use it; the HIP library never imports, links or calls it, and it
shares no code with the library.  Every function follows the paper
(García & Markov): energy from Sec. II eq. (1) and Sec. VI eq. (5), move gains
from Sec. IV, random starts, passes until no improvement and multi-start from
Sec. IV/Fig. 3.  The colour-ordered schedule, tie rule and counter-based RNG
are this project's readings (see the C file's header).

Pins (what checks this oracle against something other than itself) live in
``tests/test_oracle_pins.py``, ``tests/test_oracle_fm.py``,
``tests/test_factoring.py`` and ``tests/test_oracle_philox.py``; the last pins
the Philox4x32-10 generator to its published known-answer vectors and to the
independent engine of rocRAND's source header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GREEDY = 0
GREEDY_TIE = 1
ORDER_ASCENDING, ORDER_DESCENDING, ORDER_SIMULTANEOUS = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over restarts)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    lib.oracle_energy.restype = i64
    lib.oracle_energy.argtypes = [i32, i64, P, P, P, P, i64, P, P, P]
    lib.oracle_first_fit_colouring.restype = i32
    lib.oracle_first_fit_colouring.argtypes = [i32, i64, P, P, i64, P, P]
    lib.oracle_colouring_is_proper.restype = ctypes.c_int
    lib.oracle_colouring_is_proper.argtypes = [i32, i64, P, P, i64, P, P]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_run.argtypes = [i32, i64, P, P, P, P, i64, P, P, P, u32, i32, u64, i32, i32,
                               i32, i32, i32, P, P, P, P, P, i32]
    lib.oracle_trace.restype = i64
    lib.oracle_trace.argtypes = [i32, i64, P, P, P, P, i64, P, P, P, u32, u32, u64, i32, i32,
                                 i32, i32, i32, P, P, P, P, P, P, i64]
    lib.oracle_trace_unchecked.restype = i64
    lib.oracle_trace_unchecked.argtypes = [i32, i64, P, P, P, P, i64, P, P, P, u64, i32, i32,
                                           i32, P, P, i64]
    lib.oracle_brute_force.restype = i64
    lib.oracle_brute_force.argtypes = [i32, i64, P, P, P, P, i64, P, P, P, P]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_philox4x32_10.argtypes = [P, P, P]
    lib.oracle_philox_stream.restype = None
    lib.oracle_philox_stream.argtypes = [u64, u32, u32, u32, u32, i64, P]
    lib.oracle_fm.restype = ctypes.c_int
    lib.oracle_fm.argtypes = [i32, i64, P, P, P, P, i64, P, P, u32, i32, u64, i32, i32, i32, P, P, P, P, P,
                              i32]
    lib.oracle_dense_energy.restype = i64
    lib.oracle_dense_energy.argtypes = [i32, i64, P, P, P]
    lib.oracle_dense_run.restype = ctypes.c_int
    lib.oracle_dense_run.argtypes = [i32, i64, P, P, u32, i32, u64, i32, i32, i32, i32, P, P, P, P, P]
    lib.oracle_dense_fm.restype = ctypes.c_int
    lib.oracle_dense_fm.argtypes = [i32, i64, P, P, u32, i32, u64, i32, i32, i32, P, P, P, P, P]
    lib.oracle_dense_brute.restype = i64
    lib.oracle_dense_brute.argtypes = [i32, i64, P, P, P, P]
    lib.oracle_best.restype = i32
    lib.oracle_best.argtypes = [i32, P, P]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _arrs(inst):
    h = inst.h
    tri = np.ascontiguousarray(inst.tri, dtype=np.int32).reshape(-1)
    return (inst.n, inst.m, _p(inst.ei), _p(inst.ej), _p(inst.J), _p(h), inst.t, _p(tri),
            _p(inst.K)), tri


def energy(inst, s: np.ndarray) -> int:
    """E(s) of Sec. II eq. (1) / Sec. VI eq. (5); each term counted once."""
    s = np.ascontiguousarray(s, dtype=np.int8)
    args, _keep = _arrs(inst)
    return int(_load().oracle_energy(*args, _p(s)))


def first_fit_colouring(inst) -> np.ndarray:
    """First-fit colouring of the primal graph (edges and triple pairs)."""
    col = np.empty(inst.n, dtype=np.int32)
    tri = np.ascontiguousarray(inst.tri, dtype=np.int32).reshape(-1)
    nc = _load().oracle_first_fit_colouring(inst.n, inst.m, _p(inst.ei), _p(inst.ej), inst.t,
                                            _p(tri), _p(col))
    if nc < 0:
        raise MemoryError("oracle colouring failed")
    return col


def colouring_is_proper(inst, colour) -> bool:
    colour = np.ascontiguousarray(colour, dtype=np.int32)
    tri = np.ascontiguousarray(inst.tri, dtype=np.int32).reshape(-1)
    return bool(_load().oracle_colouring_is_proper(inst.n, inst.m, _p(inst.ei), _p(inst.ej),
                                                   inst.t, _p(tri), _p(colour)))


class ReplicaState:
    """Spins (restarts x n, external order) plus per-restart counters."""

    def __init__(self, n, restarts):
        self.spins = np.zeros((restarts, n), dtype=np.int8)
        self.energy = np.zeros(restarts, dtype=np.int64)
        self.sweeps = np.zeros(restarts, dtype=np.int64)
        self.flips = np.zeros(restarts, dtype=np.int64)
        self.converged = np.zeros(restarts, dtype=np.int8)

    def copy(self):
        c = ReplicaState(self.spins.shape[1], self.spins.shape[0])
        for k in ("spins", "energy", "sweeps", "flips", "converged"):
            setattr(c, k, getattr(self, k).copy())
        return c


def run(inst, seed: int, rule: int = GREEDY, max_sweeps: int = 10000,
        until_converged: bool = True, state: Optional[ReplicaState] = None,
        order: int = ORDER_ASCENDING, threads: int = 0, use_colour: bool = True):
    """Run every restart of ``inst``.  With ``state`` None the random starts
    are drawn; otherwise the run continues from ``state`` (updated in place).
    Returns (state, status) with status 0, or 1 when until_converged and some
    restart hit the sweep cap."""
    init = state is None
    if init:
        state = ReplicaState(inst.n, inst.restarts)
    args, _keep = _arrs(inst)
    colour = inst.colour if use_colour else None
    st = _load().oracle_run(*args, _p(colour), inst.instance_id & 0xFFFFFFFF, inst.restarts,
                            seed & 0xFFFFFFFFFFFFFFFF, rule, max_sweeps, int(until_converged),
                            order, int(init), _p(state.spins), _p(state.energy),
                            _p(state.sweeps), _p(state.flips), _p(state.converged), threads)
    if st < 0:
        raise ValueError(f"oracle_run failed with status {st}")
    return state, st


def fm(inst, seed: int, max_passes: int = 1000, until_converged: bool = True,
       state: Optional[ReplicaState] = None, threads: int = 0):
    """The paper's pass-based local search (Sec. IV, Fig. 3) on every restart:
    max-gain moves (lowest index on equal gains) with locking and
    hill-climbing, the best state of each pass kept, passes until one brings
    no improvement.  ``state.sweeps`` counts passes and ``state.flips`` the
    moves kept.  With ``state`` None the random starts are drawn.  Returns
    (state, status)."""
    init = state is None
    if init:
        state = ReplicaState(inst.n, inst.restarts)
    args, _keep = _arrs(inst)
    st = _load().oracle_fm(*args, inst.instance_id & 0xFFFFFFFF, inst.restarts, seed & 0xFFFFFFFFFFFFFFFF,
                           max_passes, int(until_converged), int(init), _p(state.spins), _p(state.energy),
                           _p(state.sweeps), _p(state.flips), _p(state.converged), threads)
    if st < 0:
        raise ValueError(f"oracle_fm failed with status {st}")
    return state, st


def _dense(d):
    masks = np.ascontiguousarray(d.masks, np.uint64)
    coefs = np.ascontiguousarray(d.coefs, np.int64)
    return masks, coefs


def dense_energy(d, s) -> int:
    """E(s) = -sum_t coef_t prod_{i in t} s_i (Sec. VI eq. (5)) of a dense instance."""
    masks, coefs = _dense(d)
    s = np.ascontiguousarray(s, np.int8)
    return int(_load().oracle_dense_energy(d.n, masks.shape[0], _p(masks), _p(coefs), _p(s)))


def dense_run(d, seed, rule=GREEDY, max_sweeps=10000, until_converged=True, state=None):
    """Colour sweeps on every restart of a dense instance (same rules, start
    and stopping rule as ``run``).  Returns (state, status)."""
    init = state is None
    if init:
        state = ReplicaState(d.n, d.restarts)
    masks, coefs = _dense(d)
    st = _load().oracle_dense_run(d.n, masks.shape[0], _p(masks), _p(coefs), d.instance_id & 0xFFFFFFFF,
                                  d.restarts, seed & 0xFFFFFFFFFFFFFFFF, rule, max_sweeps, int(until_converged),
                                  int(init), _p(state.spins), _p(state.energy), _p(state.sweeps),
                                  _p(state.flips), _p(state.converged))
    if st < 0:
        raise ValueError(f"oracle_dense_run failed with status {st}")
    return state, st


def dense_fm(d, seed, max_passes=1000, until_converged=True, state=None):
    """The pass-based search (as ``fm``) on every restart of a dense instance."""
    init = state is None
    if init:
        state = ReplicaState(d.n, d.restarts)
    masks, coefs = _dense(d)
    st = _load().oracle_dense_fm(d.n, masks.shape[0], _p(masks), _p(coefs), d.instance_id & 0xFFFFFFFF,
                                 d.restarts, seed & 0xFFFFFFFFFFFFFFFF, max_passes, int(until_converged), int(init),
                                 _p(state.spins), _p(state.energy), _p(state.sweeps), _p(state.flips),
                                 _p(state.converged))
    if st < 0:
        raise ValueError(f"oracle_dense_fm failed with status {st}")
    return state, st


def dense_brute_force(d):
    """(E_min, one minimising state, number of minimising states), n <= 30."""
    masks, coefs = _dense(d)
    best = np.zeros(d.n, np.int8)
    cnt = np.zeros(1, np.int64)
    e = _load().oracle_dense_brute(d.n, masks.shape[0], _p(masks), _p(coefs), _p(best), _p(cnt))
    if e == np.iinfo(np.int64).min:
        raise ValueError("brute force needs 1 <= n <= 30")
    return int(e), best, int(cnt[0])


def trace(inst, seed, restart=0, rule=GREEDY, max_sweeps=100, until_converged=True,
          order=ORDER_ASCENDING, spins=None, trace_cap=100000, keep_spins=True):
    """One restart with the tracked energy (and spins) after every colour
    phase.  Returns dict(E=[...], S=[...] or None, spins, sweeps, flips,
    converged)."""
    s = np.empty(inst.n, np.int8) if spins is None else np.ascontiguousarray(spins, np.int8).copy()
    sw = np.zeros(1, np.int64)
    fl = np.zeros(1, np.int64)
    cv = np.zeros(1, np.int8)
    tE = np.zeros(trace_cap, np.int64)
    tS = np.zeros((trace_cap, inst.n), np.int8) if keep_spins else None
    args, _keep = _arrs(inst)
    ln = _load().oracle_trace(*args, _p(inst.colour), inst.instance_id & 0xFFFFFFFF, restart,
                              seed, rule, max_sweeps, int(until_converged), order,
                              int(spins is None), _p(s), _p(sw), _p(fl), _p(cv), _p(tE),
                              _p(tS), trace_cap)
    if ln < 0:
        raise ValueError(f"oracle_trace failed with status {ln}")
    return dict(E=tE[:ln].copy(), S=None if tS is None else tS[:ln].copy(), spins=s,
                sweeps=int(sw[0]), flips=int(fl[0]), converged=bool(cv[0]))


def trace_unchecked(inst, colour, spins, seed=0, rule=GREEDY, max_sweeps=4,
                    order=ORDER_ASCENDING, trace_cap=1000):
    s = np.ascontiguousarray(spins, np.int8).copy()
    colour = np.ascontiguousarray(colour, np.int32)
    tE = np.zeros(trace_cap, np.int64)
    args, _keep = _arrs(inst)
    ln = _load().oracle_trace_unchecked(*args, _p(colour), seed, rule, max_sweeps, order,
                                        _p(s), _p(tE), trace_cap)
    return tE[:ln].copy(), s


def brute_force(inst):
    """(E_min, one minimising state, number of minimising states), n <= 30."""
    best = np.zeros(inst.n, np.int8)
    deg = np.zeros(1, np.int64)
    args, _keep = _arrs(inst)
    e = _load().oracle_brute_force(*args, _p(best), _p(deg))
    if e == np.iinfo(np.int64).min:
        raise ValueError("brute force needs 1 <= n <= 30")
    return int(e), best, int(deg[0])


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    _load().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_stream(seed, c0, c1, c2, c3, count):
    out = np.zeros((count, 4), np.uint32)
    _load().oracle_philox_stream(seed, c0, c1, c2, c3, count, _p(out))
    return out


def best(energies) -> tuple:
    e = np.ascontiguousarray(energies, np.int64)
    be = np.zeros(1, np.int64)
    r = _load().oracle_best(e.shape[0], _p(e), _p(be))
    return int(r), int(be[0])


def lower_bound(inst) -> int:
    """Sec. III eq. (2) extended by the hyper-couplings: -sum|J|-sum|h|-sum|K|."""
    return -int(np.abs(inst.J.astype(np.int64)).sum() + np.abs(inst.h_or_zero().astype(np.int64)).sum()
                + np.abs(inst.K.astype(np.int64)).sum())
