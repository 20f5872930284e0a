"""MI355X-native colour-ordered single-spin-flip descent for hyper-Ising
spin glasses (García & Markov, Sec. II eq. (1), Sec. IV, Sec. VI eq. (5)).

This module is a thin ctypes binding of the C-ABI in ``include/sg.h``; every
step of the method runs in the HIP kernels of ``libsg.so``.  PyTorch provides
the device workspace (a uint8 tensor) and the HIP stream.  There is no CPU
fallback: if the library or a GPU is missing the calls raise.

Typical use::

    import paper_0912_3912_amd as sg
    h = sg.load_instance([inst])            # anything with n, ei, ej, J, h, tri, K, ...
    h.bind()                                # torch workspace on cuda:0, current stream
    h.init_spins(seed=7)
    stats = h.run_sweeps(seed=7, rule=sg.GREEDY, max_sweeps=1000)
    E = h.energy()
    s = h.spins_out(0, 0)
"""
from __future__ import annotations

import ctypes
import os
import sys
from typing import Optional, Sequence

_finalizing = sys.is_finalizing  # kept: module globals may be cleared at shutdown

import numpy as np

__all__ = [
    "GREEDY", "GREEDY_TIE", "FM", "SCHED_AUTO", "SCHED_PHASE", "SCHED_GRAPH",
    "SCHED_LATTICE", "SCHED_BLOCK", "SCHED_QUEUE", "SCHED_FM", "SCHED_FIELDS", "SCHED_DENSE", "SGError", "Handle",
    "load_instance", "load_dense", "exact_ground_state",
    "run_sweeps", "energy", "spins_out", "library_path", "lib", "run_group", "group_scratch_bytes", "philox_word0",
]

SG_OK, SG_ENOTCONV, SG_EINVAL, SG_ERANGE, SG_ENOMEM, SG_EDEVICE, SG_ESTATE = 0, 1, -1, -2, -3, -4, -5
GREEDY, GREEDY_TIE, FM = 0, 1, 2
SCHED_AUTO, SCHED_PHASE, SCHED_GRAPH, SCHED_LATTICE, SCHED_BLOCK, SCHED_QUEUE, SCHED_FM, SCHED_FIELDS, SCHED_DENSE = (
    -1, 0, 1, 3, 4, 5, 6, 7, 8)
_STATUS = {SG_EINVAL: "SG_EINVAL", SG_ERANGE: "SG_ERANGE", SG_ENOMEM: "SG_ENOMEM",
           SG_EDEVICE: "SG_EDEVICE", SG_ESTATE: "SG_ESTATE", SG_ENOTCONV: "SG_ENOTCONV"}

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libsg.so")


class SGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class InstanceDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("ei", ctypes.c_void_p), ("ej", ctypes.c_void_p), ("J", ctypes.c_void_p),
                ("h", ctypes.c_void_p), ("t", ctypes.c_int64), ("tri", ctypes.c_void_p),
                ("K", ctypes.c_void_p), ("colour", ctypes.c_void_p), ("dims", ctypes.c_int32 * 3),
                ("instance_id", ctypes.c_uint32), ("restarts", ctypes.c_int32)]


class RunParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("rule", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("until_converged", ctypes.c_int32), ("schedule", ctypes.c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_int64), ("flips", ctypes.c_int64), ("sweeps_max", ctypes.c_int64),
                ("n_unconverged", ctypes.c_int32), ("schedule_used", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class InstanceInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("colours", ctypes.c_int32), ("m", ctypes.c_int64),
                ("t", ctypes.c_int64), ("restarts", ctypes.c_int32), ("lattice", ctypes.c_int32),
                ("replica_base", ctypes.c_int64)]


_lib = None

# (name, restype, argtypes) of every exported C-ABI function
_P = ctypes.c_void_p
SIGNATURES = [
    ("sg_load_instance", ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    ("sg_load_dense", ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    ("sg_exact_ground_state", ctypes.c_int32, [_P, _P, _P, _P, _P, ctypes.c_int64]),
    ("sg_workspace_bytes", ctypes.c_int32, [_P, _P]),
    ("sg_instance_info_get", ctypes.c_int32, [_P, ctypes.c_int32, _P, _P]),
    ("sg_bind", ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P]),
    ("sg_bind_noalloc", ctypes.c_int32, [_P, _P]),
    ("sg_init_spins", ctypes.c_int32, [_P, ctypes.c_uint64]),
    ("sg_set_spins", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    ("sg_run_sweeps", ctypes.c_int32, [_P, _P, _P]),
    ("sg_group_scratch_bytes", ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    ("sg_run_group", ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, ctypes.c_uint64, _P, _P]),
    ("sg_energy", ctypes.c_int32, [_P, _P, ctypes.c_int32]),
    ("sg_replica_counters", ctypes.c_int32, [_P, _P, _P, _P]),
    ("sg_spins_out", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    ("sg_spins_out_batch", ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P]),
    ("sg_best", ctypes.c_int32, [_P, _P, _P]),
    ("sg_solve", ctypes.c_int32, [_P, _P, _P, _P, _P]),
    ("sg_tune", ctypes.c_int32, [_P, ctypes.c_char_p, ctypes.c_int64]),
    ("sg_query", ctypes.c_int32, [_P, ctypes.c_char_p, _P]),
    ("sg_philox_word0", ctypes.c_int32, [_P, _P, ctypes.c_int64, ctypes.c_uint64, _P]),
    ("sg_free", ctypes.c_int32, [_P]),
    ("sg_last_error", ctypes.c_char_p, []),
    ("sg_version", ctypes.c_char_p, []),
]


def lib():
    """Load libsg.so (raises if it was not built: there is no fallback)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                              "or python paper_0912_3912_amd/_build.py")
        # PyTorch ships its own HIP and HSA runtimes under the same soname.
        # Loading torch first makes the dynamic linker resolve the library's
        # libamdhip64.so.7 to that copy, so the device memory and streams the
        # binding takes from torch belong to the runtime the library calls;
        # loaded the other way round, the process would hold two runtimes.
        import torch  # noqa: F401
        L = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status < 0:
        raise SGError(status, lib().sg_last_error().decode())
    return status


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class DenseDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nterms", ctypes.c_int64), ("mask", ctypes.c_void_p),
                ("coef", ctypes.c_void_p), ("instance_id", ctypes.c_uint32), ("restarts", ctypes.c_int32)]


class Handle:
    """One loaded batch of instances (the C handle plus the arrays it keeps
    alive).  Instances are duck-typed: attributes n, ei, ej, J and optionally
    h, tri, K, colour, dims, instance_id, restarts; with ``dense`` they are
    dense hyper-Ising instances with attributes n, masks, coefs and
    optionally instance_id, restarts."""

    def __init__(self, instances: Sequence, lattice_dims: Optional[Sequence] = None, dense: bool = False):
        self._keep = []
        if dense:
            self._load_dense(instances)
            return
        descs = (InstanceDesc * len(instances))()
        self.sizes = []
        self.restarts = []
        for k, inst in enumerate(instances):
            d = descs[k]
            n = int(inst.n)
            ei, ej, J = _i32(inst.ei), _i32(inst.ej), _i32(inst.J)
            h = getattr(inst, "h", None)
            h = None if h is None else _i32(h)
            tri = getattr(inst, "tri", None)
            tri = np.zeros(0, np.int32) if tri is None else _i32(tri).reshape(-1)
            K = getattr(inst, "K", None)
            K = np.zeros(0, np.int32) if K is None else _i32(K)
            col = getattr(inst, "colour", None)
            col = None if col is None else _i32(col)
            self._keep += [ei, ej, J, h, tri, K, col]
            d.n = n
            d.m = ei.shape[0]
            d.ei, d.ej, d.J, d.h = _ptr(ei), _ptr(ej), _ptr(J), _ptr(h)
            d.t = tri.shape[0] // 3
            d.tri, d.K, d.colour = _ptr(tri), _ptr(K), _ptr(col)
            dims = None
            if lattice_dims is not None:
                dims = lattice_dims[k]
            elif getattr(inst, "dims", None) is not None:
                dims = inst.dims
            if dims is not None:
                dd = list(dims) + [0] * (3 - len(dims))
                d.dims[0], d.dims[1], d.dims[2] = int(dd[0]), int(dd[1]), int(dd[2])
            d.instance_id = int(getattr(inst, "instance_id", 0)) & 0xFFFFFFFF
            d.restarts = int(getattr(inst, "restarts", 1))
            self.sizes.append(n)
            self.restarts.append(d.restarts)
        self._h = ctypes.c_void_p()
        _check(lib().sg_load_instance(descs, len(instances), ctypes.byref(self._h)))
        self._keep = None  # the library copied the arrays
        self.workspace = None
        self.total_replicas = int(sum(self.restarts))

    def _load_dense(self, instances):
        descs = (DenseDesc * len(instances))()
        self.sizes = []
        self.restarts = []
        for k, inst in enumerate(instances):
            d = descs[k]
            masks = np.ascontiguousarray(inst.masks, dtype=np.uint64)
            coefs = np.ascontiguousarray(inst.coefs, dtype=np.int64)
            self._keep += [masks, coefs]
            d.n = int(inst.n)
            d.nterms = masks.shape[0]
            d.mask, d.coef = _ptr(masks), _ptr(coefs)
            d.instance_id = int(getattr(inst, "instance_id", 0)) & 0xFFFFFFFF
            d.restarts = int(getattr(inst, "restarts", 1))
            self.sizes.append(d.n)
            self.restarts.append(d.restarts)
        self._h = ctypes.c_void_p()
        _check(lib().sg_load_dense(descs, len(instances), ctypes.byref(self._h)))
        self._keep = None
        self.workspace = None
        self.total_replicas = int(sum(self.restarts))

    # ------------------------------------------------------------------ host-only
    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64()
        _check(lib().sg_workspace_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def info(self, inst: int = 0) -> dict:
        inf = InstanceInfo()
        col = np.zeros(self.sizes[inst], np.int32)
        _check(lib().sg_instance_info_get(self._h, inst, ctypes.byref(inf), _ptr(col)))
        d = {k: getattr(inf, k) for k, _ in InstanceInfo._fields_}
        d["colour"] = col
        return d

    # ------------------------------------------------------------------ device
    def bind(self, workspace=None, stream=None, device=None):
        """Bind a torch uint8 device tensor (allocated here when None) and a
        torch stream (the current stream when None)."""
        import torch
        if workspace is None:
            dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
            workspace = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(workspace.device)
        self.workspace = workspace
        self.stream = stream
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().sg_bind(self._h, ctypes.c_void_p(workspace.data_ptr()),
                             workspace.numel() * workspace.element_size(), ctypes.c_void_p(sp)))
        return self

    def bind_raw(self, dev_ptr: int, nbytes: int, stream_ptr: int = 0):
        _check(lib().sg_bind(self._h, ctypes.c_void_p(dev_ptr), nbytes, ctypes.c_void_p(stream_ptr)))
        return self

    def bind_noalloc(self, stream=None, device=None):
        """Bind to the library's static device workspace (no allocation by
        the library or by torch) and a torch stream (current stream when
        None).  Every handle bound this way on one GPU shares that workspace."""
        import torch
        if stream is None:
            dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
            stream = torch.cuda.current_stream(dev)
        self.workspace = None
        self.stream = stream
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(lib().sg_bind_noalloc(self._h, ctypes.c_void_p(sp)))
        return self

    def init_spins(self, seed: int):
        _check(lib().sg_init_spins(self._h, seed & 0xFFFFFFFFFFFFFFFF))

    def set_spins(self, inst: int, r: int, s):
        s = np.ascontiguousarray(s, dtype=np.int8)
        if s.shape[0] != self.sizes[inst]:
            raise ValueError("wrong spin count")
        _check(lib().sg_set_spins(self._h, inst, r, _ptr(s)))

    def run_sweeps(self, seed: int, rule: int = GREEDY, max_sweeps: int = 10000,
                   until_converged: bool = True, schedule: int = SCHED_AUTO) -> dict:
        p = RunParams(seed & 0xFFFFFFFFFFFFFFFF, rule, max_sweeps, int(until_converged), schedule)
        st = RunStats()
        status = _check(lib().sg_run_sweeps(self._h, ctypes.byref(p), ctypes.byref(st)))
        d = st.as_dict()
        d["status"] = status
        return d

    def energy(self, recompute: bool = False) -> np.ndarray:
        E = np.zeros(self.total_replicas, np.int64)
        _check(lib().sg_energy(self._h, _ptr(E), int(recompute)))
        return E

    def counters(self):
        sw = np.zeros(self.total_replicas, np.int64)
        fl = np.zeros(self.total_replicas, np.int64)
        cv = np.zeros(self.total_replicas, np.int8)
        _check(lib().sg_replica_counters(self._h, _ptr(sw), _ptr(fl), _ptr(cv)))
        return sw, fl, cv

    def spins_out(self, inst: int, r: int) -> np.ndarray:
        s = np.zeros(self.sizes[inst], np.int8)
        _check(lib().sg_spins_out(self._h, inst, r, _ptr(s)))
        return s

    def spins_out_batch(self, inst: int, r0: int = 0, count: Optional[int] = None) -> np.ndarray:
        """Spins of restarts r0 .. r0+count-1 (all by default), shape (count, n)."""
        if count is None:
            count = self.restarts[inst] - r0
        s = np.zeros((count, self.sizes[inst]), np.int8)
        _check(lib().sg_spins_out_batch(self._h, inst, r0, count, _ptr(s)))
        return s

    def best(self):
        ni = len(self.sizes)
        E = np.zeros(ni, np.int64)
        r = np.zeros(ni, np.int32)
        _check(lib().sg_best(self._h, _ptr(E), _ptr(r)))
        return E, r

    def solve(self, seed: int, rule: int = GREEDY, max_sweeps: int = 10000, until_converged: bool = True,
              schedule: int = SCHED_AUTO):
        """init_spins(seed), run_sweeps(...), best() in one library call;
        returns (stats, E_best, r_best)."""
        p = RunParams(seed & 0xFFFFFFFFFFFFFFFF, rule, max_sweeps, int(until_converged), schedule)
        st = RunStats()
        ni = len(self.sizes)
        E = np.zeros(ni, np.int64)
        r = np.zeros(ni, np.int32)
        status = _check(lib().sg_solve(self._h, ctypes.byref(p), ctypes.byref(st), _ptr(E), _ptr(r)))
        d = st.as_dict()
        d["status"] = status
        return d, E, r

    def tune(self, key: str, value: int):
        _check(lib().sg_tune(self._h, key.encode(), int(value)))
        return self

    def query(self, key: str) -> int:
        v = ctypes.c_int64()
        _check(lib().sg_query(self._h, key.encode(), ctypes.byref(v)))
        return int(v.value)

    def free(self):
        if self._h:
            lib().sg_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        # A handle still alive at interpreter shutdown is left to the process
        # exit: by then the HIP runtime, and any profiler attached to it, may
        # already be finalised, so sg_free's event and stream destruction
        # would call into a torn-down runtime.  Call free() explicitly.
        if _finalizing is None or _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


# module-level names matching the C-ABI calls -------------------------------


def load_instance(instances, lattice_dims=None) -> Handle:
    if not isinstance(instances, (list, tuple)):
        instances = [instances]
    return Handle(instances, lattice_dims)


def exact_ground_state(inst, seed_spins=None, max_nodes: int = 0):
    """Exact ground state by branch-and-bound (Sec. III) on the host CPU.
    Returns (energy, spins, nodes, proven): proven is False when the node
    budget ran out first (then the state is only the best found)."""
    h = Handle.__new__(Handle)  # reuse the descriptor marshalling of Handle
    h._keep = []
    descs = (InstanceDesc * 1)()
    d = descs[0]
    ei, ej, J = _i32(inst.ei), _i32(inst.ej), _i32(inst.J)
    hv = getattr(inst, "h", None)
    hv = None if hv is None else _i32(hv)
    tri = getattr(inst, "tri", None)
    tri = np.zeros(0, np.int32) if tri is None else _i32(tri).reshape(-1)
    K = getattr(inst, "K", None)
    K = np.zeros(0, np.int32) if K is None else _i32(K)
    d.n, d.m = int(inst.n), ei.shape[0]
    d.ei, d.ej, d.J, d.h = _ptr(ei), _ptr(ej), _ptr(J), _ptr(hv)
    d.t, d.tri, d.K = tri.shape[0] // 3, _ptr(tri), _ptr(K)
    d.restarts = 1
    seed = None if seed_spins is None else np.ascontiguousarray(seed_spins, dtype=np.int8)
    out = np.zeros(int(inst.n), np.int8)
    E = ctypes.c_int64()
    nodes = ctypes.c_int64()
    st = lib().sg_exact_ground_state(ctypes.byref(d), _ptr(seed), _ptr(out), ctypes.byref(E), ctypes.byref(nodes),
                                     int(max_nodes))
    _check(st)
    return int(E.value), out, int(nodes.value), st == SG_OK


def load_dense(instances) -> Handle:
    """Dense hyper-Ising instances (at most 64 spins, couplings over any set of
    spins, int64 coefficients), e.g. from ``factoring.factoring_instance``."""
    if not isinstance(instances, (list, tuple)):
        instances = [instances]
    return Handle(instances, dense=True)


def _handle_array(handles):
    arr = (ctypes.c_void_p * len(handles))()
    for k, h in enumerate(handles):
        arr[k] = h._h.value if isinstance(h._h, ctypes.c_void_p) else h._h
    return arr


def group_scratch_bytes(handles) -> int:
    """Device scratch bytes that run_group needs for these handles."""
    b = ctypes.c_uint64()
    _check(lib().sg_group_scratch_bytes(_handle_array(handles), len(handles), ctypes.byref(b)))
    return int(b.value)


def run_group(handles, scratch, seed: int, rule: int = GREEDY, max_sweeps: int = 16, until_converged: bool = True):
    """One step of continuous batching (sg_run_group): the replicas of every
    handle in one launch.  ``scratch`` is a torch device tensor of at least
    group_scratch_bytes(handles) bytes.  Returns (stats dict, per-handle
    count of replicas not converged)."""
    arr = _handle_array(handles)
    p = RunParams(seed & 0xFFFFFFFFFFFFFFFF, rule, max_sweeps, int(until_converged), SCHED_AUTO)
    st = RunStats()
    unc = (ctypes.c_int32 * len(handles))()
    status = _check(lib().sg_run_group(arr, len(handles), ctypes.byref(p), ctypes.c_void_p(scratch.data_ptr()),
                                       scratch.numel() * scratch.element_size(), unc, ctypes.byref(st)))
    d = st.as_dict()
    d["status"] = status
    return d, [int(v) for v in unc]


def philox_word0(ctr, seed: int):
    """Word 0 of Philox4x32-10 computed on the GPU for an (N, 4) uint32 torch
    device tensor of counters under key ``seed``; returns an (N,) tensor."""
    import torch
    if ctr.dtype != torch.int32 and ctr.dtype != torch.uint32:
        raise TypeError("counters must be a 32-bit integer tensor")
    ctr = ctr.contiguous()
    if ctr.dim() != 2 or ctr.shape[1] != 4 or not ctr.is_cuda:
        raise ValueError("counters must be an (N, 4) device tensor")
    out = torch.empty(ctr.shape[0], dtype=ctr.dtype, device=ctr.device)
    sp = torch.cuda.current_stream(ctr.device).cuda_stream
    _check(lib().sg_philox_word0(ctypes.c_void_p(ctr.data_ptr()), ctypes.c_void_p(out.data_ptr()), ctr.shape[0],
                                 seed & 0xFFFFFFFFFFFFFFFF, ctypes.c_void_p(sp)))
    return out


def run_sweeps(handle: Handle, **kw) -> dict:
    return handle.run_sweeps(**kw)


def energy(handle: Handle, recompute: bool = False) -> np.ndarray:
    return handle.energy(recompute)


def spins_out(handle: Handle, inst: int, r: int) -> np.ndarray:
    return handle.spins_out(inst, r)
