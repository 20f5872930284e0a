"""Shared helpers of the GPU parity tests: run one workload through the HIP
library (C-ABI via the binding) and through the CPU oracle, and compare every
replica's spins, tracked and recomputed energies, sweep counts, flip counts
and converged flags, bit for bit."""
import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(insts, seed, rule, max_sweeps, until_converged, schedule=-1, runs=None,
            lattice_dims=None, start_spins=None):
    """Load, bind, start and run; ``runs`` is a list of max_sweeps values for
    consecutive calls (resume).  Returns (handle, list of stats)."""
    import paper_0912_3912_amd as sg
    h = sg.load_instance(list(insts), lattice_dims=lattice_dims)
    h.bind()
    if start_spins is None:
        h.init_spins(seed)
    else:
        for (q, r), s in start_spins.items():
            h.set_spins(q, r, s)
    stats = []
    for ms in (runs or [max_sweeps]):
        stats.append(h.run_sweeps(seed=seed, rule=rule, max_sweeps=ms,
                                  until_converged=until_converged, schedule=schedule))
    return h, stats


def oracle_run(inst, seed, rule, max_sweeps, until_converged, runs=None, state=None, threads=0):
    st = state
    for ms in (runs or [max_sweeps]):
        st, _ = oracle.run(inst, seed=seed, rule=rule, max_sweeps=ms,
                           until_converged=until_converged, state=st, threads=threads)
    return st


def compare(h, insts, states, check_recompute=True):
    """Assert that the GPU handle equals the oracle states, replica by replica."""
    E = h.energy()
    Er = h.energy(recompute=True) if check_recompute else E
    sw, fl, cv = h.counters()
    base = 0
    for q, (inst, st) in enumerate(zip(insts, states)):
        R = inst.restarts
        S = h.spins_out_batch(q)
        if not np.array_equal(S, st.spins):
            rr, ii = np.nonzero(S != st.spins)
            raise AssertionError(f"instance {q} ({inst.name}): {rr.size} spins differ, first at restart "
                                 f"{rr[0]} spin {ii[0]}")
        sl = slice(base, base + R)
        for name, got, want in (("energy", E[sl], st.energy), ("recomputed energy", Er[sl], st.energy),
                                ("sweeps", sw[sl], st.sweeps), ("flips", fl[sl], st.flips),
                                ("converged", cv[sl], st.converged)):
            if not np.array_equal(got, want):
                r = int(np.nonzero(got != want)[0][0])
                raise AssertionError(f"instance {q} ({inst.name}) restart {r}: {name} {int(got[r])} != {int(want[r])}")
        base += R


def expected_stats(insts, states_before, states_after):
    attempts = 0
    flips = 0
    for inst, a, b in zip(insts, states_before, states_after):
        da = (b.sweeps - (a.sweeps if a is not None else 0))
        attempts += int((da * inst.n).sum())
        flips += int((b.flips - (a.flips if a is not None else 0)).sum())
    return attempts, flips
