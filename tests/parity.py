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
        for r in range(R):
            s = h.spins_out(q, r)
            k = base + r
            if not np.array_equal(s, st.spins[r]):
                bad = np.nonzero(s != st.spins[r])[0]
                raise AssertionError(f"instance {q} ({inst.name}) restart {r}: {bad.size} spins differ, "
                                     f"first at {bad[:8]}")
            assert E[k] == st.energy[r], (q, r, int(E[k]), int(st.energy[r]))
            assert Er[k] == st.energy[r], (q, r, int(Er[k]), int(st.energy[r]))
            assert sw[k] == st.sweeps[r], (q, r, int(sw[k]), int(st.sweeps[r]))
            assert fl[k] == st.flips[r], (q, r, int(fl[k]), int(st.flips[r]))
            assert cv[k] == st.converged[r], (q, r, int(cv[k]), int(st.converged[r]))
        base += R


def expected_stats(insts, states_before, states_after):
    attempts = 0
    flips = 0
    for inst, a, b in zip(insts, states_before, states_after):
        da = (b.sweeps - (a.sweeps if a is not None else 0))
        attempts += int((da * inst.n).sum())
        flips += int((b.flips - (a.flips if a is not None else 0)).sum())
    return attempts, flips
