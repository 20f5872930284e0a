"""Element-wise oracle parity at the sizes of the benchmark configurations
that the other GPU tests do not reach:

* the 10^6-spin periodic 3-D lattice under GREEDY until converged (the
  stopping rule of Sec. IV, Fig. 3), on the schedule SG_SCHED_AUTO picks and
  on the per-phase method;
* the factoring hypergraphs of 612171 and 580003 at the widths the benchmark
  runs (10 + 10 free bits: 20 spins, 3135 terms; Sec. VI eqs. (6)-(8)) under
  the pass-based search and the colour sweep;
* the pass-based search (Sec. IV, Fig. 3) on 64 Chimera instances with all
  256 restarts each, every replica compared.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import instances as gen
import oracle
from paper_0912_3912_amd.factoring import factoring_instance
from parity import compare, gpu_run, log

pytestmark = pytest.mark.gpu

GREEDY, TIE, FM = 0, 1, 2


def _pool(jobs, workers=16):
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda f: f(), jobs))


@pytest.mark.parametrize("schedule", [-1, 0])
def test_cubic100_greedy_until_converged(gpu, schedule):
    inst = gen.cfg2_cubic100()
    log(f"cubic100 GREEDY until converged, schedule {schedule}")
    h, stats = gpu_run([inst], seed=7, rule=GREEDY, max_sweeps=10000, until_converged=True, schedule=schedule,
                       lattice_dims=[(100, 100, 100)])
    ref, status = oracle.run(inst, seed=7, rule=oracle.GREEDY, max_sweeps=10000, until_converged=True, threads=1)
    assert status == 0
    compare(h, [inst], [ref])
    assert stats[0]["attempts"] == int(ref.sweeps[0]) * inst.n
    assert stats[0]["flips"] == int(ref.flips[0])
    assert stats[0]["n_unconverged"] == 0
    log(f"  sweeps {int(ref.sweeps[0])}, E {int(ref.energy[0])}, schedule used {stats[0]['schedule_used']}")
    h.free()


@pytest.mark.parametrize("N", [612171, 580003])
@pytest.mark.parametrize("rule", [FM, GREEDY])
def test_factoring_bench_widths(gpu, N, rule):
    import paper_0912_3912_amd as sg
    b = N.bit_length() // 2
    # 8 instances of the same hypergraph under distinct instance ids, 64 starts each
    ds = [factoring_instance(N, b, b, instance_id=100 + k, restarts=64) for k in range(8)]
    assert ds[0].n == 20 and len(ds[0].coefs) == 3135
    log(f"factoring {N}: rule {rule}, {len(ds)} x 64 starts")
    h = sg.load_dense(ds).bind()
    h.init_spins(7)
    st = h.run_sweeps(seed=7, rule=rule, max_sweeps=1000, until_converged=True)
    assert st["schedule_used"] == sg.SCHED_DENSE
    if rule == FM:
        states = _pool([lambda d=d: oracle.dense_fm(d, seed=7, max_passes=1000, until_converged=True)[0]
                        for d in ds])
    else:
        states = _pool([lambda d=d: oracle.dense_run(d, seed=7, rule=GREEDY, max_sweeps=1000,
                                                     until_converged=True)[0] for d in ds])
    compare(h, ds, states)
    assert st["attempts"] == sum(int((s.sweeps * d.n).sum()) for d, s in zip(ds, states))
    assert st["flips"] == sum(int(s.flips.sum()) for s in states)
    # under the pass-based search some starts reach the ground energy (a factorisation): for 612171
    # the paper reports about 2.5% of starts, so 512 starts all missing would be a 1e-5 event
    if rule == FM:
        hits = sum(int((s.energy == ds[0].ground_energy()).sum()) for s in states)
        log(f"  {hits} of {64 * len(ds)} starts factor {N}")
        if N == 612171:
            assert hits > 0
    h.free()


def test_fm_chimera_all_restarts(gpu):
    import paper_0912_3912_amd as sg
    insts = gen.cfg3_chimera_batch(count=64, restarts=256)
    log("fm chimera: 64 instances x 256 restarts, every replica")
    h = sg.load_instance(insts).bind()
    h.init_spins(7)
    st = h.run_sweeps(seed=7, rule=FM, max_sweeps=1000, until_converged=True)
    assert st["schedule_used"] == sg.SCHED_FM
    states = [oracle.fm(inst, seed=7, max_passes=1000, until_converged=True, threads=16)[0] for inst in insts]
    compare(h, insts, states)
    assert st["attempts"] == sum(int((s.sweeps * i.n).sum()) for i, s in zip(insts, states))
    assert st["flips"] == sum(int(s.flips.sum()) for s in states)
    h.free()
