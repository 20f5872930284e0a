"""GPU parity of dense hyper-Ising instances (couplings over any set of at
most 64 spins, int64 coefficients; one lane per replica) against the
oracle's dense model, bit for bit, for colour sweeps (both rules) and the
pass-based search; and the factoring hypergraphs of Sec. VI."""
import numpy as np
import pytest

import instances as gen
import oracle
from paper_0912_3912_amd.factoring import factoring_instance
from parity import compare, log

pytestmark = pytest.mark.gpu

GREEDY, TIE, FM = 0, 1, 2


def _oracle(d, seed, rule, ms, uc, runs=None, state=None):
    st = state
    for m in (runs or [ms]):
        if rule == FM:
            st, _ = oracle.dense_fm(d, seed=seed, max_passes=m, until_converged=uc, state=st)
        else:
            st, _ = oracle.dense_run(d, seed=seed, rule=rule, max_sweeps=m, until_converged=uc, state=st)
    return st


def _check(ds, seed, rule, ms=1000, uc=True, runs=None):
    import paper_0912_3912_amd as sg
    log(f"dense case: {[d.name for d in ds][:3]} seed={seed} rule={rule} runs={runs or ms} uc={uc}")
    h = sg.load_dense(list(ds)).bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=rule, max_sweeps=m, until_converged=uc) for m in (runs or [ms])]
    assert all(s["schedule_used"] == sg.SCHED_DENSE for s in stats)
    states = [_oracle(d, seed, rule, ms, uc, runs) for d in ds]
    compare(h, ds, states)
    if runs is None:
        assert stats[0]["attempts"] == sum(int((st.sweeps * d.n).sum()) for d, st in zip(ds, states))
        assert stats[0]["flips"] == sum(int(st.flips.sum()) for st in states)
    return h


@pytest.mark.parametrize("rule", [GREEDY, TIE, FM])
@pytest.mark.parametrize("n,nterms,order", [(1, 1, 1), (2, 3, 2), (13, 40, 4), (33, 150, 4), (64, 300, 6)])
def test_random_dense(gpu, rule, n, nterms, order):
    d = gen.random_dense(n, nterms, max_order=order, coef_range=(-1000, 1000), seed=n, restarts=150,
                         instance_id=n + 5)
    uc = rule != TIE
    _check([d], seed=n + 1, rule=rule, ms=1000 if uc else 9, uc=uc)


def test_batch_resume_and_set_spins(gpu):
    import paper_0912_3912_amd as sg
    ds = [gen.random_dense(20, 80, seed=s, restarts=70, instance_id=s) for s in range(3)]
    _check(ds, seed=4, rule=TIE, uc=True, runs=[2, 3, 0, 1000])
    _check(ds, seed=4, rule=FM, uc=True, runs=[1, 1, 1000])
    # an explicit start: energy of the start and the run from it
    d = ds[0].replace(restarts=1)
    s0 = np.where(np.arange(d.n) % 3 == 0, -1, 1).astype(np.int8)
    h = sg.load_dense([d]).bind()
    h.set_spins(0, 0, s0)
    assert int(h.energy()[0]) == oracle.dense_energy(d, s0)
    h.run_sweeps(seed=2, rule=GREEDY)
    st = oracle.ReplicaState(d.n, 1)
    st.spins[0] = s0
    st, _ = oracle.dense_run(d, seed=2, state=st)
    compare(h, [d], [st])


@pytest.mark.parametrize("N,nx,ny", [(21, 1, 2), (143, 3, 3), (437, 4, 4), (3127, 5, 6)])
def test_factoring_instances(gpu, N, nx, ny):
    d = factoring_instance(N, nx, ny, restarts=200, instance_id=N)
    h = _check([d], seed=3, rule=FM)
    E, r = h.best()
    S = h.spins_out(0, int(r[0]))
    x, y = d.decode(S)
    log(f"N={N}: best energy {int(E[0])} (factorisation at {d.ground_energy()}), x*y = {x * y}")
    _check([d], seed=3, rule=GREEDY)


def test_wrong_schedule_and_mixed_rules(gpu):
    import paper_0912_3912_amd as sg
    h = sg.load_dense([gen.random_dense(8, 10, seed=1)]).bind()
    h.init_spins(1)
    with pytest.raises(sg.SGError) as e:
        h.run_sweeps(seed=1, schedule=sg.SCHED_PHASE)
    assert e.value.status == sg.SG_EINVAL
