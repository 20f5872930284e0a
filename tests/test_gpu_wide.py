"""GPU parity of instances beyond the packed words, which the library stores
in its wide form: couplings, fields and hyper-couplings anywhere in int32
(per-spin |h| + sum|J| + sum|K| up to 2^31 - 1, so that dE = 2 s f reaches
2^32), spins with more than 255 triples, and more restarts than one launch
dimension holds.  Spins, tracked and recomputed int64 energies, sweeps,
flips and converged flags are compared with the oracle bit for bit."""
import numpy as np
import pytest

import instances as gen
import oracle
from parity import compare, expected_stats, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

GREEDY, TIE = 0, 1


def _recoef(inst, seed, j_max, h_max=0, k_max=None, name=""):
    """The same structure with coefficients drawn uniformly in [-max, max]."""
    rng = np.random.default_rng(seed)
    k_max = j_max if k_max is None else k_max
    J = rng.integers(-j_max, j_max + 1, size=inst.m).astype(np.int32)
    h = rng.integers(-h_max, h_max + 1, size=inst.n).astype(np.int32) if h_max else None
    K = rng.integers(-k_max, k_max + 1, size=inst.t).astype(np.int32)
    return inst.replace(J=J, h=h, K=K, name=name or inst.name + "_wide")


def _check(insts, seed, rule, max_sweeps, uc, schedule=-1, runs=None, dims=None, threads=0):
    import paper_0912_3912_amd as sg
    log(f"wide case: {[i.name for i in insts][:3]} seed={seed} rule={rule} sweeps={runs or max_sweeps} uc={uc} "
        f"schedule={schedule}")
    h, stats = gpu_run(insts, seed, rule, max_sweeps, uc, schedule=schedule, runs=runs, lattice_dims=dims)
    states = [oracle_run(i, seed, rule, max_sweeps, uc, runs=runs, threads=threads) for i in insts]
    compare(h, insts, states)
    if runs is None:
        att, fl = expected_stats(insts, [None] * len(insts), states)
        assert stats[0]["attempts"] == att and stats[0]["flips"] == fl
    return h, stats


@pytest.mark.parametrize("rule,ms,uc", [(GREEDY, 10000, True), (TIE, 7, False)])
def test_er_triples_large_coefficients(gpu, rule, ms, uc):
    inst = _recoef(gen.erdos_renyi_triples(3000, seed=2), seed=1, j_max=10**5, h_max=10**5).replace(restarts=4,
                                                                                                     instance_id=9)
    h, _ = _check([inst], seed=3, rule=rule, max_sweeps=ms, uc=uc)
    assert h.query("wide_instances") == 1
    h.free()


def test_lattice_large_couplings(gpu):
    base = gen.lattice((32, 32, 32), seed=4, h_range=(-2, 2))
    inst = _recoef(base, seed=5, j_max=10**5, h_max=3).replace(colour=base.colour, instance_id=2)
    h, _ = _check([inst], seed=7, rule=TIE, max_sweeps=20, uc=False, dims=[(32, 32, 32)])
    h.free()
    h, st = _check([inst], seed=7, rule=GREEDY, max_sweeps=10000, uc=True, dims=[(32, 32, 32)])
    assert st[0]["schedule_used"] == 0  # the wide form runs on the per-phase method
    h.free()


def test_fields_near_the_int32_limit(gpu):
    """Every spin's |h| + sum|J| + sum|K| just below 2^31: fields use the whole
    int32 range and dE = 2 s f exceeds it."""
    base = gen.random_regular3(2000, seed=3, instance_id=4)
    lim = 2**31 - 1
    # degree 3, plus a field: each |coefficient| <= lim / 4 keeps every spin within the limit
    inst = _recoef(base, seed=6, j_max=lim // 4, h_max=lim // 4).replace(restarts=6)
    field = np.zeros(inst.n, np.int64)
    np.add.at(field, inst.ei, np.abs(inst.J.astype(np.int64)))
    np.add.at(field, inst.ej, np.abs(inst.J.astype(np.int64)))
    field += np.abs(inst.h.astype(np.int64))
    assert field.max() <= lim and field.max() > 2**31 - 2**30
    h, _ = _check([inst], seed=8, rule=GREEDY, max_sweeps=10000, uc=True)
    h.free()
    h, _ = _check([inst], seed=8, rule=TIE, max_sweeps=5, uc=False, schedule=1)  # graph schedule
    h.free()


def test_many_triples_per_spin(gpu):
    """A spin in more than 255 triples (beyond the packed form's per-row count)."""
    rng = np.random.default_rng(11)
    n = 40
    tri = set()
    while len(tri) < 4000:
        t = tuple(sorted(rng.choice(n, 3, replace=False).tolist()))
        tri.add(t)
    tri = np.array(sorted(tri), np.int32)
    counts = np.bincount(tri.reshape(-1), minlength=n)
    assert counts.max() > 255
    ei, ej = np.triu_indices(n, 1)
    keep = rng.random(ei.size) < 0.3
    inst = gen.Instance(n=n, ei=ei[keep], ej=ej[keep], J=rng.integers(-3, 4, keep.sum()).astype(np.int32),
                        h=rng.integers(-2, 3, n).astype(np.int32), tri=tri,
                        K=rng.integers(-2, 3, tri.shape[0]).astype(np.int32), instance_id=13, restarts=16,
                        name="dense_triples")
    h, _ = _check([inst], seed=2, rule=GREEDY, max_sweeps=10000, uc=True)
    assert h.query("wide_instances") == 1
    h.free()
    h, _ = _check([inst], seed=2, rule=TIE, max_sweeps=9, uc=False, runs=[4, 0, 5])
    h.free()


def test_more_restarts_than_one_launch_dimension(gpu):
    inst = gen.random_small(24, seed=21, n_triples=10).replace(restarts=70000, instance_id=21)
    h, _ = _check([inst], seed=4, rule=GREEDY, max_sweeps=10000, uc=True, threads=16)
    E, r = h.best()
    ref = oracle.run(inst, seed=4, threads=16)[0]
    assert int(E[0]) == int(ref.energy.min()) and int(r[0]) == int(np.argmin(ref.energy))
    h.free()


def test_mixed_handle_and_set_spins(gpu):
    """Packed and wide instances in one handle under SG_SCHED_AUTO; an explicit
    start on the wide one."""
    import paper_0912_3912_amd as sg
    narrow = gen.chimera(4, 4, seed=2, instance_id=1, restarts=40)
    wide = _recoef(gen.erdos_renyi_triples(1000, seed=5), seed=3, j_max=5000, h_max=300).replace(instance_id=2,
                                                                                                restarts=3)
    insts = [narrow, wide]
    h, _ = _check(insts, seed=5, rule=GREEDY, max_sweeps=10000, uc=True)
    assert h.query("wide_instances") == 1
    h.free()
    rng = np.random.default_rng(2)
    s0 = np.where(rng.random(wide.n) < 0.5, -1, 1).astype(np.int8)
    h = sg.load_instance([wide]).bind()
    h.init_spins(1)
    h.set_spins(0, 1, s0)
    assert int(h.energy()[1]) == oracle.energy(wide, s0) == int(h.energy(recompute=True)[1])
    st = h.run_sweeps(seed=1, rule=GREEDY, max_sweeps=10000, until_converged=True)
    ref = oracle.ReplicaState(wide.n, wide.restarts)
    ref0, _ = oracle.run(wide, seed=1, max_sweeps=0)
    ref.spins[:] = ref0.spins
    ref.spins[1] = s0
    ref.energy[:] = [oracle.energy(wide, ref.spins[r]) for r in range(wide.restarts)]
    ref, _ = oracle.run(wide, seed=1, rule=GREEDY, max_sweeps=10000, until_converged=True, state=ref)
    compare(h, [wide], [ref])
    assert st["n_unconverged"] == 0
    h.free()


def _check_fm(insts, seed, max_passes=1000, uc=True, runs=None, threads=16):
    """The pass-based search (Sec. IV, Fig. 3) on the GPU and in the oracle."""
    import paper_0912_3912_amd as sg
    log(f"wide fm case: {[i.name for i in insts][:3]} seed={seed} passes={runs or max_passes} uc={uc}")
    h = sg.load_instance(list(insts)).bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=sg.FM, max_sweeps=mp, until_converged=uc) for mp in (runs or [max_passes])]
    assert all(s["schedule_used"] == sg.SCHED_FM for s in stats)
    states = []
    for inst in insts:
        st = None
        for mp in (runs or [max_passes]):
            st, _ = oracle.fm(inst, seed=seed, max_passes=mp, until_converged=uc, state=st, threads=threads)
        states.append(st)
    compare(h, insts, states)
    if runs is None:
        assert stats[0]["attempts"] == sum(int((st.sweeps * i.n).sum()) for i, st in zip(insts, states))
        assert stats[0]["flips"] == sum(int(st.flips.sum()) for st in states)
    return h, stats


@pytest.mark.parametrize("n", [1, 2, 63, 65, 300, 700, 4096])
def test_fm_large_coefficients_ragged(gpu, n):
    """The pass-based search on the wide form: sizes around the 64-spin lane
    stride, couplings, fields and hyper-couplings up to 10^5."""
    base = gen.random_small(n, seed=n + 40, p_edge=min(1.0, 8.0 / max(n, 1)), n_triples=n // 2)
    inst = _recoef(base, seed=n, j_max=10**5, h_max=10**5).replace(restarts=5, instance_id=n + 7)
    h, _ = _check_fm([inst], seed=n + 1)
    big = max([int(np.abs(a).max()) for a in (inst.J, inst.h, inst.K) if a is not None and a.size] + [0])
    assert h.query("wide_instances") == int(big > 127)
    h.free()


def test_fm_fields_near_the_int32_limit(gpu):
    """Half-gains of the whole int32 range; move gains beyond it."""
    base = gen.random_regular3(600, seed=3, instance_id=4)
    lim = 2**31 - 1
    inst = _recoef(base, seed=6, j_max=lim // 4, h_max=lim // 4).replace(restarts=6)
    h, _ = _check_fm([inst], seed=8)
    assert h.query("wide_instances") == 1
    h.free()
    h, _ = _check_fm([inst], seed=8, uc=False, runs=[2, 0, 3])
    h.free()


def test_fm_many_triples_per_spin(gpu):
    rng = np.random.default_rng(12)
    n = 40
    tri = set()
    while len(tri) < 4000:
        tri.add(tuple(sorted(rng.choice(n, 3, replace=False).tolist())))
    tri = np.array(sorted(tri), np.int32)
    assert np.bincount(tri.reshape(-1), minlength=n).max() > 255
    inst = gen.Instance(n=n, ei=np.zeros(0, np.int32), ej=np.zeros(0, np.int32), J=np.zeros(0, np.int32),
                        h=rng.integers(-2, 3, n).astype(np.int32), tri=tri,
                        K=rng.integers(-2, 3, tri.shape[0]).astype(np.int32), instance_id=14, restarts=9,
                        name="fm_dense_triples")
    h, _ = _check_fm([inst], seed=3)
    assert h.query("wide_instances") == 1
    h.free()


def test_fm_packed_and_wide_in_one_call(gpu):
    """Instances on the lane kernel, the wavefront kernel and the wide form in
    one call."""
    lanes = gen.chimera(4, 4, seed=2, instance_id=1, restarts=70)
    waves = gen.random_small(200, seed=9, p_edge=0.04, n_triples=50, j_range=(-60, 60), h_range=(-9, 9),
                             k_range=(-9, 9)).replace(restarts=5, instance_id=3)
    wide = _recoef(gen.erdos_renyi_triples(500, seed=5), seed=3, j_max=5000, h_max=300).replace(instance_id=2,
                                                                                               restarts=3)
    h, st = _check_fm([lanes, waves, wide], seed=5)
    assert h.query("wide_instances") == 1 and h.query("last_fm_lanes") == 70
    assert st[0]["n_unconverged"] == 0
    h.free()
