"""GPU parity of the paper's pass-based local search (rule SG_RULE_FM: one
wavefront per replica, max-gain moves with locking and hill-climbing, best
prefix kept, passes until no improvement) against the CPU oracle, bit for
bit: spins, tracked and recomputed energies, pass counts, moves kept,
converged flags."""
import numpy as np
import pytest

import instances as gen
import oracle
from parity import compare, log

pytestmark = pytest.mark.gpu

FM = 2


def _oracle(insts, seed, max_passes, uc, runs=None, threads=0):
    out = []
    for inst in insts:
        st = None
        for mp in (runs or [max_passes]):
            st, _ = oracle.fm(inst, seed=seed, max_passes=mp, until_converged=uc, state=st, threads=threads)
        out.append(st)
    return out


def _check(insts, seed, max_passes=1000, uc=True, runs=None, key32=1, waves=0, lanes=1, lane_restarts=0):
    import paper_0912_3912_amd as sg
    log(f"fm case: {[i.name for i in insts][:4]} seed={seed} passes={runs or max_passes} uc={uc} key32={key32} "
        f"waves={waves} lanes={lanes} lane_restarts={lane_restarts}")
    h = sg.load_instance(list(insts))
    h.tune("fm_key32", key32)
    h.tune("fm_waves", waves)
    h.tune("fm_lanes", lanes)
    h.tune("fm_lane_restarts", lane_restarts)
    h.bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=FM, max_sweeps=mp, until_converged=uc) for mp in (runs or [max_passes])]
    assert all(s["schedule_used"] == sg.SCHED_FM for s in stats)
    states = _oracle(insts, seed, max_passes, uc, runs)
    compare(h, insts, states)
    if runs is None:
        assert stats[0]["attempts"] == sum(int((st.sweeps * i.n).sum()) for i, st in zip(insts, states))
        assert stats[0]["flips"] == sum(int(st.flips.sum()) for st in states)
    return h


@pytest.mark.parametrize("lanes", [1, 0])
@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 129, 700])
def test_ragged_random_with_triples(gpu, n, lanes):
    inst = gen.random_small(n, seed=n, p_edge=min(1.0, 8.0 / max(n, 1)), n_triples=n // 2, j_range=(-15, 15),
                            h_range=(-7, 7), k_range=(-7, 7)).replace(restarts=4, instance_id=n)
    _check([inst], seed=n + 3, lanes=lanes)


def _small_coef(n, restarts, seed=None):
    """Random instance whose per-spin sum of |coefficients| stays within one
    byte (the lane kernel's range)."""
    seed = n if seed is None else seed
    return gen.random_small(n, seed=seed, p_edge=min(1.0, 6.0 / max(n, 1)), n_triples=n // 3, j_range=(-5, 5),
                            h_range=(-3, 3), k_range=(-3, 3)).replace(restarts=restarts, instance_id=n + 1000,
                                                                       name=f"lo{n}")


@pytest.mark.parametrize("n", [1, 2, 31, 33, 64, 129, 256, 257, 511, 513, 700, 1000, 1024])
def test_lane_kernel_ragged(gpu, n):
    """One replica per lane: sizes around the 32-spin groups, the 4-spin gain
    words and the move-tag widths (n <= 256, 512, 1024), 70 restarts (a
    second wavefront item, partly filled)."""
    inst = _small_coef(n, 70)
    h = _check([inst], seed=n + 5)
    assert h.query("last_fm_lanes") == 70 and h.query("last_fm_waves") == 0


@pytest.mark.parametrize("nr", [64, 128, 256])
def test_lane_kernel_refill(gpu, nr):
    """A wavefront refills its lanes from its item's restarts as replicas
    finish: items of 64, 128 and 256 restarts give the oracle's results."""
    insts = [gen.chimera(8, 8, seed=s, instance_id=s, restarts=200) for s in range(2)] + [_small_coef(300, 90)]
    h = _check(insts, seed=4, lane_restarts=nr)
    assert h.query("last_fm_lane_nr") == nr and h.query("last_fm_lanes") == 490


@pytest.mark.parametrize("waves", [2, 4])
def test_lane_kernel_shared_items(gpu, waves):
    """Several wavefronts of a workgroup share one item's restarts (one
    counter): the results are the oracle's."""
    import paper_0912_3912_amd as sg
    insts = [gen.chimera(8, 8, seed=s + 5, instance_id=s, restarts=300) for s in range(2)]
    log(f"fm lane workgroups of {waves} wavefronts")
    h = sg.load_instance(insts)
    h.tune("fm_lane_waves", waves)
    h.bind()
    h.init_spins(8)
    st = h.run_sweeps(seed=8, rule=FM, max_sweeps=1000, until_converged=True)
    assert st["schedule_used"] == sg.SCHED_FM and h.query("last_fm_lanes") == 600
    compare(h, insts, _oracle(insts, 8, 1000, True))


def test_lane_kernel_lattice_regular_resume(gpu):
    insts = [gen.lattice((20, 20), seed=2, restarts=65), gen.lattice((32, 32), seed=3, restarts=9),
             gen.random_regular3(1000, seed=4, instance_id=9).replace(restarts=5)]
    _check(insts, seed=5, uc=True, runs=[1, 2, 0, 1000])
    h = _check(insts, seed=6, max_passes=3, uc=False)
    assert h.query("last_fm_lanes") == 79


def test_lane_and_wave_kernels_in_one_call(gpu):
    """Instances within the lane kernel's range next to ones beyond it (more
    than 1024 spins, or a per-spin sum of |coefficients| above 127) in one
    call: both kernels run, every replica matches the oracle."""
    big = gen.erdos_renyi_triples(3000, seed=8)
    wide = gen.random_small(200, seed=3, p_edge=0.2, n_triples=0, j_range=(-15, 15), instance_id=44).replace(
        restarts=3)
    insts = [gen.chimera(6, 6, seed=1, instance_id=1, restarts=80), big, wide, _small_coef(100, 3)]
    h = _check(insts, seed=9)
    assert h.query("last_fm_lanes") == 83 and h.query("last_fm_waves") > 0


@pytest.mark.parametrize("key32", [1, 0])
def test_chimera_with_triples(gpu, key32):
    """Moves chosen on 32-bit keys (the default where the gains allow) and on
    64-bit keys give the same passes (one replica per wavefront), and so does
    one replica per lane."""
    h = _check([gen.chimera(8, 8, seed=3, instance_id=17, restarts=6)], seed=11, key32=key32, lanes=0)
    assert h.query("last_key32") == key32
    h = _check([gen.chimera(8, 8, seed=3, instance_id=17, restarts=6)], seed=11, key32=key32)
    assert h.query("last_fm_lanes") == 6


def test_large_coefficients_use_wide_keys(gpu):
    """A dense instance whose gains may reach 2^19 in magnitude falls back to
    64-bit keys by itself."""
    # complete graph of 2100 spins with J = 127: sum |c| per spin >= 127 * 2099 > 2^18
    inst = gen.random_small(2100, seed=4, p_edge=1.0, n_triples=0, j_range=(127, 127), h_range=(-7, 7),
                            instance_id=5, restarts=1)
    h = _check([inst], seed=3, max_passes=1, uc=False)
    assert h.query("last_key32") == 0


def test_lattice_and_regular(gpu):
    _check([gen.lattice((16, 16), seed=2, restarts=3), gen.random_regular3(1000, seed=4, instance_id=9)], seed=5)


def test_fixed_pass_budget_and_resume(gpu):
    inst = gen.erdos_renyi_triples(900, seed=7, restarts=3)
    _check([inst], seed=2, max_passes=2, uc=False)
    _check([inst], seed=2, uc=True, runs=[1, 2, 0, 1000])


@pytest.mark.parametrize("waves", [0, 1, 3, 8, 16])
def test_mixed_batch(gpu, waves):
    """Mixed sizes in one call, one replica per wavefront, for several
    workgroup sizes (0: chosen by occupancy): blocks that stage one instance
    and blocks that read several from memory."""
    insts = [gen.chimera(6, 6, seed=s, instance_id=s, restarts=3) for s in range(3)]
    insts += [gen.random_small(40, seed=1, instance_id=77).replace(restarts=2), gen.erdos_renyi_triples(3000, seed=8)]
    _check(insts, seed=9, waves=waves, lanes=0)


def _check_big(insts, seed, slots, max_passes=1000, uc=True, runs=None):
    """Instances of more than 4096 spins on the large-instance pass kernel
    (fm_slots replicas at once), beside smaller ones, against the oracle."""
    import paper_0912_3912_amd as sg
    log(f"fm big case: {[i.name for i in insts][:4]} n={[i.n for i in insts][:4]} seed={seed} slots={slots} "
        f"passes={runs or max_passes} uc={uc}")
    h = sg.load_instance(list(insts))
    h.tune("fm_slots", slots)
    h.bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=FM, max_sweeps=mp, until_converged=uc) for mp in (runs or [max_passes])]
    assert h.query("last_fm_big") == (sum(i.restarts for i in insts if i.n > 4096) if (runs or [max_passes])[-1] else 0)
    states = _oracle(insts, seed, max_passes, uc, runs, threads=8)
    compare(h, insts, states)
    if runs is None:
        assert stats[0]["attempts"] == sum(int((st.sweeps * i.n).sum()) for i, st in zip(insts, states))
        assert stats[0]["flips"] == sum(int(st.flips.sum()) for st in states)
    return h


@pytest.mark.parametrize("slots", [1, 2, 8])
def test_big_er_with_triples(gpu, slots):
    """5000 spins with hyper-couplings, three restarts: one slot runs them in
    turn, two share them, eight leave slots idle."""
    inst = gen.erdos_renyi_triples(5000, seed=3).replace(restarts=3, instance_id=5)
    _check_big([inst], 4, slots).free()


@pytest.mark.parametrize("case", ["lattice80x80", "n4097", "n4160"])
def test_big_lattices_and_boundaries(gpu, case):
    """A 6400-spin 2-D lattice with fields; 4097 spins (a leaf group of one
    spin, two upper entries); 4160 spins (65 leaves)."""
    if case == "n4097":
        inst = gen.random_small(4097, seed=9, p_edge=4.0 / 4097, n_triples=300, j_range=(-9, 9),
                                h_range=(-5, 5), k_range=(-5, 5)).replace(restarts=2, instance_id=11, name="rs4097")
    elif case == "n4160":
        inst = gen.random_small(4160, seed=10, p_edge=5.0 / 4160, n_triples=0, j_range=(-20, 20),
                                h_range=(-3, 3)).replace(restarts=2, instance_id=12, name="rs4160")
    else:
        inst = gen.lattice((80, 80), seed=2, h_range=(-2, 2), restarts=2, instance_id=13)
    _check_big([inst], 6, 4).free()


def test_big_chimera_mixed_with_small(gpu):
    """A 5408-spin Chimera instance (26 x 26 cells, hyper-couplings in some
    cells) beside instances on the lane kernel and the wavefront kernel."""
    big = gen.chimera(26, 26, seed=4, instance_id=20, restarts=2)
    lanes = gen.chimera(4, 4, seed=2, instance_id=21, restarts=64)
    wave = gen.random_small(300, seed=5, p_edge=0.03, n_triples=30, j_range=(-60, 60), h_range=(-9, 9),
                            k_range=(-9, 9)).replace(restarts=3, instance_id=22)
    h = _check_big([big, lanes, wave], 2, 3)
    assert h.query("last_fm_lanes") == 64
    h.free()


def test_big_fixed_passes_and_resume(gpu):
    inst = gen.erdos_renyi_triples(4500, seed=8).replace(restarts=2, instance_id=30)
    _check_big([inst], 9, 2, uc=False, runs=[2, 0, 3]).free()
    _check_big([inst], 9, 2, uc=True, runs=[1, 1000]).free()


def test_big_square1000_one_pass_properties(gpu):
    """The 10^6-spin 2-D lattice of the one-pass workload, four restarts in
    four slots: the oracle's pass costs O(n^2), so the result is checked
    against what holds at any size.  The start is the oracle's; a pass moves
    every spin once and keeps a prefix, so exactly the kept moves' spins
    differ from the start; the tracked energy equals the recomputed one and
    the oracle's energy of the read-back spins, and is not above the start's."""
    import paper_0912_3912_amd as sg
    inst = gen.lattice((1000, 1000), seed=2).replace(restarts=4)
    log(f"fm big case: {inst.name} n={inst.n} seed=7 slots=4 passes=1")
    start, _ = oracle.fm(inst, seed=7, max_passes=0, until_converged=False)
    h = sg.load_instance([inst])
    h.tune("fm_slots", 4)
    h.bind()
    h.init_spins(7)
    assert np.array_equal(h.spins_out_batch(0), start.spins)
    assert np.array_equal(h.energy(), start.energy)
    st = h.run_sweeps(seed=7, rule=FM, max_sweeps=1, until_converged=False)
    assert h.query("last_fm_big") == 4
    assert st["attempts"] == 4 * inst.n
    S = h.spins_out_batch(0)
    E, Er = h.energy(), h.energy(recompute=True)
    sw, fl, cv = h.counters()
    assert np.array_equal(E, Er)
    assert (sw == 1).all() and (cv == 0).all()
    assert st["flips"] == int(fl.sum())
    for r in range(4):
        assert np.isin(S[r], (-1, 1)).all()
        assert int((S[r] != start.spins[r]).sum()) == int(fl[r])
        assert oracle.energy(inst, S[r]) == int(E[r])
        assert E[r] <= start.energy[r]
        assert 0 < fl[r] <= inst.n
    h.free()


def _hub(n, seed, scale=1):
    """A sparse random instance whose spin 7 has 400 couplings and spin
    n - 500 sits in 150 hyper-couplings, so that a move's terms take
    several 64-term chunks."""
    rng = np.random.default_rng(seed)
    base = gen.random_small(n, seed=seed, p_edge=3.0 / n, n_triples=n // 10, j_range=(-9, 9), h_range=(-4, 4),
                            k_range=(-6, 6))
    nb = rng.choice(np.setdiff1d(np.arange(n), [7]), size=400, replace=False)
    hub_j = rng.integers(1, 10, size=400) * rng.choice([-1, 1], size=400)
    ei = np.concatenate([base.ei, np.full(400, 7)]).astype(base.ei.dtype)
    ej = np.concatenate([base.ej, nb]).astype(base.ej.dtype)
    J = np.concatenate([base.J, hub_j]).astype(np.int32) * scale
    c = n - 500
    pairs = rng.choice(np.setdiff1d(np.arange(n), [c]), size=(150, 2), replace=False)
    tri = np.concatenate([base.tri, np.column_stack([np.full(150, c), pairs])]).astype(base.tri.dtype)
    K = np.concatenate([base.K, rng.integers(1, 7, size=150) * rng.choice([-1, 1], size=150)]).astype(np.int32)
    h = base.h.astype(np.int32) * scale
    return gen.Instance(n, ei, ej, J, h, tri, (K * scale).astype(np.int32), restarts=2, instance_id=40 + scale,
                        name=f"hub{n}x{scale}")


@pytest.mark.parametrize("scale", [1, 1000])
def test_big_hub_rows(gpu, scale):
    """A spin with 400 couplings and one in 150 hyper-couplings: a move's
    terms in several chunks; scale 1000 puts the instance in the wide form
    (int32 coefficients)."""
    inst = _hub(6000, seed=5, scale=scale)
    h = _check_big([inst], 3, 2)
    assert h.query("wide_instances") == (1 if scale > 1 else 0)
    h.free()


@pytest.mark.parametrize("scale", [1000, 1 << 24])
def test_big_wide_er(gpu, scale):
    """5000 spins with hyper-couplings in the wide form on the large-instance
    pass kernel: couplings scaled by 1000, or couplings and hyper-couplings by
    2^24, so that a spin's sum of |coefficients| passes 2^25 and the leaf
    maxima take full 64-bit keys."""
    big = gen.erdos_renyi_triples(5000, seed=1)
    J = (big.J.astype(np.int64) * scale).astype(np.int32)
    K = (big.K.astype(np.int64) * (scale if scale > 1000 else 1)).astype(np.int32)
    wide = big.replace(J=J, K=K, restarts=3, instance_id=6)
    if scale > 1000:
        W = np.zeros(big.n, np.int64)
        np.add.at(W, big.ei, np.abs(J.astype(np.int64)))
        np.add.at(W, big.ej, np.abs(J.astype(np.int64)))
        for c in range(3):
            np.add.at(W, big.tri[:, c], np.abs(K.astype(np.int64)))
        assert (1 << 25) <= W.max() < (1 << 31)
    h = _check_big([wide], 2, 2)
    assert h.query("wide_instances") == 1
    h.free()


def test_errors(gpu):
    import paper_0912_3912_amd as sg
    big = gen.erdos_renyi_triples(5000, seed=1)
    h = sg.load_instance([big]).bind()
    h.init_spins(1)
    with pytest.raises(sg.SGError) as e:  # no slots for the large-instance kernel
        h.run_sweeps(seed=1, rule=FM)
    assert e.value.status == sg.SG_EINVAL and "fm_slots" in str(e.value)
    with pytest.raises(sg.SGError):
        h.tune("fm_slots", 8)  # sizes the workspace: before bind only
    h.free()
    h2 = sg.load_instance([gen.chimera(2, 2, seed=1)]).bind()
    h2.init_spins(1)
    with pytest.raises(sg.SGError) as e:
        h2.run_sweeps(seed=1, rule=FM, schedule=sg.SCHED_QUEUE)
    assert e.value.status == sg.SG_EINVAL


def test_chimera_batch_full_size(gpu):
    """4096 Chimera instances x 256 restarts in one launch: sampled replicas
    bit-exact against the oracle; every replica's tracked energy equals a
    recomputation, and every result is a single-flip local minimum."""
    import paper_0912_3912_amd as sg
    insts = gen.cfg3_chimera_batch()
    h = sg.load_instance(insts).bind()
    h.init_spins(7)
    st = h.run_sweeps(seed=7, rule=FM, max_sweeps=1000, until_converged=True)
    log(f"fm chimera4096x256: {st['kernel_ms']:.1f} ms, passes max {st['sweeps_max']}, attempts {st['attempts']}")
    assert h.query("last_fm_lanes") == 4096 * 256
    E = h.energy()
    assert np.array_equal(E, h.energy(recompute=True))
    sw, fl, cv = h.counters()
    assert cv.all()
    rng = np.random.default_rng(1)
    picks = sorted({int(v) for v in rng.integers(0, len(insts), 32)})
    for q in picks:
        inst = insts[q]
        rs = sorted({int(v) for v in rng.integers(0, inst.restarts, 4)})
        sub = inst.replace(restarts=max(rs) + 1)
        ref, _ = oracle.fm(sub, seed=7, threads=8)
        S = h.spins_out_batch(q, 0, max(rs) + 1)
        base = h.info(q)["replica_base"]
        for r in rs:
            assert np.array_equal(S[r], ref.spins[r]), (q, r)
            assert int(E[base + r]) == int(ref.energy[r]) and int(sw[base + r]) == int(ref.sweeps[r])
            assert int(fl[base + r]) == int(ref.flips[r])
    # the same starts under a fixed budget of the largest pass count: passes
    # after convergence change nothing, and the replicas are not frozen, so
    # one GREEDY sweep from the results must flip nothing
    h.init_spins(7)
    st2 = h.run_sweeps(seed=7, rule=FM, max_sweeps=int(st["sweeps_max"]), until_converged=False)
    assert np.array_equal(h.energy(), E)
    g = h.run_sweeps(seed=7, rule=0, max_sweeps=1, until_converged=False)
    assert g["attempts"] == sum(i.n * i.restarts for i in insts) and g["flips"] == 0
    log(f"fixed budget run: {st2['kernel_ms']:.1f} ms")
