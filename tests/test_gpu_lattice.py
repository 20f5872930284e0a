"""GPU parity of the lattice schedules (implicit neighbours, LDS-resident):
the whole-lattice workgroup mode and the co-resident tile mode with halo
exchanges every k colour phases, in both its byte-per-spin kernel and its
bit-plane kernel (lattices with +-1 bonds and |h| <= 2), against the CPU
oracle, bit for bit."""
import numpy as np
import pytest

import instances as gen
from parity import compare, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

GREEDY, TIE = 0, 1
SCHED_LATTICE = 3


def _run(insts, dims, seed, rule, sweeps, uc, tune=None, runs=None):
    import paper_0912_3912_amd as sg
    log(f"lattice case: {[i.name for i in insts]} rule={rule} sweeps={runs or sweeps} uc={uc} tune={tune}")
    h = sg.load_instance(insts, lattice_dims=dims)
    for k, v in (tune or {}).items():
        h.tune(k, v)
    h.bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=rule, max_sweeps=ms, until_converged=uc, schedule=SCHED_LATTICE)
             for ms in (runs or [sweeps])]
    assert all(s["schedule_used"] == SCHED_LATTICE for s in stats)
    states = [oracle_run(i, seed, rule, sweeps, uc, runs) for i in insts]
    compare(h, insts, states)
    return h, stats


def test_square16_workgroup_mode(gpu):
    inst = gen.cfg1_square16()
    _run([inst], [(16, 16)], 7, GREEDY, 10000, True)


@pytest.mark.parametrize("rule,uc", [(GREEDY, True), (TIE, False), (TIE, True)])
def test_cubic_workgroup_mode(gpu, rule, uc):
    inst = gen.lattice((12, 10, 8), seed=5, h_range=(-2, 2), restarts=5)
    _run([inst], [(12, 10, 8)], 3, rule, 40, uc)


def _tile_tune(kernel, k=None, **extra):
    t = {"lattice_wg_max_n": 0}
    if kernel == "byte":
        t["lattice_msc"] = 0
        if k is not None:
            t["lattice_k"] = k
    elif k is not None:
        t["msc_k"] = k
    t.update(extra)
    return t


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("rule", [GREEDY, TIE])
@pytest.mark.parametrize("kernel", ["byte", "msc"])
def test_cubic_tile_mode_halo_widths(gpu, k, rule, kernel):
    inst = gen.lattice((20, 16, 24), seed=k, h_range=(-2, 2), restarts=2)
    h, _ = _run([inst], [(20, 16, 24)], 11, rule, 17, False, tune=_tile_tune(kernel, k))
    log(f"tiles={h.query('last_tiles')} k={h.query('last_tile_k')} msc={h.query('last_msc')}")
    assert h.query("last_tile_k") == k
    assert h.query("last_msc") == (kernel == "msc")


@pytest.mark.parametrize("k", [6, 8, 11, 16])
@pytest.mark.parametrize("rule", [GREEDY, TIE])
def test_cubic_msc_deep_halos(gpu, k, rule):
    """Deep halos of the bit-plane kernel, a box z-row of up to 64 sites."""
    inst = gen.lattice((34, 32, 64), seed=k + 40, h_range=(-2, 2), restarts=1)
    h, _ = _run([inst], [(34, 32, 64)], 17, rule, 2 * k + 3, False, tune=_tile_tune("msc", k))
    log(f"tiles={h.query('last_tiles')} k={h.query('last_tile_k')}")
    assert h.query("last_tile_k") == k and h.query("last_msc") == 1


@pytest.mark.parametrize("max_tiles", [1, 2, 3, 8, 27])
@pytest.mark.parametrize("kernel", ["byte", "msc"])
def test_cubic_tile_mode_tilings(gpu, max_tiles, kernel):
    """Few tiles: periodic self-neighbours (one or two tiles along an axis)
    and uneven tile extents."""
    inst = gen.lattice((14, 18, 10), seed=2, h_range=(-2, 2))
    h, _ = _run([inst], [(14, 18, 10)], 5, TIE, 9, False, tune=_tile_tune(kernel, 3, lattice_max_tiles=max_tiles))
    log(f"tiles={h.query('last_tiles')}")
    assert h.query("last_msc") == (kernel == "msc")


@pytest.mark.parametrize("k", [1, 4])
def test_square_tile_mode(gpu, k):
    inst = gen.lattice((64, 48), seed=3, h_range=(-1, 1), j_values=(-2, -1, 1, 2), restarts=2)
    h, _ = _run([inst], [(64, 48)], 9, TIE, 13, False, tune={"lattice_wg_max_n": 0, "lattice_k": k})
    assert h.query("last_msc") == 0  # |J| = 2 bonds: byte kernel


@pytest.mark.parametrize("k", [1, 3, 7, 12])
@pytest.mark.parametrize("rule", [GREEDY, TIE])
def test_square_msc(gpu, k, rule):
    inst = gen.lattice((96, 60), seed=k, h_range=(-2, 2), restarts=3)
    h, _ = _run([inst], [(96, 60)], 9 + k, rule, 2 * k + 5, False, tune=_tile_tune("msc", k))
    log(f"tiles={h.query('last_tiles')} k={h.query('last_tile_k')}")
    assert h.query("last_msc") == 1 and h.query("last_tile_k") == k


@pytest.mark.parametrize("kernel", ["byte", "msc"])
def test_tile_mode_resume(gpu, kernel):
    inst = gen.lattice((16, 16, 16), seed=8, h_range=(-2, 2))
    _run([inst], [(16, 16, 16)], 4, TIE, 0, False, tune=_tile_tune(kernel, 4), runs=[3, 5, 1, 0, 6])


@pytest.mark.parametrize("kernel", ["byte", "msc"])
def test_tile_mode_skips_frozen_replicas(gpu, kernel):
    """Replicas that converged in an earlier call stay frozen: a later
    fixed-sweep GREEDY_TIE call on the tile schedule (which would flip their
    ties) leaves them as they are, as the oracle does."""
    import paper_0912_3912_amd as sg
    inst = gen.lattice((16, 12, 24), seed=8, h_range=(-2, 2), restarts=6, instance_id=3)
    seed = 4
    log(f"lattice case: frozen replicas, {kernel} tile kernel")
    h = sg.load_instance([inst], lattice_dims=[(16, 12, 24)])
    for k, v in _tile_tune(kernel, 2).items():
        h.tune(k, v)
    h.bind()
    h.init_spins(seed)
    # converge a few replicas first (per-phase schedule, a short cap), then
    # sweep all of them with ties on the tile schedule
    st = h.run_sweeps(seed=seed, rule=GREEDY, max_sweeps=6, until_converged=True, schedule=0)
    assert 0 < st["n_unconverged"] < inst.restarts
    st = h.run_sweeps(seed=seed, rule=TIE, max_sweeps=9, until_converged=False, schedule=SCHED_LATTICE)
    assert st["schedule_used"] == SCHED_LATTICE and h.query("last_msc") == (1 if kernel == "msc" else 0)
    s1 = oracle_run(inst, seed, GREEDY, 6, True)
    s2 = oracle_run(inst, seed, TIE, 9, False, state=s1)
    compare(h, [inst], [s2])


def test_lattice_deferred_start_energy(gpu):
    """A start bound for the bit-plane tile kernel leaves its energy out (that
    kernel sums the final energies itself).  Energies equal the oracle's when
    read right after the start, after a bit-plane run, and after a run that
    ends up on another kernel (byte tile kernel, or until_converged on the
    per-phase schedule), each read back after its run."""
    import paper_0912_3912_amd as sg
    dims = (16, 12, 24)
    inst = gen.lattice(dims, seed=9, h_range=(-2, 2), restarts=3, instance_id=5)
    seed = 6

    def handle(**after):
        h = sg.load_instance([inst], lattice_dims=[dims])
        h.tune("lattice_wg_max_n", 0)
        h.bind()
        h.init_spins(seed)
        assert h.query("energy_pending") == 1
        for k, v in after.items():  # knobs changed between the start and the run
            h.tune(k, v)
        return h

    log("lattice case: deferred start energy")
    h = handle()
    compare(h, [inst], [oracle_run(inst, seed, GREEDY, 0, False)])
    for rule, ms, uc, tune, sched, msc in ((TIE, 11, False, {}, SCHED_LATTICE, 1),
                                           (GREEDY, 7, False, {}, SCHED_LATTICE, 1),
                                           (TIE, 11, False, {"lattice_msc": 0}, SCHED_LATTICE, 0),
                                           (GREEDY, 50, True, {}, -1, None)):
        h = handle(**tune)
        st = h.run_sweeps(seed=seed, rule=rule, max_sweeps=ms, until_converged=uc, schedule=sched)
        if msc is not None:
            assert st["schedule_used"] == SCHED_LATTICE and h.query("last_msc") == msc
        assert h.query("energy_pending") == 0
        compare(h, [inst], [oracle_run(inst, seed, rule, ms, uc)])


def test_msc_restarts_and_fields(gpu):
    """h = 0 everywhere (every tie rule branch at g = 0) and several restarts."""
    inst = gen.lattice((18, 22, 26), seed=3, h_range=(0, 0), restarts=4)
    h, _ = _run([inst], [(18, 22, 26)], 31, TIE, 11, False, tune=_tile_tune("msc"))
    assert h.query("last_msc") == 1


def test_msc_not_used_when_ineligible(gpu):
    inst = gen.lattice((16, 16, 16), seed=8, h_range=(-3, 3))
    h, _ = _run([inst], [(16, 16, 16)], 4, TIE, 5, False, tune=_tile_tune("msc"))
    assert h.query("last_msc") == 0


def test_tile_mode_stopping_rule_availability(gpu):
    """The stopping rule runs on the tile kernels only as the bit-plane kernel
    under GREEDY (where a sweep without a flip is a fixed point): GREEDY_TIE
    and the byte kernel refuse it on the tile schedule, and SG_SCHED_AUTO
    then falls back to a schedule that supports it."""
    import paper_0912_3912_amd as sg
    inst = gen.lattice((16, 16, 16), seed=8, h_range=(-2, 2))
    h = sg.load_instance([inst], lattice_dims=[(16, 16, 16)]).tune("lattice_wg_max_n", 0).bind()
    h.init_spins(1)
    with pytest.raises(sg.SGError) as e:
        h.run_sweeps(seed=1, rule=TIE, until_converged=True, schedule=SCHED_LATTICE)
    assert e.value.status == sg.SG_EINVAL
    h.tune("lattice_msc", 0)
    with pytest.raises(sg.SGError) as e:
        h.run_sweeps(seed=1, rule=GREEDY, until_converged=True, schedule=SCHED_LATTICE)
    assert e.value.status == sg.SG_EINVAL
    st = h.run_sweeps(seed=1, rule=GREEDY, until_converged=True)
    assert st["schedule_used"] != SCHED_LATTICE
    h.tune("lattice_msc", 1)
    h.init_spins(1)
    st = h.run_sweeps(seed=1, rule=GREEDY, until_converged=True)
    assert st["schedule_used"] == SCHED_LATTICE and h.query("last_msc") == 1


@pytest.mark.parametrize("dims,R,chunk", [((100, 100, 100), 1, 0), ((64, 64, 64), 3, 0), ((512, 512), 2, 0),
                                          ((40, 48, 56), 2, 3), ((32, 32, 32), 4, 1)])
def test_msc_greedy_until_converged(gpu, dims, R, chunk):
    """GREEDY until converged on the bit-plane tile kernel: tiles keep sweeping
    until every tile has reported a sweep without a flip, stop together, and
    the replica's sweep count is the first such sweep plus one.  Small chunks
    split a run into several launches; capped and resumed calls too."""
    inst = gen.lattice(dims, seed=len(dims) * 7 + R, h_range=(-2, 2) if len(dims) == 3 else None, restarts=R,
                       instance_id=40 + R)
    tune = {"lattice_wg_max_n": 0}
    if chunk:
        tune["lattice_conv_chunk"] = chunk
    h, st = _run([inst], [dims], 5, GREEDY, 10000, True, tune=tune)
    assert h.query("last_msc") == 1 and st[0]["n_unconverged"] == 0
    log(f"  tiles={h.query('last_tiles')} k={h.query('last_tile_k')} sweeps_max={st[0]['sweeps_max']} "
        f"launches={h.query('hot_launches')} kernel_ms={st[0]['kernel_ms']:.3f}")
    h.free()
    h, st = _run([inst], [dims], 6, GREEDY, 0, True, tune=tune, runs=[2, 1, 0, 10000])
    assert st[0]["status"] == 1 and st[-1]["status"] == 0  # the capped call reports SG_ENOTCONV
    h.free()


def test_mixed_lattice_batch(gpu):
    insts = [gen.lattice((8, 8), seed=1, restarts=3, instance_id=1),
             gen.lattice((6, 6, 6), seed=2, h_range=(-2, 2), restarts=2, instance_id=2)]
    _run(insts, [(8, 8), (6, 6, 6)], 21, GREEDY, 100, True)


def test_cubic100_full_tile_mode(gpu):
    """The 10^6-spin workload in the launch configuration the benchmark
    times (tile mode, default tiling and kernel), 1000 GREEDY_TIE sweeps."""
    inst = gen.cfg2_cubic100()
    h, st = _run([inst], [(100, 100, 100)], 7, TIE, 1000, False)
    log(f"tiles={h.query('last_tiles')} k={h.query('last_tile_k')} msc={h.query('last_msc')} "
        f"kernel_ms={st[0]['kernel_ms']:.2f}")
    assert h.query("last_msc") == 1


def test_cubic100_byte_kernel(gpu):
    """The same workload through the byte-per-spin tile kernel, 200 sweeps."""
    inst = gen.cfg2_cubic100()
    h, st = _run([inst], [(100, 100, 100)], 7, TIE, 200, False, tune={"lattice_msc": 0})
    assert h.query("last_msc") == 0


def _solve_check(insts, dims, seed, rule, sweeps, uc, tune=None, schedule=-1, then=None, one_launch=True):
    """sg_solve (start, run and best in one call) against the oracle, and
    against the three calls it stands for on a second handle: spins, energies,
    counters, call totals and the best restart agree bit for bit; ``then``
    continues both handles with one more run (resume after a solve)."""
    import paper_0912_3912_amd as sg
    log(f"solve case: {[i.name for i in insts]} rule={rule} sweeps={sweeps} uc={uc} tune={tune} "
        f"schedule={schedule} then={then}")
    hs = []
    for _ in range(2):
        h = sg.load_instance(insts, lattice_dims=dims)
        for k, v in (tune or {}).items():
            h.tune(k, v)
        hs.append(h.bind())
    st, Eb, rb = hs[0].solve(seed, rule=rule, max_sweeps=sweeps, until_converged=uc, schedule=schedule)
    if one_launch:
        assert hs[0].query("hot_launches") == len(insts)
    hs[1].init_spins(seed)
    st2 = hs[1].run_sweeps(seed=seed, rule=rule, max_sweeps=sweeps, until_converged=uc, schedule=schedule)
    Eb2, rb2 = hs[1].best()
    for k in ("attempts", "flips", "sweeps_max", "n_unconverged", "schedule_used", "status"):
        assert st[k] == st2[k], k
    assert np.array_equal(Eb, Eb2) and np.array_equal(rb, rb2)
    runs = [sweeps] + ([then] if then is not None else [])
    if then is not None:
        for h in hs:
            h.run_sweeps(seed=seed, rule=rule, max_sweeps=then, until_converged=uc, schedule=schedule)
    states = [oracle_run(i, seed, rule, sweeps, uc, runs) for i in insts]
    for h in hs:
        compare(h, insts, states)
    if then is None:
        for q, s in enumerate(states):
            assert Eb[q] == s.energy.min() and rb[q] == int(np.argmin(s.energy))
    # a second solve on each handle (after a solve, and after a run) starts
    # afresh and gives the first one's results again
    for h in hs:
        st3, Eb3, rb3 = h.solve(seed, rule=rule, max_sweeps=sweeps, until_converged=uc, schedule=schedule)
        for k in ("attempts", "flips", "sweeps_max", "n_unconverged", "status"):
            assert st3[k] == st[k], k
        assert np.array_equal(Eb3, Eb) and np.array_equal(rb3, rb)
        h.free()
    return st


def test_solve_square16(gpu):
    st = _solve_check([gen.cfg1_square16()], [(16, 16)], 7, GREEDY, 10000, True)
    assert st["n_unconverged"] == 0 and st["schedule_used"] == SCHED_LATTICE


@pytest.mark.parametrize("rule,sweeps,uc", [(GREEDY, 10000, True), (TIE, 40, False), (TIE, 40, True),
                                            (GREEDY, 0, True), (TIE, 0, False), (GREEDY, 3, True)])
def test_solve_cubic(gpu, rule, sweeps, uc):
    """3-D lattice with fields; no sweeps (start and energy only); a cap the
    stopping rule does not reach (SG_ENOTCONV with every output written)."""
    inst = gen.lattice((12, 10, 8), seed=5, h_range=(-2, 2), restarts=5)
    st = _solve_check([inst], [(12, 10, 8)], 3, rule, sweeps, uc)
    if rule == GREEDY and sweeps == 3:
        assert st["status"] == 1 and st["n_unconverged"] > 0


def test_solve_two_lattices_and_resume(gpu):
    a = gen.cfg1_square16().replace(instance_id=4)
    b = gen.lattice((8, 8, 6), seed=2, h_range=(-3, 3), restarts=9).replace(instance_id=5)
    _solve_check([a, b], [(16, 16), (8, 8, 6)], 11, TIE, 25, False, then=17)
    _solve_check([a, b], [(16, 16), (8, 8, 6)], 11, GREEDY, 4, False, then=200)


@pytest.mark.parametrize("case", ["graph", "phase", "tiles"])
def test_solve_other_schedules(gpu, case):
    """Handles that the one-launch form does not take make the three calls."""
    if case == "graph":
        inst = gen.random_small(300, seed=3, p_edge=0.02, n_triples=40).replace(restarts=6, instance_id=8)
        _solve_check([inst], None, 5, GREEDY, 10000, True, one_launch=False)
    elif case == "phase":
        inst = gen.lattice((8, 8, 8), seed=4, h_range=(-2, 2), restarts=3)
        _solve_check([inst], [(8, 8, 8)], 5, TIE, 20, False, schedule=0, one_launch=False)
    else:
        inst = gen.lattice((16, 16, 16), seed=6, h_range=(-2, 2), restarts=2)
        _solve_check([inst], [(16, 16, 16)], 5, TIE, 30, False, tune={"lattice_wg_max_n": 0}, one_launch=False)
