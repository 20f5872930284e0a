"""GPU parity of the batched schedules (one launch over many instances and
restarts): the block schedule (restarts of an instance on the lanes of a
workgroup, everything in LDS), the persistent queue schedule (uneven
instances, workgroup or wavefront per item) and mixed handles under
SG_SCHED_AUTO, all bit-exact against the CPU oracle."""
import numpy as np
import pytest

import instances as gen
from parity import compare, expected_stats, log, oracle_run

pytestmark = pytest.mark.gpu

GREEDY, TIE = 0, 1
SCHED_AUTO, SCHED_PHASE, SCHED_BLOCK, SCHED_QUEUE = -1, 0, 4, 5


def _run(insts, seed, rule, sweeps, uc, schedule, tune=None, runs=None, expect_sched=None, dims=None):
    import paper_0912_3912_amd as sg
    log(f"batch case: {len(insts)} instances ({insts[0].name}..) rule={rule} sweeps={runs or sweeps} uc={uc} "
        f"schedule={schedule} tune={tune}")
    h = sg.load_instance(insts, lattice_dims=dims)
    for k, v in (tune or {}).items():
        h.tune(k, v)
    h.bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=rule, max_sweeps=ms, until_converged=uc, schedule=schedule)
             for ms in (runs or [sweeps])]
    if expect_sched is not None:
        assert stats[0]["schedule_used"] == expect_sched, stats[0]
    states = [oracle_run(i, seed, rule, sweeps, uc, runs, threads=8) for i in insts]
    compare(h, insts, states)
    if runs is None:
        att, fl = expected_stats(insts, [None] * len(insts), states)
        assert stats[0]["attempts"] == att and stats[0]["flips"] == fl
        if uc:
            assert stats[0]["n_unconverged"] == sum(int((s.converged == 0).sum()) for s in states)
    return h, stats


def chimera_batch(count, restarts, seed=3):
    return gen.cfg3_chimera_batch(count=count, restarts=restarts, seed=seed)


@pytest.mark.parametrize("rg", [0, 64, 128, 256])
def test_block_chimera_restart_groups(gpu, rg):
    import paper_0912_3912_amd as sg
    insts = chimera_batch(6, 256)
    try:
        _run(insts, 7, GREEDY, 10000, True, SCHED_BLOCK, tune={"block_rg": rg}, expect_sched=SCHED_BLOCK)
    except sg.SGError as e:
        # 256 restarts of a 512-spin instance plus its padded couplings exceed LDS
        assert rg == 256 and e.status == sg.SG_EINVAL, e


@pytest.mark.parametrize("groups", [1, 2, 3, 64])
def test_block_restart_refill(gpu, groups):
    """Slots take the next restart of their workgroup's range as replicas
    stop: ranges of 1, 2, 3 and 64 slot-fulls with ragged restart counts,
    both rules, and resumed calls in which converged replicas are frozen
    (skipped when a slot looks for its next restart)."""
    insts = chimera_batch(3, 200, seed=groups) + [gen.lattice((8, 8), seed=2, restarts=150, instance_id=77)]
    _run(insts, 3, GREEDY, 10000, True, SCHED_BLOCK, tune={"block_groups": groups}, expect_sched=SCHED_BLOCK)
    _run(insts, 3, TIE, 0, True, SCHED_BLOCK, tune={"block_groups": groups}, runs=[4, 0, 30])


def test_deferred_start_energy(gpu):
    """Start energies that sg_init_spins leaves out for instances bound for the
    bit-sliced kernel: equal to the oracle's when read right after the start
    (energy, best), when the bit-sliced kernel writes them, when another rule
    or a zero-sweep call runs first, and under the pass rule (whose tracked
    energies continue from them); the same with the deferral switched off."""
    import paper_0912_3912_amd as sg
    # enough replicas for the lane start kernel (16384), ragged restart counts
    insts = [gen.chimera(4, 4, seed=20 + k, restarts=R, instance_id=90 + k)
             for k, R in enumerate((4096, 4100, 4200, 4000))]
    seed = 5
    start = [oracle_run(i, seed, GREEDY, 0, False) for i in insts]

    def handle(defer):
        h = sg.load_instance(insts).tune("defer_energy", defer).bind()
        h.init_spins(seed)
        assert h.query("energy_pending") == defer
        return h

    for defer in (1, 0):
        log(f"deferred start energy: defer={defer}")
        h = handle(defer)
        Eb, rb = h.best()
        assert h.query("energy_pending") == 0
        for q, st in enumerate(start):
            assert Eb[q] == st.energy.min() and rb[q] == int(np.argmin(st.energy))
        compare(h, insts, start)

        h = handle(defer)
        h.run_sweeps(seed=seed, rule=GREEDY, max_sweeps=10000, until_converged=True, schedule=SCHED_AUTO)
        assert h.query("last_bits") == 1 and h.query("energy_pending") == 0
        compare(h, insts, [oracle_run(i, seed, GREEDY, 10000, True, threads=8) for i in insts])

        h = handle(defer)
        h.run_sweeps(seed=seed, rule=TIE, max_sweeps=6, until_converged=False, schedule=SCHED_AUTO)
        compare(h, insts, [oracle_run(i, seed, TIE, 6, False, threads=8) for i in insts])

        h = handle(defer)
        h.run_sweeps(seed=seed, rule=GREEDY, max_sweeps=0, until_converged=False, schedule=SCHED_AUTO)
        assert h.query("energy_pending") == 0
        compare(h, insts, start)

        h = handle(defer)
        h.run_sweeps(seed=seed, rule=sg.FM, max_sweeps=2, until_converged=False)
        assert np.array_equal(h.energy(), h.energy(recompute=True))

        # the byte block kernel after all (knob changed between start and run)
        h = handle(defer)
        h.tune("block_bits", 0)
        h.run_sweeps(seed=seed, rule=GREEDY, max_sweeps=10000, until_converged=True, schedule=SCHED_AUTO)
        assert h.query("last_bits") == 0
        compare(h, insts, [oracle_run(i, seed, GREEDY, 10000, True, threads=8) for i in insts])

        # binding again drops the replica state, left-out energies included
        h = handle(defer)
        h.bind()
        assert h.query("energy_pending") == 0

        # a second start with another seed replaces the first
        h = handle(defer)
        h.init_spins(seed + 1)
        h.run_sweeps(seed=seed + 1, rule=GREEDY, max_sweeps=10000, until_converged=True, schedule=SCHED_AUTO)
        compare(h, insts, [oracle_run(i, seed + 1, GREEDY, 10000, True, threads=8) for i in insts])


def test_deferred_start_energy_queue(gpu):
    """Start energies left out for a batch bound for the queue schedule: the
    queue kernel stores each converged replica's exact energy from its last
    sweep (which flips nothing), and any other ending computes them from the
    final spins.  Equal to the oracle's in every case: read right after the
    start, converged runs under both rules, runs that stop on the sweep cap
    with and without until_converged; the same with the deferral off."""
    import paper_0912_3912_amd as sg
    insts = [i for i in gen.cfg4_uneven_batch(count=48, seed=13) if i.n <= 20000]
    assert len(insts) >= 32
    seed = 4
    start = [oracle_run(i, seed, GREEDY, 0, False) for i in insts]

    def handle(defer):
        h = sg.load_instance(insts).tune("defer_energy", defer).bind()
        h.init_spins(seed)
        assert h.query("energy_pending") == defer
        return h

    for defer in (1, 0):
        log(f"deferred start energy, queue: defer={defer}")
        compare(handle(defer), insts, start)
        for rule, sweeps, uc in ((GREEDY, 10000, True), (TIE, 30, True), (GREEDY, 2, True), (GREEDY, 3, False)):
            h = handle(defer)
            st = h.run_sweeps(seed=seed, rule=rule, max_sweeps=sweeps, until_converged=uc, schedule=SCHED_AUTO)
            assert st["schedule_used"] == SCHED_QUEUE and h.query("energy_pending") == 0
            compare(h, insts, [oracle_run(i, seed, rule, sweeps, uc, threads=8) for i in insts])


@pytest.mark.parametrize("ng", [2, 4, 8, 16])
def test_block_bits_groups(gpu, ng):
    """The bit-sliced GREEDY block kernel with at most 2, 4, 8 and 16 groups
    of 32 restarts per workgroup (instances of 150 to 530 restarts, so several
    group counts in one call): ragged restart counts (partial groups), refill
    of finished groups, a fixed sweep budget, and resumed calls with frozen
    restarts (the 0-sweep call runs on the byte kernel)."""
    insts = chimera_batch(3, 200, seed=ng) + [gen.lattice((8, 8), seed=2, restarts=150, instance_id=77),
                                              gen.chimera(4, 4, seed=9, restarts=530, instance_id=78)]
    h, _ = _run(insts, 3, GREEDY, 10000, True, SCHED_BLOCK, tune={"bits_groups": ng}, expect_sched=SCHED_BLOCK)
    assert h.query("last_bits") == 1
    _run(insts, 5, GREEDY, 0, True, SCHED_BLOCK, tune={"bits_groups": ng, "block_groups": 1}, runs=[2, 0, 3, 40])
    _run(insts, 6, GREEDY, 7, False, SCHED_BLOCK, tune={"bits_groups": ng})


def test_block_bits_off_and_mixed(gpu):
    """block_bits = 0 keeps GREEDY on the byte kernel; an instance with a
    coupling above 15 in magnitude runs on the byte kernel beside bit-sliced
    ones in the same call."""
    big = gen.random_small(60, seed=5, p_edge=0.2, n_triples=10, j_range=(-40, 40), h_range=(-7, 7),
                           k_range=(-7, 7), instance_id=5, restarts=64)
    insts = chimera_batch(2, 96) + [big]
    h, _ = _run(insts, 4, GREEDY, 10000, True, SCHED_BLOCK, tune={"block_bits": 0})
    assert h.query("last_bits") == 0
    h, _ = _run(insts, 4, GREEDY, 10000, True, SCHED_BLOCK)
    assert h.query("last_bits") == 1


@pytest.mark.parametrize("R", [1, 33, 64, 100, 200])
def test_block_ragged_restart_counts(gpu, R):
    insts = chimera_batch(3, R, seed=R)
    _run(insts, 5, GREEDY, 10000, True, SCHED_BLOCK)


@pytest.mark.parametrize("rule,uc", [(TIE, False), (TIE, True)])
def test_block_tie_rule(gpu, rule, uc):
    insts = chimera_batch(4, 96) + [gen.lattice((8, 8), seed=1, restarts=64, instance_id=999)]
    _run(insts, 9, rule, 25, uc, SCHED_BLOCK)


def test_block_resume(gpu):
    insts = chimera_batch(3, 80)
    _run(insts, 4, TIE, 0, True, SCHED_BLOCK, runs=[2, 3, 0, 40])


def test_block_random_small_with_triples(gpu):
    insts = [gen.random_small(n, seed=n, p_edge=min(1.0, 8.0 / n), n_triples=n // 2, j_range=(-15, 15),
                              h_range=(-7, 7), k_range=(-7, 7), instance_id=n, restarts=70)
             for n in (3, 50, 300, 700)]
    _run(insts, 2, GREEDY, 10000, True, SCHED_BLOCK)


@pytest.mark.parametrize("wave_max", [0, 1000, 4096, 9000])
def test_queue_uneven_er(gpu, wave_max):
    sizes = [100, 150, 300, 800, 1500, 4096, 4097, 6000, 9000, 12000, 30000]
    insts = gen.cfg4_uneven_batch(count=len(sizes), sizes=np.array(sizes))
    _run(insts, 3, GREEDY, 10000, True, SCHED_QUEUE, tune={"queue_wave_max_n": wave_max},
         expect_sched=SCHED_QUEUE)


@pytest.mark.parametrize("grid", [1, 3, 0])
def test_queue_grid_sizes(gpu, grid):
    insts = gen.cfg4_uneven_batch(count=40, seed=11)
    insts = [i for i in insts if i.n <= 20000]
    _run(insts, 6, GREEDY, 10000, True, SCHED_QUEUE, tune={"queue_grid": grid})


@pytest.mark.parametrize("rule,uc", [(TIE, False), (TIE, True), (GREEDY, False)])
def test_queue_rules_and_restarts(gpu, rule, uc):
    insts = [gen.erdos_renyi_triples(n, seed=n, instance_id=n, restarts=3) for n in (120, 2000, 7000)]
    insts += [gen.random_regular3(5000, seed=1, instance_id=5), gen.chimera(8, 8, seed=2, instance_id=6)]
    _run(insts, 8, rule, 20, uc, SCHED_QUEUE)


@pytest.mark.parametrize("rule,uc", [(GREEDY, True), (TIE, False)])
def test_queue_single_colour_items(gpu, rule, uc):
    """Workgroup items with one colour class (fields only, no couplings),
    beside items with several: a sweep is then a single phase, so its flip
    flag is written with no phase barrier after the previous sweep's."""
    rng = np.random.default_rng(5)
    lone = []
    for k, n in enumerate((2000, 5000)):
        h = rng.integers(-3, 4, size=n).astype(np.int32)
        e = np.zeros(0, np.int32)
        lone.append(gen.Instance(n, e, e, e, h, restarts=2, instance_id=70 + k, name=f"fields{n}"))
    insts = lone + [gen.erdos_renyi_triples(3000, seed=4, instance_id=80, restarts=2)]
    _run(insts, 5, rule, 12, uc, SCHED_QUEUE, tune={"queue_wave_max_n": 256})


def test_queue_resume(gpu):
    insts = [gen.erdos_renyi_triples(n, seed=n, instance_id=n) for n in (300, 5000, 10000)]
    _run(insts, 1, GREEDY, 0, True, SCHED_QUEUE, runs=[1, 2, 0, 100])


def test_auto_mixed_handle(gpu):
    """AUTO assigns lattice, block, queue and per-phase schedules per
    instance inside one call; the results match the oracle replica by replica."""
    insts = [gen.lattice((8, 8), seed=1, restarts=4, instance_id=1),
             gen.chimera(4, 4, seed=2, restarts=64, instance_id=2)]
    insts += [gen.erdos_renyi_triples(n, seed=n, instance_id=100 + k) for k, n in enumerate(range(200, 6200, 150))]
    insts += [gen.erdos_renyi_triples(200000, seed=9, instance_id=7)]
    dims = [(8, 8), None] + [None] * (len(insts) - 2)
    h, st = _run(insts, 12, GREEDY, 10000, True, SCHED_AUTO, dims=dims)
    assert st[0]["schedule_used"] == SCHED_AUTO  # mixed


def test_chimera_4096x256_reduced(gpu):
    """The batched Chimera workload at 64 of its 4096 instances (all 256
    restarts each), AUTO schedule."""
    insts = chimera_batch(64, 256)
    _run(insts, 7, GREEDY, 10000, True, SCHED_AUTO, expect_sched=SCHED_BLOCK)


def test_uneven_er_reduced(gpu):
    """The uneven Erdos-Renyi workload at 60 of its 2000 instances."""
    insts = gen.cfg4_uneven_batch(count=60, seed=4)
    _run(insts, 7, GREEDY, 10000, True, SCHED_AUTO, expect_sched=SCHED_QUEUE)


def _oracle_many(insts, seed, rule, sweeps, uc, workers=16):
    """Oracle over many instances, one instance per pool task (the C oracle
    releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda i: oracle_run(i, seed, rule, sweeps, uc, threads=1 if i.restarts == 1 else 4),
                           insts))


def test_chimera_4096x256_full(gpu):
    """The batched Chimera workload at full size: 4096 instances x 256
    restarts (1,048,576 replicas), in the configuration the benchmark times,
    every replica compared with the oracle."""
    import paper_0912_3912_amd as sg
    insts = chimera_batch(4096, 256)
    log("chimera 4096x256 full: loading")
    h = sg.load_instance(insts).bind()
    h.init_spins(7)
    st = h.run_sweeps(seed=7, rule=GREEDY, max_sweeps=10000, until_converged=True)
    assert st["schedule_used"] == SCHED_BLOCK
    log(f"gpu done: {st}")
    states = _oracle_many(insts, 7, GREEDY, 10000, True, workers=4)
    log("oracle done")
    compare(h, insts, states)
    E, r = h.best()
    for q in range(len(insts)):
        assert E[q] == states[q].energy.min() and r[q] == int(np.argmin(states[q].energy))


def test_uneven_er_2000_full(gpu):
    """The uneven Erdos-Renyi workload at full size (2000 instances, sum n ~
    2.9e7), AUTO schedule as benchmarked, every instance compared."""
    import paper_0912_3912_amd as sg
    insts = gen.cfg4_uneven_batch()
    log("er 2000 full: loading")
    h = sg.load_instance(insts).bind()
    h.init_spins(7)
    st = h.run_sweeps(seed=7, rule=GREEDY, max_sweeps=10000, until_converged=True)
    assert st["schedule_used"] == SCHED_QUEUE
    log(f"gpu done: {st}")
    states = _oracle_many(insts, 7, GREEDY, 10000, True)
    log("oracle done")
    compare(h, insts, states)
