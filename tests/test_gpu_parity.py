"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle,
bit-exact on spins, tracked and recomputed int64 energies, sweep and flip
counts and converged flags of every replica."""
import numpy as np
import pytest

import instances as gen
import oracle
from parity import compare, expected_stats, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu

GREEDY, TIE = 0, 1


def _check(insts, seed, rule, max_sweeps, until_converged, schedule=-1, runs=None, lattice_dims=None):
    log(f"case: {[i.name for i in insts][:4]} seed={seed} rule={rule} sweeps={runs or max_sweeps} "
        f"until_converged={until_converged} schedule={schedule}")
    h, stats = gpu_run(insts, seed, rule, max_sweeps, until_converged, schedule, runs, lattice_dims)
    states = [oracle_run(i, seed, rule, max_sweeps, until_converged, runs) for i in insts]
    compare(h, insts, states)
    if runs is None:
        att, fl = expected_stats(insts, [None] * len(insts), states)
        assert stats[0]["attempts"] == att
        assert stats[0]["flips"] == fl
    h.free()
    return states


def test_square16_64_starts(gpu):
    """16x16 periodic +-J lattice, 64 starts, GREEDY until converged."""
    _check([gen.cfg1_square16()], seed=7, rule=GREEDY, max_sweeps=10000, until_converged=True)


def test_square4_against_exhaustive(gpu):
    inst = gen.cfg1_square4().replace(restarts=64)
    e_gs, _, _ = oracle.brute_force(inst)
    _check([inst], seed=7, rule=GREEDY, max_sweeps=10000, until_converged=True)
    import paper_0912_3912_amd as sg
    h = sg.load_instance([inst]).bind()
    h.init_spins(7)
    h.run_sweeps(seed=7)
    Eb, rb = h.best()
    assert Eb[0] >= e_gs
    E = h.energy()
    assert Eb[0] == E.min() and rb[0] == int(np.argmin(E))


@pytest.mark.parametrize("rule,uc,sweeps", [(TIE, False, 40), (GREEDY, True, 1000), (TIE, True, 60)])
def test_cubic20(gpu, rule, uc, sweeps):
    inst = gen.cfg2_cubic100(L=20).replace(restarts=3)
    _check([inst], seed=7, rule=rule, max_sweeps=sweeps, until_converged=uc)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 129, 1000])
@pytest.mark.parametrize("rule", [GREEDY, TIE])
def test_ragged_random_with_triples(gpu, n, rule):
    inst = gen.random_small(n, seed=n, p_edge=min(1.0, 8.0 / max(n, 1)), n_triples=n // 2,
                            j_range=(-15, 15), h_range=(-7, 7), k_range=(-7, 7)).replace(restarts=5)
    _check([inst], seed=n + 1, rule=rule, max_sweeps=25, until_converged=(rule == GREEDY))


@pytest.mark.parametrize("rule", [GREEDY, TIE])
def test_chimera_with_triples(gpu, rule):
    inst = gen.chimera(8, 8, seed=3, instance_id=17, restarts=6)
    _check([inst], seed=11, rule=rule, max_sweeps=30, until_converged=(rule == GREEDY))


def test_batch_of_mixed_instances(gpu):
    insts = [gen.chimera(8, 8, seed=s, instance_id=s, restarts=3) for s in range(3)]
    insts += [gen.erdos_renyi_triples(n, seed=n, instance_id=100 + n) for n in (100, 517, 3000)]
    insts += [gen.random_regular3(1000, seed=4, instance_id=7)]
    _check(insts, seed=5, rule=GREEDY, max_sweeps=10000, until_converged=True)


@pytest.mark.parametrize("rule,uc", [(GREEDY, True), (TIE, False), (TIE, True)])
def test_resume_exact(gpu, rule, uc):
    inst = gen.lattice((10, 10, 10), seed=3, h_range=(-2, 2), restarts=3)
    _check([inst], seed=8, rule=rule, max_sweeps=0, until_converged=uc, runs=[5, 7, 0, 3])


def test_factor21_all_starts_via_set_spins(gpu):
    import itertools
    import paper_0912_3912_amd as sg
    from test_oracle_pins import factor21_instance
    inst, N, const, _ = factor21_instance()
    inst = inst.replace(restarts=8)
    h = sg.load_instance([inst]).bind()
    for r, S in enumerate(itertools.product([1, -1], repeat=3)):
        h.set_spins(0, r, np.array(S, np.int8))
    h.run_sweeps(seed=1)
    E = h.energy()
    assert np.all(E == -const)
    for r in range(8):
        assert list(h.spins_out(0, r)) == [-1, -1, -1]


def test_lattice_hint_and_explicit_colouring(gpu):
    inst = gen.lattice((8, 6, 4), seed=9, h_range=(-2, 2), restarts=2)
    _check([inst], seed=3, rule=TIE, max_sweeps=12, until_converged=False, lattice_dims=[(8, 6, 4)])


def test_errors(gpu):
    import paper_0912_3912_amd as sg
    h = sg.load_instance([gen.cfg1_square16()])
    with pytest.raises(sg.SGError) as e:
        h.run_sweeps(seed=1)
    assert e.value.status == sg.SG_ESTATE
    h.bind()
    with pytest.raises(sg.SGError) as e:
        h.run_sweeps(seed=1)
    assert e.value.status == sg.SG_ESTATE
    h.init_spins(1)
    with pytest.raises(sg.SGError) as e:
        h.set_spins(0, 0, np.zeros(256, np.int8))
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SGError) as e:
        h.run_sweeps(seed=1, rule=5)
    assert e.value.status == sg.SG_EINVAL
    st = h.run_sweeps(seed=1, max_sweeps=1)
    assert st["status"] == sg.SG_ENOTCONV and st["n_unconverged"] == 64


def test_cubic100_full_1000_sweeps(gpu):
    """The 10^6-spin workload at full size: 1000 GREEDY_TIE sweeps from one
    random start, compared with the oracle (spins, energies, flips)."""
    inst = gen.cfg2_cubic100()
    _check([inst], seed=7, rule=TIE, max_sweeps=1000, until_converged=False,
           lattice_dims=[(100, 100, 100)])


# ---------------------------------------------------------------------------
# SG_SCHED_GRAPH: phase launches of a segment of sweeps recorded in a HIP graph
# and replayed; the sweep index of each replay comes from a device counter.

def _check_graph(insts, seed, rule, uc, runs, graph_sweeps):
    import paper_0912_3912_amd as sg
    log(f"case: graph {[i.name for i in insts][:3]} seed={seed} rule={rule} uc={uc} runs={runs} "
        f"graph_sweeps={graph_sweeps}")
    h = sg.load_instance(list(insts))
    h.tune("graph_sweeps", graph_sweeps)
    h.bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=rule, max_sweeps=ms, until_converged=uc, schedule=sg.SCHED_GRAPH)
             for ms in runs]
    assert all(s["schedule_used"] == sg.SCHED_GRAPH for s in stats)
    states = [oracle_run(i, seed, rule, 0, uc, runs) for i in insts]
    compare(h, insts, states)
    if len(runs) == 1:
        att, fl = expected_stats(insts, [None] * len(insts), states)
        assert stats[0]["attempts"] == att and stats[0]["flips"] == fl
    h.free()


@pytest.mark.parametrize("graph_sweeps,runs", [(1, [9]), (4, [10]), (32, [70]), (32, [5]), (8, [3, 8, 0, 17])])
@pytest.mark.parametrize("rule,uc", [(GREEDY, True), (TIE, False), (TIE, True)])
def test_graph_schedule(gpu, graph_sweeps, runs, rule, uc):
    inst = gen.erdos_renyi_triples(700, seed=9, instance_id=3, restarts=4)
    _check_graph([inst], seed=13, rule=rule, uc=uc, runs=runs, graph_sweeps=graph_sweeps)


def test_graph_schedule_batch_until_converged(gpu):
    insts = [gen.chimera(6, 6, seed=s, instance_id=s, restarts=3) for s in range(2)]
    insts += [gen.lattice((12, 12), seed=2, instance_id=40, restarts=2), gen.random_small(65, seed=1)]
    _check_graph(insts, seed=21, rule=GREEDY, uc=True, runs=[10000], graph_sweeps=16)


# ---------------------------------------------------------------------------
# SG_SCHED_FIELDS: phases over maintained local fields (flips scatter the
# change of their partners' fields).

def _check_fields(insts, seed, rule, uc, runs):
    import paper_0912_3912_amd as sg
    log(f"case: fields {[i.name for i in insts][:3]} seed={seed} rule={rule} uc={uc} runs={runs}")
    h = sg.load_instance(list(insts)).tune("fields", 1)
    h.bind()
    h.init_spins(seed)
    stats = [h.run_sweeps(seed=seed, rule=rule, max_sweeps=ms, until_converged=uc, schedule=sg.SCHED_FIELDS)
             for ms in runs]
    assert all(s["schedule_used"] == sg.SCHED_FIELDS for s in stats)
    states = [oracle_run(i, seed, rule, 0, uc, runs) for i in insts]
    compare(h, insts, states)
    h.free()


@pytest.mark.parametrize("rule,uc", [(GREEDY, True), (TIE, False), (TIE, True)])
@pytest.mark.parametrize("kind", ["er_triples", "chimera", "ragged"])
def test_fields_schedule(gpu, rule, uc, kind):
    inst = {"er_triples": gen.erdos_renyi_triples(3000, seed=5, instance_id=4, restarts=3),
            "chimera": gen.chimera(8, 8, seed=2, instance_id=8, restarts=4),
            "ragged": gen.random_small(129, seed=3, p_edge=0.06, n_triples=60, j_range=(-15, 15), h_range=(-7, 7),
                                       k_range=(-7, 7)).replace(restarts=5)}[kind]
    runs = [10000] if uc else [7]
    _check_fields([inst], seed=17, rule=rule, uc=uc, runs=runs)


def test_fields_schedule_resume_and_batch(gpu):
    insts = [gen.erdos_renyi_triples(2000, seed=s, instance_id=s, restarts=2) for s in (1, 2)]
    insts += [gen.lattice((10, 10, 10), seed=3, h_range=(-2, 2), restarts=2, instance_id=40)]
    _check_fields(insts, seed=3, rule=TIE, uc=True, runs=[2, 5, 0, 10000])


def test_fields_knob_before_bind_only(gpu):
    import paper_0912_3912_amd as sg
    h = sg.load_instance([gen.chimera(2, 2, seed=1)]).bind()
    h.init_spins(1)
    with pytest.raises(sg.SGError) as e:
        h.run_sweeps(seed=1, schedule=sg.SCHED_FIELDS)  # no fields in this workspace
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SGError) as e:
        h.tune("fields", 1)  # would change the bound workspace
    assert e.value.status == sg.SG_EINVAL


def test_gpu_restarts_seed_branch_and_bound(gpu):
    """The GPU descent's best restart seeds the exact search (Sec. III: a
    greedy approximation as the initial bound)."""
    import paper_0912_3912_amd as sg
    inst = gen.lattice((8, 8), seed=8, h_range=(-1, 1)).replace(restarts=256)
    h = sg.load_instance([inst]).bind()
    h.init_spins(5)
    h.run_sweeps(seed=5, rule=GREEDY)
    Eb, rb = h.best()
    seed_state = h.spins_out(0, int(rb[0]))
    E, s, nodes, proven = sg.exact_ground_state(inst, seed_spins=seed_state)
    log(f"8x8: GPU best of 256 restarts {int(Eb[0])}, exact {E} after {nodes} nodes")
    assert proven and E <= int(Eb[0]) and oracle.energy(inst, s) == E
