"""Branch-and-bound ground states (Sec. III), host CPU code of the library:
against the oracle's exhaustive search, seeded and unseeded, with the node
budget.  Needs the built library, not a GPU."""
import numpy as np
import pytest

import instances as gen
import oracle


@pytest.fixture(scope="module")
def sg():
    import paper_0912_3912_amd as sg
    sg.lib()
    return sg


@pytest.mark.parametrize("seed", range(8))
def test_matches_exhaustive_search(sg, seed):
    inst = gen.random_small(18 + seed % 5, seed=seed, p_edge=0.3, n_triples=5, j_range=(-9, 9), h_range=(-4, 4),
                            k_range=(-5, 5))
    e_bf, _, _ = oracle.brute_force(inst)
    E, s, nodes, proven = sg.exact_ground_state(inst)
    assert proven and E == e_bf and oracle.energy(inst, s) == E
    # seeded with a greedy local minimum: same energy, no more nodes than
    # twice the unseeded search (the seed changes the value order)
    st, _ = oracle.run(inst.replace(restarts=4), seed=seed)
    r = int(np.argmin(st.energy))
    E2, s2, nodes2, proven2 = sg.exact_ground_state(inst, seed_spins=st.spins[r])
    assert proven2 and E2 == e_bf and oracle.energy(inst, s2) == E2


def test_ground_state_seed_is_returned(sg):
    inst = gen.random_small(16, seed=3, p_edge=0.3, n_triples=4)
    e_bf, s_bf, _ = oracle.brute_force(inst)
    E, s, nodes, proven = sg.exact_ground_state(inst, seed_spins=s_bf)
    assert proven and E == e_bf and np.array_equal(s, s_bf)


@pytest.mark.parametrize("dims", [(4, 4), (5, 6), (6, 6)])
def test_lattices_seeded_and_unseeded_agree(sg, dims):
    inst = gen.lattice(dims, seed=7, h_range=(-1, 1))
    E0, s0, n0, p0 = sg.exact_ground_state(inst)
    st, _ = oracle.run(inst.replace(restarts=16), seed=2)
    r = int(np.argmin(st.energy))
    E1, s1, n1, p1 = sg.exact_ground_state(inst, seed_spins=st.spins[r])
    assert p0 and p1 and E0 == E1 <= int(st.energy.min())
    assert E0 >= oracle.lower_bound(inst)
    assert oracle.energy(inst, s0) == E0 and oracle.energy(inst, s1) == E1
    # far fewer nodes than the 2^(n+1) - 2 of the full binary tree
    assert n0 < 2 ** (inst.n + 1) // 100


def test_node_budget(sg):
    inst = gen.lattice((6, 6), seed=7, h_range=(-1, 1))
    E, s, nodes, proven = sg.exact_ground_state(inst, max_nodes=1000)
    assert not proven and nodes == 1000
    assert oracle.energy(inst, s) == E


def test_bad_seed(sg):
    inst = gen.random_small(8, seed=1)
    with pytest.raises(sg.SGError):
        sg.exact_ground_state(inst, seed_spins=np.zeros(8, np.int8))
