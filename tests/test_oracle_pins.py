"""Pins for the CPU oracle: each test checks the oracle against something
other than itself -- the paper's worked example, closed forms, exhaustive
search, symmetries of the energy and invariants of the descent.  A plausible
slip anywhere in the oracle (a dropped term, a wrong sign or index, a
transposed triple member, a misapplied flip, a wrong RNG counter) fails at
least one of them.
"""
import itertools
import os

import numpy as np
import pytest

import instances as gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers


def load_poly(path):
    """Polynomial fixture -> (N, const, {tuple(indices): coef})."""
    N, const, terms = None, 0, {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("N "):
            N = int(line.split()[1])
            continue
        parts = [int(x) for x in line.split()]
        if len(parts) == 1:
            const = parts[0]
        else:
            terms[tuple(parts[1:])] = parts[0]
    return N, const, terms


def poly_eval(const, terms, S):
    v = const
    for idx, c in terms.items():
        p = c
        for i in idx:
            p *= S[i]
        v += p
    return v


def factor21_instance():
    """E = f - const: every coefficient c of a product term becomes a coupling
    -c (the energy carries a minus sign in front of every term)."""
    N, const, terms = load_poly(os.path.join(GOLDEN, "factor21.txt"))
    h = np.zeros(3, np.int32)
    ei, ej, J, tri, K = [], [], [], [], []
    for idx, c in terms.items():
        if len(idx) == 1:
            h[idx[0]] = -c
        elif len(idx) == 2:
            ei.append(idx[0]); ej.append(idx[1]); J.append(-c)
        else:
            tri.append(idx); K.append(-c)
    inst = gen.Instance(n=3, ei=ei, ej=ej, J=J, h=h, tri=tri, K=K,
                        colour=np.array([0, 1, 2], np.int32), name="factor21")
    return inst, N, const, terms


def all_states(n):
    return np.array(list(itertools.product([1, -1], repeat=n)), dtype=np.int8)


def flip_deltas(inst, s):
    """E(s with i flipped) - E(s) for every i, by direct energy evaluation."""
    e0 = oracle.energy(inst, s)
    out = np.empty(inst.n, np.int64)
    for i in range(inst.n):
        t = s.copy()
        t[i] = -t[i]
        out[i] = oracle.energy(inst, t) - e0
    return out


SMALL = [gen.random_small(n, seed=100 + n) for n in (5, 8, 11, 14)]


# ---------------------------------------------------------- paper example


def test_factor21_fixture_is_the_factoring_square():
    """Caption polynomial == (N - x y)^2 with x = 2 - S0, y = 4 - 2 S1 - S2
    (bit = (1 - S)/2, the two least-significant bits fixed to 1)."""
    _, N, const, terms = factor21_instance()
    for S in all_states(3):
        S = [int(v) for v in S]
        x = 2 - S[0]
        y = 4 - 2 * S[1] - S[2]
        assert poly_eval(const, terms, S) == (N - x * y) ** 2


def test_factor21_energy_and_ground_state():
    inst, N, const, terms = factor21_instance()
    for S in all_states(3):
        assert oracle.energy(inst, S) == poly_eval(const, terms, [int(v) for v in S]) - const
    e, s, deg = oracle.brute_force(inst)
    assert e == -const and deg == 1
    assert list(s) == [-1, -1, -1]
    x, y = 2 - s[0], 4 - 2 * s[1] - s[2]
    assert x * y == N and (x, y) == (3, 7)


def test_factor21_greedy_reaches_factors_from_every_start():
    """(-1,-1,-1) is the only single-flip local minimum of the N=21 energy
    (checked by direct energies), so colour-ordered greedy descent must reach
    it from all 8 starts."""
    inst, N, const, _ = factor21_instance()
    minima = [tuple(S) for S in all_states(3) if np.all(flip_deltas(inst, S) >= 0)]
    assert minima == [(-1, -1, -1)]
    st = oracle.ReplicaState(3, 8)
    st.spins[:] = all_states(3)
    inst8 = inst.replace(restarts=8)
    st, rc = oracle.run(inst8, seed=1, state=st)
    assert rc == 0
    assert np.all(st.energy == -const)
    assert np.all(st.spins == -1)
    assert np.all(st.sweeps <= 3)


# ------------------------------------------------------------ closed forms


def _closed_form_instances():
    out = [gen.ferromagnet(gen.random_small(n, seed=n)) for n in (6, 10, 13)]
    out.append(gen.ferromagnet(gen.lattice((4, 4), seed=3, j_values=(1, 2, 3), h_range=(0, 2))))
    out.append(gen.ferromagnet(gen.chimera(2, 2, seed=5, triple_cells_frac=0.5)))
    return out


@pytest.mark.parametrize("inst", _closed_form_instances(), ids=lambda i: i.name)
def test_ferromagnet_ground_state(inst):
    """No term can be frustrated: E_gs = -sum|J| - sum|h| - sum|K| at all +1
    (Sec. II unfrustrated ground state; Sec. III eq. (2) bound is tight)."""
    lb = oracle.lower_bound(inst)
    ones = np.ones(inst.n, np.int8)
    assert oracle.energy(inst, ones) == lb
    if inst.n <= 20:
        e, _, _ = oracle.brute_force(inst)
        assert e == lb
    st = oracle.ReplicaState(inst.n, 1)
    st.spins[:] = 1
    st, rc = oracle.run(inst, seed=3, state=st)
    assert st.flips[0] == 0 and st.sweeps[0] == 1 and st.energy[0] == lb


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mattis_ground_state(seed):
    """Mattis (gauge-transformed ferromagnet): ground state s = xi with
    E = -sum|J| - sum|h| - sum|K|."""
    rng = np.random.default_rng(seed)
    for base in (gen.random_small(12, seed=seed + 40), gen.chimera(2, 2, seed=seed, triple_cells_frac=0.5),
                 gen.lattice((3, 3, 3), seed=seed, h_range=(-2, 2))):
        xi = np.where(rng.random(base.n) < 0.5, -1, 1).astype(np.int8)
        m = gen.gauge(base, xi, absolute=True)
        lb = oracle.lower_bound(m)
        assert oracle.energy(m, xi) == lb
        if m.n <= 20:
            e, _, _ = oracle.brute_force(m)
            assert e == lb


def test_chain_ground_state_is_unfrustrated():
    """1-D open chain, h = 0 (Table I, first row: solvable analytically; a
    tree is never frustrated): E_gs = -sum|J|."""
    for n in (2, 5, 9, 16):
        c = gen.chain(n, seed=n)
        e, _, _ = oracle.brute_force(c)
        assert e == -int(np.abs(c.J).sum())


def test_lower_bound_holds_everywhere():
    """Sec. III eq. (2) (plus -sum|K|) bounds every state."""
    for inst in SMALL[:3]:
        lb = oracle.lower_bound(inst)
        for S in all_states(inst.n):
            assert oracle.energy(inst, S) >= lb


# --------------------------------------------------------------- symmetries


@pytest.mark.parametrize("inst", SMALL, ids=lambda i: i.name)
def test_gauge_invariance_of_energy(inst):
    rng = np.random.default_rng(7)
    xi = np.where(rng.random(inst.n) < 0.5, -1, 1).astype(np.int8)
    g = gen.gauge(inst, xi)
    for _ in range(20):
        s = np.where(rng.random(inst.n) < 0.5, -1, 1).astype(np.int8)
        assert oracle.energy(g, xi * s) == oracle.energy(inst, s)


@pytest.mark.parametrize("rule", [oracle.GREEDY, oracle.GREEDY_TIE])
def test_gauge_covariance_of_the_descent(rule):
    """Flip decisions depend on dE_i = 2 s_i f_i, which a gauge transform
    leaves unchanged, and on RNG counters that do not involve spins: the
    trajectory on (gauge instance, xi*s0) is xi times the original one."""
    for inst in (gen.random_small(40, seed=3, n_triples=30).replace(restarts=4),
                 gen.chimera(3, 3, seed=9, triple_cells_frac=0.5).replace(restarts=4),
                 gen.lattice((6, 6, 6), seed=4, h_range=(-2, 2)).replace(restarts=2)):
        rng = np.random.default_rng(11)
        xi = np.where(rng.random(inst.n) < 0.5, -1, 1).astype(np.int8)
        g = gen.gauge(inst, xi)
        a, _ = oracle.run(inst, seed=5, rule=rule, max_sweeps=30, until_converged=(rule == 0))
        st = oracle.ReplicaState(inst.n, inst.restarts)
        # same starts as `a` drew: redraw them with a zero-sweep run
        s0, _ = oracle.run(inst, seed=5, rule=rule, max_sweeps=0)
        st.spins[:] = s0.spins * xi
        b, _ = oracle.run(g, seed=5, rule=rule, max_sweeps=30, until_converged=(rule == 0), state=st)
        assert np.array_equal(b.spins, a.spins * xi)
        assert np.array_equal(b.energy, a.energy)
        assert np.array_equal(b.flips, a.flips)
        assert np.array_equal(b.sweeps, a.sweeps)


def test_global_flip_symmetry():
    """h = 0 and no triples: E(-s) = E(s) and the trajectory from -s0 is the
    negated trajectory."""
    inst = gen.lattice((8, 8), seed=6, restarts=3)
    s0, _ = oracle.run(inst, seed=2, max_sweeps=0)
    a, _ = oracle.run(inst, seed=2, max_sweeps=50, state=s0.copy())
    neg = s0.copy()
    neg.spins = -neg.spins
    b, _ = oracle.run(inst, seed=2, max_sweeps=50, state=neg)
    assert np.array_equal(b.spins, -a.spins)
    assert np.array_equal(b.energy, a.energy)


# ------------------------------------------------------------ exhaustive search


@pytest.mark.parametrize("inst", SMALL[:3], ids=lambda i: i.name)
def test_brute_force_matches_enumeration(inst):
    """Gray-code search (incremental single-flip changes) == minimum over all
    2^n direct energy evaluations, including the number of ground states."""
    S = all_states(inst.n)
    E = np.array([oracle.energy(inst, s) for s in S])
    e, s, deg = oracle.brute_force(inst)
    assert e == E.min()
    assert deg == int((E == e).sum())
    assert oracle.energy(inst, s) == e


def test_square4_exhaustive_and_greedy_above_it():
    """4x4 periodic +-J lattice: exhaustive ground state; every greedy result
    lies at or above it and at or above the eq. (2) bound."""
    inst = gen.cfg1_square4().replace(restarts=64)
    e, _, _ = oracle.brute_force(inst)
    st, rc = oracle.run(inst, seed=7)
    assert rc == 0
    assert np.all(st.energy >= e)
    assert e >= oracle.lower_bound(inst)
    assert st.energy.min() == e  # 64 starts find it on this 16-spin instance


# ----------------------------------------------------------- descent invariants


@pytest.mark.parametrize("rule", [oracle.GREEDY, oracle.GREEDY_TIE])
@pytest.mark.parametrize("inst", [gen.random_small(30, seed=8, n_triples=20),
                                  gen.chimera(2, 3, seed=2, triple_cells_frac=0.5),
                                  gen.lattice((6, 6), seed=1, h_range=(-2, 2))],
                         ids=["small30", "chimera2x3", "sq6"])
def test_tracked_energy_equals_recomputed_after_every_phase(inst, rule):
    """The tracked energy (start energy plus the 2 s_i f_i of every flip) equals
    a fresh evaluation of eq. (1)/(5) after every colour phase; it never
    increases, changes by even amounts and stays above the bound."""
    tr = oracle.trace(inst, seed=9, rule=rule, max_sweeps=20, until_converged=(rule == 0))
    lb = oracle.lower_bound(inst)
    prev = None
    for e, s in zip(tr["E"], tr["S"]):
        assert e == oracle.energy(inst, s)
        assert e >= lb
        if prev is not None:
            assert e <= prev and (prev - e) % 2 == 0
        prev = e


@pytest.mark.parametrize("inst", SMALL + [gen.cfg1_square16(), gen.chimera(4, 4, seed=3)],
                         ids=lambda i: i.name)
def test_greedy_result_is_a_local_minimum(inst):
    """At GREEDY convergence no single flip lowers the energy (the stopping
    rule of Fig. 3: a pass brings no improvement)."""
    inst = inst.replace(restarts=3)
    st, rc = oracle.run(inst, seed=4)
    assert rc == 0 and np.all(st.converged == 1)
    for r in range(3):
        assert np.all(flip_deltas(inst, st.spins[r]) >= 0)
        assert st.energy[r] == oracle.energy(inst, st.spins[r])


def test_greedy_flip_count_bound():
    """Every GREEDY flip lowers E by at least 2, so flips <= (E0 - E_lb)/2."""
    inst = gen.random_small(60, seed=5, n_triples=40).replace(restarts=8)
    s0, _ = oracle.run(inst, seed=3, max_sweeps=0)
    st, _ = oracle.run(inst, seed=3, state=s0.copy())
    lb = oracle.lower_bound(inst)
    for r in range(8):
        e0 = oracle.energy(inst, s0.spins[r])
        assert st.flips[r] <= (e0 - lb) // 2
        assert e0 - st.energy[r] >= 2 * st.flips[r]


@pytest.mark.parametrize("rule", [oracle.GREEDY, oracle.GREEDY_TIE])
def test_order_inside_a_colour_does_not_matter(rule):
    """Under a proper colouring of the primal graph every energy term holds at
    most one spin of a colour, so ascending, descending and simultaneous
    updates of a colour class give identical trajectories."""
    for inst in (gen.random_small(50, seed=12, n_triples=40), gen.chimera(3, 3, seed=1),
                 gen.lattice((6, 6, 6), seed=4, h_range=(-2, 2))):
        ref = oracle.trace(inst, seed=21, rule=rule, max_sweeps=15, until_converged=False)
        for order in (oracle.ORDER_DESCENDING, oracle.ORDER_SIMULTANEOUS):
            got = oracle.trace(inst, seed=21, rule=rule, max_sweeps=15, until_converged=False,
                               order=order)
            assert np.array_equal(got["E"], ref["E"])
            assert np.array_equal(got["S"], ref["S"])


def test_order_test_detects_an_improper_colouring():
    """Sensitivity check for the test above: with every spin in one colour,
    simultaneous and sequential updates differ on a frustrated triangle."""
    inst = gen.Instance(n=3, ei=[0, 1, 0], ej=[1, 2, 2], J=[-1, -1, -1])
    s = np.ones(3, np.int8)
    seq, _ = oracle.trace_unchecked(inst, np.zeros(3, np.int32), s, max_sweeps=1)
    sim, _ = oracle.trace_unchecked(inst, np.zeros(3, np.int32), s, max_sweeps=1,
                                    order=oracle.ORDER_SIMULTANEOUS)
    assert not np.array_equal(seq, sim)


@pytest.mark.parametrize("rule,uc", [(oracle.GREEDY, True), (oracle.GREEDY_TIE, False),
                                     (oracle.GREEDY_TIE, True)])
def test_resume_is_exact(rule, uc):
    """run(a) then run(b) == run(a+b): the RNG is keyed on the absolute sweep
    index, so splitting a run changes nothing."""
    inst = gen.lattice((10, 10, 10), seed=3, h_range=(-2, 2), restarts=3)
    full, _ = oracle.run(inst, seed=8, rule=rule, max_sweeps=12, until_converged=uc)
    part, _ = oracle.run(inst, seed=8, rule=rule, max_sweeps=5, until_converged=uc)
    part, _ = oracle.run(inst, seed=8, rule=rule, max_sweeps=7, until_converged=uc, state=part)
    for k in ("spins", "energy", "sweeps", "flips", "converged"):
        assert np.array_equal(getattr(part, k), getattr(full, k)), k


def test_tie_rule_uses_the_sweep_word():
    """GREEDY_TIE keeps moving on a +-J lattice (zero-cost flips keep
    happening in every sweep) while GREEDY stops."""
    inst = gen.lattice((12, 12), seed=2)
    g, _ = oracle.run(inst, seed=1, rule=oracle.GREEDY, max_sweeps=200, until_converged=True)
    t, _ = oracle.run(inst, seed=1, rule=oracle.GREEDY_TIE, max_sweeps=200, until_converged=False)
    assert g.sweeps[0] < 200 and g.converged[0] == 1
    assert t.sweeps[0] == 200 and t.flips[0] > g.flips[0] + 100


def test_multistart_best_lowest_restart_on_ties():
    assert oracle.best([5, -3, -7, -7, 0]) == (2, -7)
    assert oracle.best([1]) == (0, 1)


# ------------------------------------------------------------------ colouring


@pytest.mark.parametrize("dims", [(4, 4), (16, 16), (6, 8), (4, 4, 4), (10, 10, 10), (6, 4, 8)])
def test_first_fit_on_even_periodic_lattice_is_checkerboard(dims):
    inst = gen.lattice(dims, seed=0)
    col = oracle.first_fit_colouring(inst)
    coords = np.indices(dims).reshape(len(dims), -1)
    assert np.array_equal(col, coords.sum(axis=0) % 2)


def test_first_fit_small_graphs():
    path = gen.chain(7)
    assert list(oracle.first_fit_colouring(path)) == [0, 1, 0, 1, 0, 1, 0]
    k5 = gen.complete_graph(5)
    assert list(oracle.first_fit_colouring(k5)) == [0, 1, 2, 3, 4]
    tri_only = gen.Instance(n=4, ei=[], ej=[], J=[], tri=[[0, 1, 2]], K=[1])
    assert list(oracle.first_fit_colouring(tri_only)) == [0, 1, 2, 0]
    odd_ring = gen.chain(5, periodic=True)
    assert list(oracle.first_fit_colouring(odd_ring)) == [0, 1, 0, 1, 2]


def test_colourings_are_proper():
    for inst in (gen.chimera(8, 8, seed=3), gen.erdos_renyi_triples(2000, seed=1),
                 gen.random_regular3(1000, seed=2)):
        col = oracle.first_fit_colouring(inst)
        assert oracle.colouring_is_proper(inst, col)
        bad = col.copy()
        bad[inst.ei[0]] = bad[inst.ej[0]]
        assert not oracle.colouring_is_proper(inst, bad)


# ---------------------------------------------------------------------- RNG


def test_philox_bits_are_balanced():
    """Frequency test over 2^18 outputs: every bit position of every word is
    1 with probability 1/2 within 5 sigma."""
    out = oracle.philox_stream(12345, 0, 7, 3, 1, 1 << 18)
    bits = np.unpackbits(out.view(np.uint8), bitorder="little").reshape(out.shape[0], 128)
    p = bits.mean(axis=0)
    sigma = 0.5 / np.sqrt(out.shape[0])
    assert np.all(np.abs(p - 0.5) < 5 * sigma)


def test_philox_avalanche_and_key_dependence():
    """One flipped counter or key bit changes about half of the 128 output bits."""
    rng = np.random.default_rng(0)
    flips = []
    for _ in range(400):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64).astype(np.uint32)
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64).astype(np.uint32)
        base = oracle.philox(c, k)
        for which in range(6):
            c2, k2 = c.copy(), k.copy()
            bit = np.uint32(1 << int(rng.integers(0, 32)))
            if which < 4:
                c2[which] ^= bit
            else:
                k2[which - 4] ^= bit
            diff = np.unpackbits((base ^ oracle.philox(c2, k2)).view(np.uint8)).sum()
            flips.append(diff)
    flips = np.array(flips)
    assert abs(flips.mean() - 64) < 1.0
    assert flips.min() > 20


def test_random_start_is_uniform():
    """Start spins are +-1 with probability 1/2 (Sec. IV, uniform random start)."""
    inst = gen.lattice((64, 64), seed=0, restarts=16)
    st, _ = oracle.run(inst, seed=99, max_sweeps=0)
    frac = (st.spins == 1).mean()
    n = st.spins.size
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n)
    assert not np.array_equal(st.spins[0], st.spins[1])


@pytest.mark.parametrize("inst", [gen.random_small(40, seed=31, n_triples=30), gen.cfg1_square16(),
                                  gen.chimera(3, 3, seed=8)], ids=lambda i: i.name)
def test_stopping_rule_counts_the_first_zero_flip_sweep(inst):
    """Fig. 3 stops when a pass fails to improve: the last sweep of a GREEDY
    run changes no spin, every earlier sweep changes at least one, and the
    sweep count includes the final zero-flip sweep."""
    col = inst.colour if inst.colour is not None else oracle.first_fit_colouring(inst)
    C = int(col.max()) + 1
    for seed in range(4):
        tr = oracle.trace(inst, seed=seed, max_sweeps=1000)
        assert tr["converged"]
        S = tr["S"]
        assert S.shape[0] == tr["sweeps"] * C
        ends = S[C - 1::C]                       # state after each sweep
        start = oracle.run(inst.replace(restarts=1), seed=seed, max_sweeps=0)[0].spins[0]
        before = np.concatenate([start[None], ends[:-1]])
        changed = np.any(ends != before, axis=1)
        assert not changed[-1]
        assert np.all(changed[:-1])
        assert tr["flips"] == int(sum(np.sum(a != b) for a, b in zip(ends, before)))
