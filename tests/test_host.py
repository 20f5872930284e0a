"""Host-side checks of the C-ABI library that need no GPU: every declared
symbol is exported, ingest validation and range errors, colouring (given,
first-fit, lattice checkerboard) against the oracle's independent
implementation, workspace arithmetic, knobs and call-order errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import instances as gen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sg():
    import paper_0912_3912_amd as sg
    sg.lib()
    return sg


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "sg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(sg):
    names = declared_symbols()
    assert len(names) >= 15
    lib = ctypes.CDLL(sg.library_path())
    for name in names:
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in sg.SIGNATURES}
    assert set(names) == bound


def test_version(sg):
    assert sg.lib().sg_version().decode().startswith("sg ")


def _err(sg, insts, **kw):
    with pytest.raises(sg.SGError) as e:
        sg.load_instance(insts, **kw)
    return e.value


def test_validation_errors(sg):
    base = gen.random_small(10, seed=1)
    e = _err(sg, [base.replace(ei=np.append(base.ei, 3), ej=np.append(base.ej, 3), J=np.append(base.J, 1))])
    assert e.status == sg.SG_EINVAL and "self-loop" in str(e)
    a, b = int(base.ei[0]), int(base.ej[0])
    e = _err(sg, [base.replace(ei=np.append(base.ei, b), ej=np.append(base.ej, a), J=np.append(base.J, 1))])
    assert e.status == sg.SG_EINVAL and "twice" in str(e)
    e = _err(sg, [base.replace(ei=np.append(base.ei, 0), ej=np.append(base.ej, 10), J=np.append(base.J, 1))])
    assert e.status == sg.SG_EINVAL and "out of range" in str(e)
    t = base.tri[0]
    e = _err(sg, [base.replace(tri=np.vstack([base.tri, t[::-1]]), K=np.append(base.K, 1))])
    assert e.status == sg.SG_EINVAL and "twice" in str(e)
    e = _err(sg, [base.replace(tri=np.vstack([base.tri, [1, 2, 1]]), K=np.append(base.K, 1))])
    assert e.status == sg.SG_EINVAL and "repeats" in str(e)
    e = _err(sg, [base.replace(restarts=0)])
    assert e.status == sg.SG_EINVAL
    e = _err(sg, [base.replace(n=0)])
    assert e.status == sg.SG_EINVAL
    # the error names the failing instance of a batch
    e = _err(sg, [base, base.replace(ei=np.append(base.ei, 3), ej=np.append(base.ej, 3), J=np.append(base.J, 1))])
    assert "instance 1" in str(e)


def test_range_errors(sg):
    """The boundary takes any int32 coefficient and rejects (SG_ERANGE) only a
    spin whose |h| + sum|J| + sum|K| exceeds 2^31 - 1, i.e. whose local field
    would overflow int32 (and a total beyond 2^63 - 1, which no instance of
    test size reaches).  Values or sizes beyond the packed words select the
    wide form, invisibly to the caller."""
    base = gen.random_small(10, seed=2)
    for kind, v in (("J", 128), ("h", -128), ("K", 200), ("J", 10**6), ("h", -(2**30))):
        arr = getattr(base, kind).copy()
        arr[0] = v
        h = sg.load_instance([base.replace(**{kind: arr})])
        assert h.query("wide_instances") == 1, (kind, v)
        h.free()
    # a star whose centre field is exactly 2^31 - 1: accepted; one more: SG_ERANGE
    n = 3
    c = 2**31 - 1
    star = gen.Instance(n=n, ei=np.zeros(n - 1, np.int32), ej=np.arange(1, n, dtype=np.int32),
                        J=np.array([c // 2, c - c // 2], np.int32))
    h = sg.load_instance([star])
    assert h.query("wide_instances") == 1
    h.free()
    over = star.replace(h=np.array([1, 0, 0], np.int32))
    e = _err(sg, [over])
    assert e.status == sg.SG_ERANGE and "2147483647" in str(e)
    lowest = base.J.copy()
    lowest[0] = -2**31           # |J| = 2^31 alone exceeds the limit
    assert _err(sg, [base.replace(J=lowest)]).status == sg.SG_ERANGE
    # the old packed limits are no longer visible: 2^23 per spin, restarts beyond one launch dimension
    n = 70000
    big = gen.Instance(n=n, ei=np.zeros(n - 1, np.int32), ej=np.arange(1, n, dtype=np.int32),
                       J=np.full(n - 1, 127, np.int32))
    h = sg.load_instance([big])
    assert h.query("wide_instances") == 1
    h.free()
    h = sg.load_instance([base.replace(restarts=70000)])
    assert h.query("wide_instances") == 1 and h.query("total_replicas") == 70000
    h.free()
    h = sg.load_instance([base])
    assert h.query("wide_instances") == 0
    h.free()


def test_improper_colouring_rejected(sg):
    inst = gen.lattice((6, 6), seed=1)
    col = inst.colour.copy()
    col[0] = col[1]
    e = _err(sg, [inst.replace(colour=col)])
    assert e.status == sg.SG_EINVAL and "not proper" in str(e)
    neg = inst.colour.copy()
    neg[3] = -1
    assert _err(sg, [inst.replace(colour=neg)]).status == sg.SG_EINVAL


@pytest.mark.parametrize("inst", [gen.chimera(8, 8, seed=3), gen.erdos_renyi_triples(3000, seed=2),
                                  gen.random_regular3(2000, seed=1), gen.random_small(40, seed=5),
                                  gen.lattice((5, 7), seed=1), gen.lattice((6, 6, 6), seed=1).replace(colour=None)],
                         ids=lambda i: i.name)
def test_first_fit_matches_oracle(sg, inst):
    inst = inst.replace(colour=None)
    h = sg.load_instance([inst])
    info = h.info(0)
    ref = oracle.first_fit_colouring(inst)
    assert np.array_equal(info["colour"], ref)
    assert info["colours"] == int(ref.max()) + 1
    assert oracle.colouring_is_proper(inst, info["colour"])


@pytest.mark.parametrize("dims", [(8, 6), (4, 10), (5, 7), (6, 4, 8), (4, 4, 4), (5, 6, 4), (10, 12, 14)])
def test_first_fit_matches_oracle_with_lattice_hint(sg, dims):
    """With the lattice hint, even extents take the checkerboard directly; it
    must be the first-fit colouring in index order (odd extents run first-fit)."""
    inst = gen.lattice(dims, seed=2, h_range=(-2, 2)).replace(colour=None)
    info = sg.load_instance([inst], lattice_dims=[dims]).info(0)
    ref = oracle.first_fit_colouring(inst)
    assert np.array_equal(info["colour"], ref)
    assert info["colours"] == int(ref.max()) + 1


def test_given_colouring_is_kept(sg):
    inst = gen.lattice((8, 8), seed=1)
    col = 1 - inst.colour  # the other checkerboard
    h = sg.load_instance([inst.replace(colour=col)], lattice_dims=[(8, 8)])
    assert np.array_equal(h.info(0)["colour"], col)
    assert h.info(0)["lattice"] == 1


def test_lattice_hint_checks(sg):
    inst = gen.lattice((6, 4, 8), seed=2)
    assert sg.load_instance([inst], lattice_dims=[(6, 4, 8)]).info(0)["lattice"] == 1
    e = _err(sg, [inst], lattice_dims=[(4, 6, 8)])
    assert e.status == sg.SG_EINVAL and "not a lattice bond" in str(e)
    e = _err(sg, [inst], lattice_dims=[(6, 4, 4)])
    assert e.status == sg.SG_EINVAL
    # odd extent: accepted as a lattice, but the lattice schedules stay off
    odd = gen.lattice((5, 6), seed=1)
    assert sg.load_instance([odd], lattice_dims=[(5, 6)]).info(0)["lattice"] == 0
    # triples: lattice schedules stay off
    assert sg.load_instance([gen.lattice((6, 6), seed=1)], lattice_dims=[(6, 6)]).info(0)["lattice"] == 1


def test_workspace_and_info(sg):
    insts = [gen.chimera(4, 4, seed=1, restarts=3), gen.erdos_renyi_triples(500, seed=1, restarts=2)]
    h = sg.load_instance(insts)
    assert h.info(0)["replica_base"] == 0 and h.info(1)["replica_base"] == 3
    assert h.query("total_replicas") == 5 and h.query("instances") == 2
    b1 = h.workspace_bytes()
    h2 = sg.load_instance([insts[0].replace(restarts=30), insts[1]])
    assert h2.workspace_bytes() > b1 > 0
    assert b1 % 256 == 0


def test_knobs(sg):
    h = sg.load_instance([gen.chimera(2, 2, seed=1)])
    for k, v in [("lattice_k", 3), ("lattice_max_tiles", 8), ("lattice_wg_max_n", 1000), ("block_rg", 128),
                 ("block_min_restarts", 8), ("queue_wave_max_n", 2048), ("queue_grid", 100),
                 ("queue_min_items", 4), ("graph_sweeps", 64), ("lattice_msc", 0), ("msc_k", 9),
                 ("block_groups", 3), ("block_bits", 0), ("bits_groups", 8), ("fm_key32", 0),
                 ("defer_energy", 0), ("fm_waves", 8)]:
        h.tune(k, v)
        assert h.query(k) == v
    for k, v in [("lattice_k", 0), ("lattice_k", 17), ("block_rg", 100), ("queue_wave_max_n", 20000),
                 ("graph_sweeps", 0), ("graph_sweeps", 1025), ("lattice_msc", 2), ("msc_k", 63),
                 ("block_groups", 65), ("block_groups", -1), ("block_bits", 2), ("bits_groups", 3), ("fm_key32", 2),
                 ("defer_energy", 2), ("fm_waves", 17), ("fm_waves", -1), ("no_such_knob", 1)]:
        with pytest.raises(sg.SGError) as e:
            h.tune(k, v)
        assert e.value.status == sg.SG_EINVAL


def test_fields_knob_changes_the_workspace(sg):
    inst = gen.erdos_renyi_triples(1000, seed=1, restarts=3)
    h = sg.load_instance([inst])
    b0 = h.workspace_bytes()
    h.tune("fields", 1)
    assert h.query("fields") == 1
    assert h.workspace_bytes() >= b0 + 3 * 4 * 1000
    h.tune("fields", 0)
    assert h.workspace_bytes() == b0
    with pytest.raises(sg.SGError):
        h.tune("fields", 2)


def test_calls_before_bind(sg):
    h = sg.load_instance([gen.chimera(2, 2, seed=1)])
    for fn in (lambda: h.run_sweeps(seed=1), lambda: h.energy(), lambda: h.spins_out(0, 0), lambda: h.best(),
               lambda: h.init_spins(1), lambda: h.counters()):
        with pytest.raises(sg.SGError) as e:
            fn()
        assert e.value.status == sg.SG_ESTATE


def test_free_is_idempotent(sg):
    h = sg.load_instance([gen.chimera(2, 2, seed=1)])
    h.free()
    h.free()
    assert sg.lib().sg_free(None) == 0


def test_dense_validation(sg):
    d = gen.random_dense(10, 20, seed=1)
    h = sg.load_dense([d])
    assert h.info(0)["n"] == 10 and h.workspace_bytes() > 0
    bad = [d.replace(n=65), d.replace(n=0),
           d.replace(masks=np.append(d.masks, np.uint64(1 << 12)), coefs=np.append(d.coefs, 1)),
           d.replace(masks=np.append(d.masks, d.masks[0]), coefs=np.append(d.coefs, 1)),
           d.replace(masks=np.append(d.masks, np.uint64(0)), coefs=np.append(d.coefs, 1)),
           d.replace(restarts=0)]
    for b in bad:
        with pytest.raises(sg.SGError) as e:
            sg.load_dense([b])
        assert e.value.status == sg.SG_EINVAL
    big = d.replace(masks=np.array([1, 2], np.uint64), coefs=np.array([1 << 61, 1 << 61], np.int64))
    with pytest.raises(sg.SGError) as e:
        sg.load_dense([big])
    assert e.value.status == sg.SG_ERANGE


def test_dense_colouring_is_first_fit(sg):
    """The sweep order of a dense instance: first-fit colouring of the graph of
    shared terms, equal to the sparse ingest's colouring of the same graph."""
    inst = gen.random_small(30, seed=4, p_edge=0.2, n_triples=6)
    d = gen.dense_from_sparse(inst)
    col = sg.load_dense([d]).info(0)["colour"]
    assert np.array_equal(col, oracle.first_fit_colouring(inst))
