"""sg_bind_noalloc (the library's static device workspace; no allocation by
the library or the caller) against sg_bind (a torch workspace): identical
spins, energies and counters bit for bit, on consecutive calls whose second
input is smaller than the first, and the size limit enforced."""
import ctypes

import numpy as np
import pytest

import instances as gen
from parity import log

pytestmark = pytest.mark.gpu


def _bind_noalloc(sg, h):
    import torch
    sp = torch.cuda.current_stream().cuda_stream
    st = sg.lib().sg_bind_noalloc(h._h, ctypes.c_void_p(sp))
    if st != 0:
        raise sg.SGError(st, sg.lib().sg_last_error().decode())


def _run(inst, noalloc, seed, rule, max_sweeps, until_converged, dims=None):
    import paper_0912_3912_amd as sg
    h = sg.load_instance([inst], lattice_dims=dims)
    if noalloc:
        _bind_noalloc(sg, h)
    else:
        h.bind()
    h.init_spins(seed)
    st = h.run_sweeps(seed=seed, rule=rule, max_sweeps=max_sweeps, until_converged=until_converged)
    out = {"E": h.energy(), "Er": h.energy(recompute=True), "counters": h.counters(),
           "spins": h.spins_out_batch(0), "best": h.best(), "attempts": st["attempts"], "flips": st["flips"],
           "schedule": st["schedule_used"]}
    h.free()
    return out


def _same(a, b):
    for k in ("E", "Er", "spins"):
        assert np.array_equal(a[k], b[k]), k
    for x, y in zip(a["counters"], b["counters"]):
        assert np.array_equal(x, y)
    for x, y in zip(a["best"], b["best"]):
        assert np.array_equal(x, y)
    assert (a["attempts"], a["flips"], a["schedule"]) == (b["attempts"], b["flips"], b["schedule"])


CASES = [
    # (name, instance, seed, rule, max_sweeps, until_converged, lattice dims), by decreasing workspace
    ("cubic100 TIE 40 sweeps (tile kernel)", lambda: gen.cfg2_cubic100(), 7, 1, 40, False, [(100, 100, 100)]),
    ("square 16x16, 64 restarts", lambda: gen.cfg1_square16(), 7, 0, 10000, True, [(16, 16)]),
    ("chimera 8x8, 256 restarts", lambda: gen.chimera(8, 8, seed=3, instance_id=9, restarts=256), 5, 0, 10000, True,
     None),
    ("ER 3000 with triples, 4 restarts", lambda: gen.erdos_renyi_triples(3000, seed=2, restarts=4), 3, 0, 10000, True,
     None),
]


def test_noalloc_matches_bind_on_consecutive_calls(gpu):
    import paper_0912_3912_amd as sg
    sizes = []
    for name, mk, seed, rule, ms, uc, dims in CASES:
        inst = mk()
        h = sg.load_instance([inst], lattice_dims=dims)
        sizes.append(h.workspace_bytes())
        h.free()
        log(f"noalloc case: {name}, workspace {sizes[-1]} B")
        ref = _run(inst, False, seed, rule, ms, uc, dims)
        got = _run(inst, True, seed, rule, ms, uc, dims)
        _same(ref, got)
        # the static workspace keeps the last call's contents: a second call in a row
        again = _run(inst, True, seed, rule, ms, uc, dims)
        _same(ref, again)
    assert sizes == sorted(sizes, reverse=True), sizes


def test_noalloc_rejects_oversized(gpu):
    import paper_0912_3912_amd as sg
    inst = gen.erdos_renyi_triples(1_000_000, seed=1, restarts=64)
    h = sg.load_instance([inst])
    need = h.workspace_bytes()
    assert need > (64 << 20)
    with pytest.raises(sg.SGError) as e:
        _bind_noalloc(sg, h)
    assert e.value.status == sg.SG_ENOMEM and "static workspace" in str(e.value), (need, str(e.value))
    h.free()
