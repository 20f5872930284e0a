"""GPU checks of the serving loop: a Poisson mix of lattice, Chimera and
3-regular requests under a tight HBM budget, admitted as slots and memory
free up, with overlapping work.  Every result must equal the same request
run alone (tolerance zero) and the CPU oracle."""
import numpy as np
import pytest

import instances as gen
import oracle
from parity import log

pytestmark = pytest.mark.gpu


def _trace(count, seed, n_lo, n_hi):
    reqs, gaps = gen.cfg5_trace(count=count, seed=seed, n_lo=n_lo, n_hi=n_hi)
    return [gen.serving_instance(f, n, s, i) for (f, n, s, i) in reqs], gaps


def _alone(inst, seed):
    import paper_0912_3912_amd as sg
    h = sg.load_instance([inst]).bind()
    h.init_spins(seed)
    st = h.run_sweeps(seed=seed)
    E, r = h.best()
    s = h.spins_out(0, int(r[0]))
    h.free()
    return int(E[0]), int(r[0]), s, st


def test_serving_mix_equals_alone_and_oracle(gpu):
    from paper_0912_3912_amd.serve import Request, Server
    insts, gaps = _trace(30, 5, 500, 30000)
    import paper_0912_3912_amd as sg
    fps = [sg.load_instance([i]).workspace_bytes() for i in insts]
    budget = int(2.5 * max(fps))
    log(f"serving: 30 requests, footprints {min(fps)}..{max(fps)} B, budget {budget} B")
    server = Server(budget_bytes=budget, slots=3, ingest_workers=4, keep_spins=True)
    reqs = [Request(rid=k, instance=inst, seed=11) for k, inst in enumerate(insts)]
    results = server.run_trace(reqs, gaps, time_scale=0.001)
    server.close()
    assert all(r.status == "ok" for r in results), [r.status for r in results]
    assert server.pool.peak <= server.pool.size
    assert max(t[2] for t in server.timeline) >= 2, "no two requests were ever resident together"
    # intervals on the GPU overlap for some pair
    iv = sorted((r.started, r.done) for r in results)
    assert any(b[0] < a[1] for a, b in zip(iv, iv[1:]))
    for inst, res in zip(insts, results):
        E, r, s, st = _alone(inst, 11)
        assert (res.energy, res.best_restart) == (E, r), inst.name
        assert np.array_equal(res.spins, s), inst.name
        assert res.flips == st["flips"] and res.attempts == st["attempts"]
        ref, _ = oracle.run(inst, seed=11)
        assert res.energy == int(ref.energy.min())
        assert np.array_equal(res.spins, ref.spins[int(np.argmin(ref.energy))])


def test_serving_rejects_oversized_and_cancels(gpu):
    from paper_0912_3912_amd.serve import Request, Server
    small = gen.lattice((16, 16), seed=1, instance_id=1)
    big = gen.random_regular3(200000, seed=2, instance_id=2)
    long_ = gen.lattice((200, 200), seed=3, instance_id=3)
    import paper_0912_3912_amd as sg
    budget = 3 * sg.load_instance([long_]).workspace_bytes()
    server = Server(budget_bytes=budget, slots=1, ingest_workers=2)
    server.t0 = None
    server.submit(Request(rid=0, instance=long_, seed=1, rule=1, max_sweeps=3000, until_converged=False))
    server.submit(Request(rid=1, instance=big, seed=1))
    server.submit(Request(rid=2, instance=small, seed=1))
    cancelled = server.cancel(2)
    res = server.wait([0, 1, 2])
    server.close()
    assert res[0].status == "ok"
    assert res[1].status == "rejected"
    assert res[2].status == ("cancelled" if cancelled else "ok")
