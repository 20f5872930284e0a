"""GPU checks of continuous batching:

* sg_run_group (the shared launch of the serving loop) against the oracle
  bit for bit, with handles joining at different launches and runs split
  into short launches;
* the serving loop over the whole range of the mixed workload (n from 10^3 to
  10^6, 2-D/3-D +-J lattices, Chimera with hyper-couplings, 3-regular),
  including a 10^6-spin lattice and a 10^6-spin 3-regular request, under a
  tight HBM budget: every result equals the same request run alone
  (tolerance zero) and the CPU oracle;
* admission: oversized requests are rejected and a waiting request is
  cancelled deterministically.
"""
import numpy as np
import pytest

import instances as gen
import oracle
from parity import compare, log

pytestmark = pytest.mark.gpu

GREEDY, TIE = 0, 1


def _alone(inst, seed, rule=GREEDY, max_sweeps=10000, until_converged=True):
    import paper_0912_3912_amd as sg
    h = sg.load_instance([inst]).bind()
    h.init_spins(seed)
    st = h.run_sweeps(seed=seed, rule=rule, max_sweeps=max_sweeps, until_converged=until_converged)
    E, r = h.best()
    s = h.spins_out(0, int(r[0]))
    h.free()
    return int(E[0]), int(r[0]), s, st


def _bound(insts, stream):
    import paper_0912_3912_amd as sg
    hs = []
    for inst in insts:
        h = sg.load_instance([inst])
        h.bind(stream=stream)
        hs.append(h)
    return hs


def _group_instances():
    return [gen.chimera(8, 8, seed=2, instance_id=1, restarts=3),
            gen.erdos_renyi_triples(2000, seed=3).replace(instance_id=2, restarts=2),
            gen.lattice((64, 64), seed=4, instance_id=3),
            gen.random_regular3(20000, seed=5, instance_id=4),
            gen.lattice((24, 24, 24), seed=6, instance_id=5, h_range=(-2, 2))]


def test_run_group_joins_and_splits_until_converged(gpu):
    """GREEDY until converged in 3-sweep shared launches: the first two
    handles run two launches alone, then the rest join; handles leave as
    they converge.  Every replica equals the oracle's uninterrupted run."""
    import torch

    import paper_0912_3912_amd as sg
    insts = _group_instances()
    stream = torch.cuda.Stream()
    hs = _bound(insts, stream)
    seed = 9
    for h in hs:
        h.init_spins(seed)
    scratch = torch.empty(sg.group_scratch_bytes(hs), dtype=torch.uint8, device=gpu)
    active = [0, 1]
    launches = 0
    for step in range(400):
        if step == 2:
            active += [2, 3, 4]
        group = [hs[k] for k in active]
        st, unc = sg.run_group(group, scratch, seed=seed, rule=GREEDY, max_sweeps=3, until_converged=True)
        assert st["schedule_used"] == sg.SCHED_QUEUE
        launches += 1
        active = [k for k, u in zip(active, unc) if u > 0]
        if not active and step >= 2:
            break
    log(f"run_group GREEDY: {launches} launches")
    assert not active
    for inst, h in zip(insts, hs):
        ref, _ = oracle.run(inst, seed=seed, rule=GREEDY, max_sweeps=100000, until_converged=True)
        compare(h, [inst], [ref])
        h.free()


def test_run_group_tie_fixed_budget(gpu):
    """GREEDY_TIE (its tie draws key on the absolute sweep count) for fixed
    budgets split into 3-sweep shared launches, handles joining late."""
    import torch

    import paper_0912_3912_amd as sg
    insts = _group_instances()
    stream = torch.cuda.Stream()
    hs = _bound(insts, stream)
    seed = 5
    for h in hs:
        h.init_spins(seed)
    scratch = torch.empty(sg.group_scratch_bytes(hs), dtype=torch.uint8, device=gpu)
    done = [0] * len(hs)
    for step in range(6):
        active = [0, 1] if step < 2 else [0, 1, 2, 3, 4]
        st, _ = sg.run_group([hs[k] for k in active], scratch, seed=seed, rule=TIE, max_sweeps=3,
                             until_converged=False)
        for k in active:
            done[k] += 3
    assert done == [18, 18, 12, 12, 12]
    for inst, h, d in zip(insts, hs, done):
        ref, _ = oracle.run(inst, seed=seed, rule=TIE, max_sweeps=d, until_converged=False)
        compare(h, [inst], [ref])
        h.free()


def test_run_group_errors(gpu):
    import torch

    import paper_0912_3912_amd as sg
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = _bound([gen.chimera(2, 2, seed=1)], s1)[0]
    b = _bound([gen.chimera(2, 2, seed=2)], s2)[0]
    big = sg.load_instance([gen.random_regular3(200000, seed=1)])
    for h in (a, b):
        h.init_spins(1)
    scratch = torch.empty(1 << 20, dtype=torch.uint8, device=gpu)
    with pytest.raises(sg.SGError) as e:
        sg.run_group([a, b], scratch, seed=1)
    assert e.value.status == sg.SG_EINVAL and "stream" in str(e.value)
    with pytest.raises(sg.SGError) as e:
        sg.group_scratch_bytes([a, big])
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SGError) as e:
        sg.run_group([a, a], scratch, seed=1)
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SGError) as e:
        sg.run_group([a], scratch[:16], seed=1)
    assert e.value.status == sg.SG_ENOMEM
    assert big.query("queue_ok") == 0 and a.query("queue_ok") == 1
    for h in (a, b, big):
        h.free()


def _full_range_requests():
    reqs, gaps = gen.cfg5_trace(count=24, seed=5, n_lo=1e3, n_hi=1e6)
    insts = [gen.serving_instance(f, n, s, i) for (f, n, s, i) in reqs]
    # the top of the range: a 10^6-spin 3-D lattice and a 10^6-spin 3-regular graph
    insts.append(gen.serving_instance("cub3", 10**6, 101, 24))
    insts.append(gen.serving_instance("reg3", 10**6, 102, 25))
    gaps = np.concatenate([gaps, [0.5, 0.5]])
    return insts, gaps


def test_serving_full_range_equals_alone_and_oracle(gpu):
    import paper_0912_3912_amd as sg
    from paper_0912_3912_amd.serve import Request, Server
    insts, gaps = _full_range_requests()
    fams = {i.name[:3] for i in insts}
    assert max(i.n for i in insts) == 10**6 and min(i.n for i in insts) < 2000
    fps = [sg.load_instance([i]).workspace_bytes() for i in insts]
    budget = int(2.5 * max(fps))
    log(f"serving: {len(insts)} requests, n {min(i.n for i in insts)}..{max(i.n for i in insts)}, families {fams}, "
        f"budget {budget} B")
    server = Server(budget_bytes=budget, slots=2, ingest_workers=4, keep_spins=True, tick_sweeps=4)
    reqs = [Request(rid=k, instance=inst, seed=11) for k, inst in enumerate(insts)]
    # a 10^6-spin lattice under a fixed GREEDY_TIE budget (the co-resident tile launch) among the others
    tie = dict(rule=TIE, max_sweeps=200, until_converged=False)
    reqs[-2] = Request(rid=len(insts) - 2, instance=insts[-2], seed=11, **tie)
    results = server.run_trace(reqs, gaps, time_scale=0.002)
    server.close()
    assert all(r.status == "ok" for r in results), [r.status for r in results]
    assert results[-2].slot >= 0  # the fixed-budget lattice ran solo, beside the shared launches
    assert server.pool.peak <= server.pool.size
    assert max(t[2] for t in server.timeline) >= 2, "no two requests were ever resident together"
    assert server.shared_launches > 0 and max(server.shared_batch_sizes) >= 2, "no launch was shared"
    log(f"  {server.shared_launches} shared launches, up to {max(server.shared_batch_sizes)} requests each; "
        f"{sum(r.slot >= 0 for r in results)} solo requests")
    iv = sorted((r.started, r.done) for r in results)
    assert any(b[0] < a[1] for a, b in zip(iv, iv[1:]))
    for req, inst, res in zip(reqs, insts, results):
        kw = dict(rule=req.rule, max_sweeps=req.max_sweeps, until_converged=req.until_converged)
        E, r, s, st = _alone(inst, 11, **kw)
        assert (res.energy, res.best_restart) == (E, r), inst.name
        assert np.array_equal(res.spins, s), inst.name
        assert res.flips == st["flips"] and res.attempts == st["attempts"], inst.name
        ref, _ = oracle.run(inst, seed=11, threads=1, **kw)
        assert res.energy == int(ref.energy.min()), inst.name
        assert np.array_equal(res.spins, ref.spins[int(np.argmin(ref.energy))]), inst.name


def test_serving_rejects_oversized_and_cancels(gpu):
    import paper_0912_3912_amd as sg
    from paper_0912_3912_amd.serve import Request, Server
    small = gen.lattice((16, 16), seed=1, instance_id=1)
    big = gen.random_regular3(200000, seed=2, instance_id=2)
    other = gen.chimera(6, 6, seed=3, instance_id=3)
    budget = 3 * sg.load_instance([other]).workspace_bytes()
    server = Server(budget_bytes=budget, slots=1, ingest_workers=2)
    server.pause_admission()
    server.submit(Request(rid=0, instance=other, seed=1))
    server.submit(Request(rid=1, instance=big, seed=1))
    server.submit(Request(rid=2, instance=small, seed=1))
    server.wait_ingested([0, 1, 2])
    assert server.cancel(2) is True        # ingested and waiting for admission
    assert server.cancel(2) is False       # already cancelled
    server.resume_admission()
    res = server.wait([0, 1, 2])
    assert server.cancel(0) is False       # finished
    server.close()
    assert res[0].status == "ok"
    assert res[1].status == "rejected"
    assert res[2].status == "cancelled"
