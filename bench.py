"""Benchmark: spin-flip attempts per second of colour-ordered single-spin-flip
descent on one MI355X, the roofline position of the dominant kernel, the
plain per-phase method on the same GPU, and the CPU oracle timed beside it.

Workloads (--workload):
  cubic100     (default) 10^6-spin periodic 100^3 +-J lattice, h in {-2..2},
               checkerboard, one random start, GREEDY_TIE for exactly 1000
               sweeps (10^9 attempts).  Step = random start + start energy +
               1000 sweeps + best-of-restarts, all on the GPU, couplings
               already resident in HBM.
  square16     16x16 periodic +-J lattice, h = 0, 64 starts, GREEDY until
               converged; step = one sg_solve call (starts, sweeps, exact
               energies and best restart in one launch).
  chimera4096  4096 Chimera-like 8x8-cell instances with hyper-couplings,
               256 restarts each, GREEDY until converged, one batched launch.
  chimera4096_fm  the same batch under the paper's pass-based search
               (max-gain moves with locking and hill-climbing, best prefix
               kept, passes until no improvement); value = moves/s.
  square1000_fm  one pass of that search on each of 512 restarts of a
               1000x1000 +-J lattice (10^6 spins, beyond one wavefront's LDS:
               the large-instance pass kernel, fm_slots = 512); value = moves/s.
  er2000       2000 Erdos-Renyi instances, n log-uniform in [100, 1e5], mean
               degree 6, n/2 triples, GREEDY until converged, one launch.
  factoring    Sec. VI: random starts of the factoring hypergraphs of
               612171 and 580003 (pass-based search to convergence, one lane
               per start); success probability per start and starts/s.
  serving      Poisson arrivals of mixed requests (2-D/3-D +-J lattices,
               Chimera with hyper-couplings, 3-regular), n log-uniform in
               [1e3, 1e6], admitted by HBM footprint into a device pool,
               rate 0.7 x the measured capacity; p50/p99 latency, flips/s.
The default run measures the headline lattice and then every other workload
of the configuration list as a leg of the same JSON line: ``square16`` (the
small lattice, microseconds per solve), ``batched`` (the Chimera batch against
per-instance per-phase launches), ``uneven`` (the 2000 uneven instances
against the per-phase method on every instance), ``serving`` and ``fm`` (the
Chimera batch under the pass-based search).  Every leg
carries the roofline position of its dominant kernel and the CPU oracle timed
on a stated sample (``cpu_baseline``).

Prints one JSON line.  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
# Plain (non-packed) int32 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.3 T lane-ops/s (the published 157.3 TFLOP/s fp32 vector figure
# counts an FMA as two operations and packed fp32 as two lanes).
PEAK_INT_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

GREEDY, TIE = 0, 1
SCHED_AUTO, SCHED_PHASE = -1, 0
KERNEL_NAME = {0: "k_phase", 3: "k_lattice_tiles", 4: "k_block", 5: "k_queue"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Per-attempt HBM bytes of the 3-D lattice sweep in two reference formats:
# CSR with 4-byte row pointers and column indices and 1-byte couplings
# (4 + 6 (4 + 1) + 1 (h) + 2 (own spin read and written) + 1 (other colours'
# spins) = 38 B), and the compact lattice form with implicit indices and
# 1-byte couplings (6 + 1 + 2 + 1 = 10 B).
CSR_BYTES_PER_ATTEMPT = 38.0
COMPACT_BYTES_PER_ATTEMPT = 10.0


def int_ops_per_attempt(deg: float, tau: float = 0.0) -> float:
    """Algorithmic integer operations of one attempt: a multiply and an add
    per coupling, two multiplies and an add per hyper-coupling, the field
    add, dE = 2 s f (two multiplies) and the decision compare."""
    return 2.0 * deg + 3.0 * tau + 1 + 2 + 1


def sell_bytes_per_attempt(deg: float, tau: float = 0.0, spins_in_lds: bool = False) -> float:
    """Algorithmic HBM bytes of one attempt in the sliced coupling layout:
    deg 4-byte coupling words, 2 tau 4-byte hyper-coupling words, the 1-byte
    field, and (spins in memory) the own spin read and written plus one byte
    of the other colours' spins (read once per phase, cache-reuse bound)."""
    b = 4.0 * deg + 8.0 * tau + 1
    if not spins_in_lds:
        b += 2 + 1
    return b


def sources_sha256(paths) -> str:
    """sha256 over the concatenated bytes of the given repository files."""
    import hashlib
    d = hashlib.sha256()
    for p in paths:
        d.update(open(os.path.join(ROOT, p), "rb").read())
    return d.hexdigest()


def measured_traffic(kernel: str, geometry=None):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs (scaled by a plain-copy calibration), or None when a source of the
    kernel has changed since the counters were taken, or when the record names
    a launch geometry (tiling, halo width) other than this run's."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    srcs = rec.get("sources") or [rec["source"]]
    if not all(os.path.exists(os.path.join(ROOT, p)) for p in srcs) or sources_sha256(srcs) != rec["sha256"]:
        return None
    if rec.get("geometry") is not None and rec["geometry"] != geometry:
        return None
    return rec["bytes_per_launch"]


def host_cores() -> int:
    """Host threads the CPU baselines use: the CPUs this process may run on,
    capped by OMP_NUM_THREADS and at 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, min(n, 16))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_parallel(jobs, cores):
    """Run oracle calls (callables) on `cores` host threads; the oracle's C
    functions run without the interpreter lock."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=cores) as ex:
        return list(ex.map(lambda f: f(), jobs))


def timed(fn, steps, warmup, sync):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    outs = [fn() for _ in range(steps)]
    sync()
    return (time.perf_counter() - t0) / steps, outs


def run_cubic(args, sg, gen, torch):
    L = args.L
    inst = gen.cfg2_cubic100(L=L)
    n = inst.n
    h = sg.load_instance([inst], lattice_dims=[(L, L, L)]).bind()
    ws_mb = h.workspace_bytes() / 1e6
    log(f"cubic{L}: n={n} m={inst.m} workspace={ws_mb:.1f} MB sweeps={args.sweeps}")

    def step(schedule=args.schedule):
        h.init_spins(args.seed)
        st = h.run_sweeps(seed=args.seed, rule=TIE, max_sweeps=args.sweeps, until_converged=False,
                          schedule=schedule)
        h.best()
        st["hot_ns"] = h.query("hot_ns")
        st["hot_launches"] = h.query("hot_launches")
        return st

    dt, outs = timed(step, args.steps, args.warmup, torch.cuda.synchronize)
    attempts = n * args.sweeps
    assert all(o["attempts"] == attempts for o in outs)
    value = attempts / dt
    sched = outs[-1]["schedule_used"]
    hot_us = sum(o["hot_ns"] for o in outs) / len(outs) / 1e3
    launches = outs[-1]["hot_launches"]
    E = int(h.energy()[0])
    log(f"timed {args.steps} steps: {dt * 1e3:.3f} ms/step, hot kernel {hot_us:.1f} us over {launches} launch(es), "
        f"schedule {sched}, E={E}")

    # the plain method: one launch per colour phase, same workload, same GPU
    plain_ms = None
    if not args.no_plain:
        plain_ms, _ = timed(lambda: step(SCHED_PHASE), 1, 1, torch.cuda.synchronize)
        plain_ms *= 1e3
        log(f"plain per-phase method: {plain_ms:.3f} ms/step")

    launches = max(launches, 1)
    per_launch_s = hot_us / 1e6 / launches
    apl = attempts // launches
    kname = KERNEL_NAME.get(sched, str(sched))
    if sched == 3 and h.query("last_msc"):
        kname = "k_lattice_msc"
    geometry = {"tiles": h.query("last_tiles"), "halo_k": h.query("last_tile_k")}
    traffic = measured_traffic(kname, geometry) if sched == 3 else None
    # The compact-lattice model (implicit neighbours, int8 couplings and
    # field) for the tile kernels, the sliced-layout model otherwise.
    bpa = COMPACT_BYTES_PER_ATTEMPT if sched == 3 else sell_bytes_per_attempt(6)
    ach = bpa * apl / per_launch_s / 1e9
    ops = int_ops_per_attempt(6)
    alu = ops * apl / per_launch_s / 1e12
    roofline = {
        "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": kname,
        "model": ("compact lattice: 10 B per attempt (six int8 couplings, int8 field, own spin read and written, "
                  "the other colour's spins once)") if sched == 3 else
                 "sliced coupling layout: 4 B per coupling word, int8 field, own spin read and written, neighbours once",
        "bytes_per_attempt": bpa, "attempts_per_launch": apl, "launches_per_step": launches,
        "avg_launch_us": round(hot_us / launches, 2),
        "traffic_source": None if traffic is None else (
            "profiles/traffic.json: rocprofv3 FETCH_SIZE and WRITE_SIZE of this kernel at this tiling, scaled by a "
            "plain-copy calibration, taken by a profiled run of this command (not in this run); it is dropped "
            "(null) as soon as a source of the kernel changes"),
        "counter_GBps": None if traffic is None else round(traffic / per_launch_s / 1e9, 1),
        "counter_frac": None if traffic is None else round(traffic / per_launch_s / 1e9 / PEAK_HBM_GBS, 4),
        "csr_model": {"bytes_per_attempt": CSR_BYTES_PER_ATTEMPT,
                      "frac": round(CSR_BYTES_PER_ATTEMPT * apl / per_launch_s / 1e9 / PEAK_HBM_GBS, 4),
                      "note": "the CSR stream model (row pointers, column indices and values per coupling); this kernel streams no CSR structure, so it is not "
                              "a bandwidth figure"},
        "alu": {"ops_per_attempt": ops, "achieved_TOPs": round(alu, 3), "peak_TOPs": round(PEAK_INT_TOPS, 2),
                "frac": round(alu / PEAK_INT_TOPS, 4),
                "note": "algorithmic integer operations; the bit-plane kernel decides 32 sites per word operation"},
    }
    if kname == "k_lattice_msc":
        ph_us = h.query("last_model_phase_ns") / 1e3
        ex_us = h.query("last_model_exchange_ns") / 1e3
        nph, nex = h.query("last_model_phases"), h.query("last_model_exchanges")
        pred = ph_us * nph + ex_us * nex
        roofline["limiter"] = "latency"
        roofline["latency_model"] = {
            "phase_us": round(ph_us, 3), "exchange_us": round(ex_us, 3), "phases": nph, "exchanges": nex,
            "predicted_us": round(pred, 1), "measured_us": round(hot_us / launches, 1),
            "note": "the launch is a dependent chain of colour phases (LDS loads, decision, tie draws, barrier) "
                    "and halo exchanges between tiles; the tiling's fitted cost model predicts its time"}
    cpu = None
    if args.cpu_sweeps > 0:
        import oracle
        t1 = time.perf_counter()
        oracle.run(inst, seed=args.seed, rule=oracle.GREEDY_TIE, max_sweeps=args.cpu_sweeps, until_converged=False,
                   threads=1)
        ct = time.perf_counter() - t1
        cpu = {"value": n * args.cpu_sweeps / ct, "unit": "attempts/s", "cores": 1, "kind": "oracle",
               "sample": f"cubic{L}, 1 start, {args.cpu_sweeps} of the step's {args.sweeps} GREEDY_TIE sweeps "
                         f"({n * args.cpu_sweeps:.3g} attempts in {ct:.1f} s, one replica so one core)"}
        log(f"cpu oracle: {cpu['value']:.3e} attempts/s over {ct:.1f} s")
    out = {
        "metric": "spin-flip attempts/s (10^6-spin 3-D +-J lattice, 1000 sweeps)",
        "value": value, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8 spins/couplings, int32 fields, int64 energy", "data": "synthetic",
        "config": {"workload": f"cubic{L}_pmJ_h2_tie_{args.sweeps}sweeps", "n_spins": n, "bonds": inst.m,
                   "sweeps": args.sweeps, "restarts": 1, "rule": "GREEDY_TIE", "schedule": sched,
                   "tiles": h.query("last_tiles"), "halo_k": h.query("last_tile_k"), "energy": E,
                   "workspace_mb": round(ws_mb, 1)},
        "plain_method": None if plain_ms is None else {
            "ms_per_step": round(plain_ms, 3), "attempts_per_s": attempts / plain_ms * 1e3,
            "speedup": round(plain_ms / (dt * 1e3), 3)},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    h.free()
    return out


def run_chimera(args, sg, gen, torch, count=4096, sample=16):
    insts = gen.cfg3_chimera_batch(count=count, restarts=256)
    t0 = time.perf_counter()
    h = sg.load_instance(insts).bind()
    log(f"chimera{count}x256: ingest {time.perf_counter() - t0:.1f} s, workspace {h.workspace_bytes() / 1e6:.0f} MB")
    n = insts[0].n
    deg = 2 * insts[0].m / n
    tau = 3 * insts[0].t / n

    def step(schedule=SCHED_AUTO, hh=h):
        hh.init_spins(args.seed)
        st = hh.run_sweeps(seed=args.seed, rule=GREEDY, max_sweeps=10000, until_converged=True, schedule=schedule)
        hh.best()
        st["hot_ns"] = hh.query("hot_ns")
        st["hot_launches"] = hh.query("hot_launches")
        return st

    dt, outs = timed(step, args.batch_steps, 1, torch.cuda.synchronize)
    st = outs[-1]
    attempts = st["attempts"]
    hot_us = st["hot_ns"] / 1e3
    kname = "k_block_bits" if h.query("last_bits") else "k_block"
    log(f"batched: {dt * 1e3:.2f} ms/step, {attempts:.3g} attempts, sweeps_max {st['sweeps_max']}, "
        f"schedule {st['schedule_used']}, hot {hot_us:.0f} us")
    h.free()
    extrap = None
    if not args.no_plain:
        # per-instance baseline: the plain per-phase method on a sample, one instance at a time
        hs = sg.load_instance(insts[:sample]).bind()
        dts, outs_s = timed(lambda: step(SCHED_PHASE, hs), 1, 1, torch.cuda.synchronize)
        extrap = dts * count / sample
        log(f"per-instance per-phase: {dts * 1e3:.1f} ms for {sample} instances -> {extrap * 1e3:.0f} ms "
            "extrapolated")
        hs.free()
    ops = int_ops_per_attempt(deg, tau)
    ach = ops * attempts / (hot_us / 1e6) / 1e12
    cpu = None
    if args.cpu_sweeps > 0:
        import oracle
        cores = host_cores()
        cpu_sample = insts[:min(args.cpu_chimera, count)]
        t1 = time.perf_counter()
        catt = 0
        for inst in cpu_sample:
            sto, _ = oracle.run(inst, seed=args.seed, rule=oracle.GREEDY, max_sweeps=10000, until_converged=True,
                                threads=cores)
            catt += int(sto.sweeps.sum()) * inst.n
        ct = time.perf_counter() - t1
        cpu = {"value": catt / ct, "unit": "attempts/s", "cores": cores, "kind": "oracle",
               "sample": f"instances 0..{len(cpu_sample) - 1} of the {count}, all 256 restarts each, GREEDY until "
                         f"converged ({catt:.3g} attempts in {ct:.1f} s; restarts spread over {cores} threads of "
                         f"{cpu_model()}, nproc {os.cpu_count()})"}
        log(f"chimera cpu oracle: {cpu['value']:.3e} attempts/s on {cores} threads")
    return {"workload": f"chimera{count}x256_greedy", "attempts_per_s": attempts / dt, "ms_per_step": dt * 1e3,
            "attempts": attempts, "schedule": st["schedule_used"],
            "per_instance_ms": None if extrap is None else round(extrap * 1e3, 2), "per_instance_sample": sample,
            "per_instance_extrapolated": True, "speedup": None if extrap is None else round(extrap / dt, 2),
            "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": round(PEAK_INT_TOPS, 2),
                         "unit": "TOP/s", "frac": round(ach / PEAK_INT_TOPS, 4), "kernel": kname,
                         "ops_per_attempt": round(ops, 2),
                         "note": "instance and restarts stay in LDS, so HBM carries only the structure and the "
                                 "spins read out; algorithmic integer operations against the int32 VALU issue rate"},
            "cpu_baseline": cpu}


def fm_ops_per_move(n: float, deg: float, tau: float) -> float:
    """Algorithmic integer operations of one move of the pass-based search: a
    gain update per coupling partner (4 s_j J s_i, three multiplies and an
    add), two per hyper-coupling incidence, and the log2(n) comparisons of a
    heap selection (the paper's gain container)."""
    import math
    return 4.0 * deg + 8.0 * tau + math.log2(max(n, 2.0))


def run_chimera_fm(args, sg, gen, torch, count=4096):
    """The paper's pass-based search (max-gain moves, locking, hill-climbing)
    on every replica of the Chimera batch, one launch, until no pass improves."""
    insts = gen.cfg3_chimera_batch(count=count, restarts=256)
    h = sg.load_instance(insts).bind()
    n = insts[0].n
    deg = 2 * insts[0].m / n
    tau = 3 * insts[0].t / n

    def step():
        h.init_spins(args.seed)
        st = h.run_sweeps(seed=args.seed, rule=sg.FM, max_sweeps=10000, until_converged=True)
        h.best()
        st["hot_ns"] = h.query("hot_ns")
        return st

    dt, outs = timed(step, args.batch_steps, 1, torch.cuda.synchronize)
    st = outs[-1]
    moves = st["attempts"]
    hot_us = st["hot_ns"] / 1e3
    Eb, _ = h.best()
    lanes = h.query("last_fm_lanes")
    kname = "k_fm_lanes" if lanes else "k_fm"
    log(f"fm: {dt * 1e3:.2f} ms/step, {moves:.3g} moves, passes max {st['sweeps_max']}, hot {hot_us:.0f} us "
        f"({kname}), mean best energy {float(Eb.mean()):.1f}")
    h.free()
    ops = fm_ops_per_move(n, deg, tau)
    ach = ops * moves / (hot_us / 1e6) / 1e12
    cpu = None
    if args.cpu_sweeps > 0:
        import oracle
        sample = insts[:32]  # 32 instances x all 256 restarts
        t1 = time.perf_counter()
        cmoves = 0
        cores = host_cores()
        for inst in sample:
            sst, _ = oracle.fm(inst, seed=args.seed, threads=cores)
            cmoves += int(sst.sweeps.sum()) * inst.n
        ct = time.perf_counter() - t1
        cpu = {"value": cmoves / ct, "unit": "moves/s", "cores": cores, "kind": "oracle",
               "sample": f"32 instances x 256 restarts of the batch ({cmoves:.3g} moves in {ct:.1f} s; the oracle "
                         f"evaluates every unlocked gain from the definition at each move)"}
    return {"workload": f"chimera{count}x256_fm", "attempts_per_s": moves / dt, "ms_per_step": dt * 1e3,
            "attempts": moves, "schedule": st["schedule_used"], "passes_max": st["sweeps_max"],
            "moves_kept": st["flips"], "mean_best_energy": float(Eb.mean()),
            "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": round(PEAK_INT_TOPS, 2),
                         "unit": "TOP/s", "frac": round(ach / PEAK_INT_TOPS, 4), "kernel": kname,
                         "avg_launch_us": round(hot_us, 1), "ops_per_attempt": round(ops, 2),
                         "attempt": "one move of a pass",
                         "note": "one replica per lane: each move is a serial chain of LDS round trips and "
                                 "one row load; the lane kernel issues about 600 instructions per wavefront "
                                 "step, so the algorithmic integer rate stays a small fraction of the VALU peak"},
            "cpu_baseline": cpu}


def run_square_fm(args, sg, gen, torch, L=1000, restarts=512):
    """One pass of the pass-based search on every restart of a 10^6-spin 2-D
    lattice: instances beyond one wavefront's LDS run on the large-instance
    pass kernel, one replica per slot (fm_slots = restarts)."""
    inst = gen.lattice((L, L), seed=2).replace(restarts=restarts)
    h = sg.load_instance([inst])
    h.tune("fm_slots", restarts)
    h.bind()
    log(f"square{L}_fm: workspace {h.workspace_bytes() / 1e9:.2f} GB")
    h.init_spins(args.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = h.run_sweeps(seed=args.seed, rule=sg.FM, max_sweeps=1, until_converged=False)
    dt = time.perf_counter() - t0
    hot_us = h.query("hot_ns") / 1e3
    big = h.query("last_fm_big")
    h.free()
    log(f"square{L}_fm: one pass of {restarts} restarts in {dt:.3f} s (hot {hot_us / 1e3:.1f} ms), "
        f"{st['attempts'] / dt:.3g} moves/s")
    return {"workload": f"square{L}_fm_{restarts}restarts_1pass", "metric": "moves/s", "unit": "moves/s",
            "attempts_per_s": st["attempts"] / dt, "ms_per_step": dt * 1e3, "attempts": st["attempts"],
            "replicas_on_large_kernel": big, "avg_launch_us": round(hot_us, 1),
            "us_per_move_per_replica": round(dt / (st["attempts"] / restarts) * 1e6, 3), "cpu_baseline": None}


def run_factoring(args, sg, gen, torch, copies=16, restarts=65535):
    """Sec. VI factoring experiments: every random start of the factoring
    hypergraph runs the pass-based search to convergence; a start succeeds
    when it ends at energy -c0 (a factorisation; with bit_length(N)//2 free
    bits per factor both factors are below N, so it is non-trivial)."""
    from paper_0912_3912_amd.factoring import factoring_instance
    out = {"workload": "factoring_fm", "cases": []}
    total_starts, total_s = 0, 0.0
    for N, paper_p in ((612171, 0.025), (580003, 0.005)):
        b = N.bit_length() // 2
        ds = [factoring_instance(N, b, b, instance_id=k, restarts=restarts) for k in range(copies)]
        h = sg.load_dense(ds).bind()

        def step():
            h.init_spins(args.seed)
            return h.run_sweeps(seed=args.seed, rule=sg.FM, max_sweeps=1000, until_converged=True)

        dt, outs = timed(step, args.batch_steps, 1, torch.cuda.synchronize)
        E = h.energy()
        starts = len(E)
        p = float((E == ds[0].ground_energy()).mean())
        Eb, rb = h.best()
        k = int(np.argmin(Eb))
        x, y = ds[k].decode(h.spins_out(k, int(rb[k])))
        log(f"factor {N}: {starts} starts in {dt * 1e3:.1f} ms, P(success per start) = {p:.4f} "
            f"(paper {paper_p}), best x*y = {x}*{y} = {x * y}, passes max {outs[-1]['sweeps_max']}")
        h.free()
        case = {"N": N, "free_bits": [b, b], "spins": 2 * b, "terms": int(len(ds[0].coefs)), "starts": starts,
                "ms": round(dt * 1e3, 2), "starts_per_s": starts / dt, "p_success_per_start": p,
                "paper_p_success": paper_p, "best_factors": [int(x), int(y)], "moves": outs[-1]["attempts"]}
        if args.cpu_sweeps > 0:
            import oracle
            sample = ds[0].replace(restarts=400)
            t1 = time.perf_counter()
            st, _ = oracle.dense_fm(sample, seed=args.seed)
            ct = time.perf_counter() - t1
            case["cpu_baseline"] = {"value": 400 / ct, "unit": "starts/s", "cores": 1, "kind": "oracle",
                                    "sample": f"400 starts of instance 0 ({ct:.1f} s)",
                                    "p_success_sample": float((st.energy == ds[0].ground_energy()).mean())}
        out["cases"].append(case)
        total_starts += starts
        total_s += dt
    out["attempts_per_s"] = total_starts / total_s
    out["ms_per_step"] = total_s * 1e3
    out["metric"] = "random starts searched to convergence per second (factoring 612171 and 580003)"
    out["unit"] = "starts/s"
    return out


def run_er(args, sg, gen, torch, count=2000):
    t0 = time.perf_counter()
    insts = gen.cfg4_uneven_batch(count=count)
    log(f"er{count}: generated in {time.perf_counter() - t0:.1f} s, sum n = {sum(i.n for i in insts)}")
    t0 = time.perf_counter()
    h = sg.load_instance(insts).bind()
    log(f"er{count}: ingest {time.perf_counter() - t0:.1f} s, workspace {h.workspace_bytes() / 1e6:.0f} MB")

    from paper_0912_3912_amd import autotune
    tune = autotune.autotune(h, seed=args.seed, rule=GREEDY, max_sweeps=10000, until_converged=True)
    log(f"er{count}: autotuned {tune['setting']} in {tune['calibration_ms']:.0f} ms "
        f"({len(tune['measured'])} candidates: " + ", ".join(f"{m['setting']} {m['ms']:.2f} ms" for m in tune["measured"])
        + ")")

    def step(schedule=SCHED_AUTO):
        h.init_spins(args.seed)
        st = h.run_sweeps(seed=args.seed, rule=GREEDY, max_sweeps=10000, until_converged=True, schedule=schedule)
        h.best()
        st["hot_ns"] = h.query("hot_ns")
        return st

    dt, outs = timed(step, args.batch_steps, 1, torch.cuda.synchronize)
    st = outs[-1]
    attempts = st["attempts"]
    dtp = None
    if not args.no_plain:
        dtp, outp = timed(lambda: step(SCHED_PHASE), 1, 0, torch.cuda.synchronize)
        assert outp[-1]["attempts"] == attempts
    hot_us = st["hot_ns"] / 1e3
    ntot = sum(i.n for i in insts)
    deg = sum(2 * i.m for i in insts) / ntot
    tau = sum(3 * i.t for i in insts) / ntot
    # the layout's own bytes (coupling and hyper-coupling words, field; spins in LDS)
    bpa = sell_bytes_per_attempt(deg, tau, spins_in_lds=True)
    # the CSR stream model: row pointers (edges and triples), deg (4 + 1), tau (2 * 4 + 1), field, own spin
    # read and written, other spins once
    bpa_csr = 4 + 4 + deg * 5 + tau * 9 + 1 + 2 + 1
    ach = bpa * attempts / (hot_us / 1e6) / 1e9
    traffic = measured_traffic("k_queue")
    log(f"batched {dt * 1e3:.2f} ms, hot {hot_us:.0f} us"
        + ("" if dtp is None else f", per-instance per-phase {dtp * 1e3:.1f} ms, speedup {dtp / dt:.2f}"))
    h.free()
    cpu = None
    if args.cpu_sweeps > 0:
        import oracle
        cores = host_cores()
        order = sorted(range(len(insts)), key=lambda k: -insts[k].n)  # largest first balances the threads
        t1 = time.perf_counter()
        res = oracle_parallel([lambda k=k: oracle.run(insts[k], seed=args.seed, rule=oracle.GREEDY, max_sweeps=10000,
                                                      until_converged=True, threads=1)[0] for k in order], cores)
        ct = time.perf_counter() - t1
        catt = sum(int(r.sweeps.sum()) * insts[k].n for r, k in zip(res, order))
        assert catt == attempts, (catt, attempts)
        cpu = {"value": catt / ct, "unit": "attempts/s", "cores": cores, "kind": "oracle",
               "sample": f"all {count} instances, one per task on {cores} threads of {cpu_model()} (nproc "
                         f"{os.cpu_count()}), GREEDY until converged ({catt:.3g} attempts in {ct:.1f} s)"}
        log(f"er cpu oracle: {cpu['value']:.3e} attempts/s on {cores} threads")
    algo_launch = bpa * attempts
    return {"workload": f"er{count}_greedy", "attempts_per_s": attempts / dt, "ms_per_step": dt * 1e3,
            "attempts": attempts, "schedule": st["schedule_used"],
            "autotune": {"key": tune["key"], "setting": tune["setting"],
                         "calibration_ms": round(tune["calibration_ms"], 1),
                         "candidates_ms": {json.dumps(m["setting"], sort_keys=True): round(m["ms"], 3)
                                           for m in tune["measured"]}},
            "per_instance_ms": None if dtp is None else round(dtp * 1e3, 2),
            "per_instance_extrapolated": False, "speedup": None if dtp is None else round(dtp / dt, 2),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(ach / PEAK_HBM_GBS, 4), "kernel": "k_queue", "avg_launch_us": round(hot_us, 1),
                         "bytes_per_attempt": round(bpa, 2),
                         "model": "the sliced layout's own stream: 4 B per coupling word, 8 B per hyper-coupling "
                                  "incidence, 1 B field (spins in LDS)",
                         "csr_model": {"bytes_per_attempt": round(bpa_csr, 2),
                                          "frac": round(bpa_csr * attempts / (hot_us / 1e6) / 1e9 / PEAK_HBM_GBS, 4)},
                         "traffic": traffic,
                         "traffic_source": None if traffic is None else (
                             "profiles/traffic.json: rocprofv3 FETCH_SIZE and WRITE_SIZE of this kernel on this "
                             "workload, copy-calibrated, taken by a profiled run (not in this run)"),
                         "traffic_over_model": None if traffic is None else round(traffic / algo_launch, 3),
                         "counter_frac": None if traffic is None else round(
                             traffic / (hot_us / 1e6) / 1e9 / PEAK_HBM_GBS, 4)},
            "cpu_baseline": cpu}


def run_square(args, sg, gen, torch):
    inst = gen.cfg1_square16()
    h = sg.load_instance([inst], lattice_dims=[(16, 16)]).bind()

    def step(schedule=SCHED_AUTO):
        # the whole solve in one library call: random starts, sweeps until
        # converged, exact energies, best restart
        st, _, _ = h.solve(args.seed, rule=GREEDY, max_sweeps=10000, until_converged=True, schedule=schedule)
        return st

    def step_calls():
        h.init_spins(args.seed)
        st = h.run_sweeps(seed=args.seed, rule=GREEDY, max_sweeps=10000, until_converged=True)
        h.best()
        return st

    def step_hot():
        st = step()
        st["hot_ns"] = h.query("hot_ns")
        st["hot_launches"] = h.query("hot_launches")
        return st

    dt, outs = timed(step_hot, max(args.steps, 20), args.warmup, torch.cuda.synchronize)
    dtc, _ = timed(step_calls, max(args.steps, 20), args.warmup, torch.cuda.synchronize)
    dtp, _ = timed(lambda: step(SCHED_PHASE), 5, 1, torch.cuda.synchronize)
    st = outs[-1]
    hot_us = sum(o["hot_ns"] for o in outs) / len(outs) / 1e3
    h.free()
    ops = int_ops_per_attempt(4)
    ach = ops * st["attempts"] / (hot_us / 1e6) / 1e12
    cpu = None
    if args.cpu_sweeps > 0:
        import oracle
        reps, catt = 0, 0
        t1 = time.perf_counter()
        while True:
            sto, _ = oracle.run(inst, seed=args.seed, rule=oracle.GREEDY, max_sweeps=10000, until_converged=True,
                                threads=1)
            catt += int(sto.sweeps.sum()) * inst.n
            reps += 1
            if time.perf_counter() - t1 > 1.0:
                break
        ct = time.perf_counter() - t1
        cpu = {"value": catt / ct, "unit": "attempts/s", "cores": 1, "kind": "oracle",
               "us_per_solve": ct / reps * 1e6,
               "sample": f"the whole 64-start solve, repeated {reps} times on one core ({catt:.3g} attempts in "
                         f"{ct:.2f} s)"}
    return {"workload": "square16_64starts_greedy", "attempts_per_s": st["attempts"] / dt,
            "us_per_solve": dt * 1e6, "ms_per_step": dt * 1e3, "attempts": st["attempts"],
            "schedule": st["schedule_used"], "launches_per_solve": outs[-1]["hot_launches"],
            "three_calls_us_per_solve": dtc * 1e6, "per_phase_us_per_solve": dtp * 1e6,
            "speedup": round(dtp / dt, 2),
            "roofline": {"bound": "alu", "achieved": round(ach, 4), "peak": round(PEAK_INT_TOPS, 2), "unit": "TOP/s",
                         "frac": round(ach / PEAK_INT_TOPS, 5), "kernel": "k_lattice_wg (solve: start, sweeps, "
                                                                        "energies and best restart in one launch)",
                         "avg_launch_us": round(hot_us, 2), "ops_per_attempt": ops, "limiter": "latency",
                         "note": "256 spins x 64 starts occupy a handful of workgroups: the solve is bound by launch "
                                 "and phase latency, not by any throughput roof"},
            "cpu_baseline": cpu}


def run_serving(args, sg, gen, torch):
    from paper_0912_3912_amd.serve import Request, Server, summarize
    count = args.serving_requests
    t0 = time.perf_counter()
    reqs, gaps = gen.cfg5_trace(count=count)
    insts = [gen.serving_instance(f, n, s, i) for (f, n, s, i) in reqs]
    log(f"serving: {count} requests generated in {time.perf_counter() - t0:.1f} s, "
        f"sum n = {sum(i.n for i in insts)}")
    budget = args.serving_budget_mb << 20
    server = Server(budget_bytes=budget, slots=args.serving_slots, ingest_workers=args.serving_ingest)
    # capacity: the first requests submitted at once, back to back, after an
    # untimed burst of the next ones (first launches of every kernel, host pools)
    ncal = min(40, count)
    nwarm = min(8, max(0, count - ncal))
    warm = [Request(rid=3_000_000 + k, instance=insts[ncal + k], seed=args.seed) for k in range(nwarm)]
    server.run_trace(warm, [0.0] * nwarm)
    l0, b0 = server.shared_launches, len(server.shared_batch_sizes)
    cal = [Request(rid=1_000_000 + k, instance=insts[k], seed=args.seed) for k in range(ncal)]
    t1 = time.perf_counter()
    server.run_trace(cal, [0.0] * ncal)
    cap = ncal / (time.perf_counter() - t1)
    server.close()
    bs = server.shared_batch_sizes[b0:]
    burst = {"requests": ncal, "warmup_requests": nwarm, "shared_launches": server.shared_launches - l0,
             "max_requests_per_shared_launch": max(bs, default=0),
             "mean_requests_per_shared_launch": float(np.mean(bs)) if bs else 0.0}
    del server
    # the same burst with every request on its own handle and stream (no shared launches)
    solo = Server(budget_bytes=budget, slots=args.serving_slots, ingest_workers=args.serving_ingest, shared=False)
    warm = [Request(rid=4_000_000 + k, instance=insts[ncal + k], seed=args.seed) for k in range(nwarm)]
    solo.run_trace(warm, [0.0] * nwarm)
    cal = [Request(rid=2_000_000 + k, instance=insts[k], seed=args.seed) for k in range(ncal)]
    t1 = time.perf_counter()
    solo.run_trace(cal, [0.0] * ncal)
    cap_solo = ncal / (time.perf_counter() - t1)
    solo.close()
    del solo
    lam = 0.7 * cap
    log(f"capacity {cap:.1f} req/s (every request solo: {cap_solo:.1f} req/s) -> arrival rate {lam:.1f} req/s")
    server2 = Server(budget_bytes=budget, slots=args.serving_slots, ingest_workers=args.serving_ingest)
    requests = [Request(rid=k, instance=inst, seed=args.seed) for k, inst in enumerate(insts)]
    t2 = time.perf_counter()
    results = server2.run_trace(requests, gaps, time_scale=1.0 / lam)
    wall = time.perf_counter() - t2
    server2.close()
    summ = summarize(results, wall)
    summ.update({"capacity_req_per_s": cap, "capacity_all_solo_req_per_s": cap_solo, "burst": burst,
                 "arrival_rate_req_per_s": lam, "budget_bytes": budget,
                 "slots": args.serving_slots, "peak_resident_bytes": server2.pool.peak,
                 "max_resident_requests": max(t[2] for t in server2.timeline),
                 "shared_launches": server2.shared_launches,
                 "max_requests_per_shared_launch": max(server2.shared_batch_sizes, default=0),
                 "mean_requests_per_shared_launch": float(np.mean(server2.shared_batch_sizes))
                 if server2.shared_batch_sizes else 0.0})
    log(f"serving: p50 {summ['p50_ms']:.1f} ms, p99 {summ['p99_ms']:.1f} ms (ingest p50 {summ['ingest_p50_ms']:.1f} "
        f"p99 {summ['ingest_p99_ms']:.1f}, waiting p99 {summ['admission_wait_p99_ms']:.1f}, device p50 "
        f"{summ['device_p50_ms']:.1f} p99 {summ['device_p99_ms']:.1f} ms), {summ['flips_per_s']:.3g} flips/s, "
        f"{summ['shared_launches']} shared launches of up to {summ['max_requests_per_shared_launch']} requests")
    summ["workload"] = f"serving{count}_mixed_greedy"
    summ["ms_per_step"] = wall * 1e3
    # algorithmic bytes of the sliced layout per attempt, request by request
    tot_b = 0.0
    for inst, r in zip(insts, results):
        if r.status in ("ok", "notconv"):
            n = inst.n
            tot_b += sell_bytes_per_attempt(2 * inst.m / n, 3 * inst.t / n) * r.attempts
    gbps = tot_b / wall / 1e9
    summ["roofline"] = {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbps / PEAK_HBM_GBS, 5), "kernel": "mixed (per-request schedules)",
                        "model": "sliced layout per request: 4 B per coupling word, 8 B per hyper-coupling "
                                 "incidence, field, own spin read and written, neighbours once",
                        "note": "over the whole trace's wall time, including the gaps between Poisson arrivals "
                                "(the offered load is 0.7 of capacity)"}
    if args.cpu_sweeps > 0:
        import oracle
        cores = host_cores()
        order = sorted(range(len(insts)), key=lambda k: -insts[k].n)
        t1 = time.perf_counter()
        res = oracle_parallel([lambda k=k: oracle.run(insts[k], seed=args.seed, rule=oracle.GREEDY, max_sweeps=10000,
                                                      until_converged=True, threads=1)[0] for k in order], cores)
        ct = time.perf_counter() - t1
        catt = sum(int(r.sweeps.sum()) * insts[k].n for r, k in zip(res, order))
        gpu_att = sum(r.attempts for r in results if r.status in ("ok", "notconv"))
        summ["cpu_baseline"] = {
            "value": catt / ct, "unit": "attempts/s", "cores": cores, "kind": "oracle",
            "requests_per_s": len(insts) / ct, "same_attempts_as_gpu": catt == gpu_att,
            "sample": f"the same {count} requests replayed back to back, one per task on {cores} threads of "
                      f"{cpu_model()} (nproc {os.cpu_count()}), throughput only ({catt:.3g} attempts in {ct:.1f} s)"}
        log(f"serving cpu oracle: {catt / ct:.3e} attempts/s on {cores} threads")
    return summ


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cubic100",
                    choices=["cubic100", "square16", "chimera4096", "chimera4096_fm", "square1000_fm", "er2000",
                             "serving", "factoring"])
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--L", type=int, default=100)
    ap.add_argument("--schedule", type=int, default=SCHED_AUTO)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--cpu-sweeps", type=int, default=1000,
                    help="sweeps of the CPU oracle sample (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--no-batched", action="store_true", help="skip the Chimera batch in the default run")
    ap.add_argument("--legs", default="square16,batched,uneven,serving,fm",
                    help="comma-separated workloads measured after the headline in the default run")
    ap.add_argument("--cpu-chimera", type=int, default=2048,
                    help="Chimera instances (x 256 restarts) in the batched leg's CPU oracle sample")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the per-phase comparison runs (the plain method and per-instance baselines)")
    ap.add_argument("--serving-requests", type=int, default=200)
    ap.add_argument("--serving-budget-mb", type=int, default=4096)
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-ingest", type=int, default=12)
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device-to-device 3 times (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU; multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import instances as gen
    import paper_0912_3912_amd as sg

    torch.cuda.set_device(0)
    if args.copy_calibrate:
        nb = args.copy_calibrate << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nb, "copies": 3}), flush=True)
        return
    if args.workload == "cubic100":
        out = run_cubic(args, sg, gen, torch)
        legs = [x for x in args.legs.split(",") if x]
        if args.no_batched and "batched" in legs:
            legs.remove("batched")
        for leg in legs:
            fn = {"square16": run_square, "batched": run_chimera, "uneven": run_er, "serving": run_serving,
                  "fm": run_chimera_fm}[leg]
            t_leg = time.perf_counter()
            out[leg] = fn(args, sg, gen, torch)
            log(f"leg {leg} done in {time.perf_counter() - t_leg:.1f} s")
    else:
        fn = {"square16": run_square, "chimera4096": run_chimera, "chimera4096_fm": run_chimera_fm,
              "square1000_fm": run_square_fm, "er2000": run_er, "serving": run_serving,
              "factoring": run_factoring}[args.workload]
        r = fn(args, sg, gen, torch)
        out = {"metric": r.get("metric", f"spin-flip attempts/s ({r['workload']})"), "value": r["attempts_per_s"],
               "unit": r.get("unit", "attempts/s"), "n_gpus": 1, "steps": args.batch_steps, "warmup": 1,
               "ms_per_step": r.get("ms_per_step", r.get("us_per_solve", 0) / 1e3), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "int8/int32, int64 energy", "data": "synthetic",
               "config": {"workload": r["workload"]}, "roofline": r.get("roofline"),
               "cpu_baseline": r.get("cpu_baseline"), "detail": r}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
