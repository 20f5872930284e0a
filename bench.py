"""Benchmark: spin-flip attempts per second of the colour-ordered descent on
one MI355X, with the roofline position of the dominant kernel and the CPU
oracle timed on the host beside it.

Default workload: the 10^6-spin periodic 100^3 +-J lattice with fields
h in {-2..2}, checkerboard colouring, one random start, GREEDY_TIE for
exactly 1000 sweeps (10^9 attempts).  One step = random start + start
energy + 1000 sweeps + best-of-restarts + energy readout, all on the GPU,
with the coupling structure already resident in HBM.

Prints one JSON line (rank 0).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_attempt(kind: str, deg: int = 6, tau: float = 0.0) -> float:
    """Algorithmic bytes one attempt must move in the layout the kernel reads.

    sliced-CSR: deg coupling words of 4 bytes (24-bit partner | int8 J),
      2*tau hyper-coupling words of 4 bytes, 1 byte field, 1 byte own spin
      read + 1 byte write, 1 byte of the other colours' spins (each read once
      per phase: cache-reuse lower bound); slice metadata (16 B per 64 rows)
      is below 1 byte.
    """
    if kind == "sell":
        return 4.0 * deg + 8.0 * tau + 1 + 2 + 1
    raise ValueError(kind)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--L", type=int, default=100)
    ap.add_argument("--schedule", type=int, default=-1)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--cpu-sweeps", type=int, default=500,
                    help="sweeps of the oracle CPU-baseline sample (0 = skip)")
    ap.add_argument("--no-parity", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: multi-GPU runs are not supported by this build",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import instances as gen
    import paper_0912_3912_amd as sg

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    L = args.L
    inst = gen.cfg2_cubic100(L=L)
    n = inst.n
    h = sg.load_instance([inst], lattice_dims=[(L, L, L)]).bind()
    ws_mb = h.workspace_bytes() / 1e6
    log(f"workload cubic{L}: n={n} m={inst.m} workspace={ws_mb:.1f} MB sweeps={args.sweeps}")

    def step():
        h.init_spins(args.seed)
        st = h.run_sweeps(seed=args.seed, rule=sg.GREEDY_TIE, max_sweeps=args.sweeps,
                          until_converged=False, schedule=args.schedule)
        h.best()
        return st

    for w in range(args.warmup):
        st = step()
        log(f"warmup {w}: kernel_ms={st['kernel_ms']:.3f} schedule={st['schedule_used']}")
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = step()
        kms.append(st["kernel_ms"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    attempts = n * args.sweeps
    value = attempts * args.steps / dt
    ms_step = dt / args.steps * 1e3
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, sweep kernels {np.mean(kms):.3f} ms")
    E = int(h.energy()[0])

    # roofline of the dominant kernel (the sweep kernels of this step)
    bpa = bytes_per_attempt("sell", deg=6)
    sched = st["schedule_used"]
    launches = args.sweeps * 2 if sched in (0, 1) else 1
    kernel_ms = float(np.mean(kms))
    per_launch_s = kernel_ms / 1e3 / launches
    achieved = bpa * attempts / launches / per_launch_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                "kernel": {0: "k_phase", 1: "k_phase (graph)", 2: "k_persistent", 3: "k_lattice"}.get(sched, str(sched)),
                "bytes_per_attempt": bpa, "launches_per_step": launches,
                "avg_launch_us": round(per_launch_s * 1e6, 3)}

    cpu = None
    if args.cpu_sweeps > 0:
        import oracle
        t1 = time.perf_counter()
        ref, _ = oracle.run(inst, seed=args.seed, rule=oracle.GREEDY_TIE, max_sweeps=args.cpu_sweeps,
                            until_converged=False, threads=1)
        ct = time.perf_counter() - t1
        cpu = {"value": n * args.cpu_sweeps / ct, "unit": "attempts/s", "cores": 1, "kind": "oracle",
               "sample": f"cubic{L}, 1 start, first {args.cpu_sweeps} of {args.sweeps} GREEDY_TIE sweeps "
                         f"({n * args.cpu_sweeps:.3g} attempts, {ct:.1f} s)"}
        log(f"cpu oracle: {cpu['value']:.3e} attempts/s over {ct:.1f} s")

    out = {
        "metric": "spin-flip attempts/s (1M-spin 3-D +-J lattice, 1000 sweeps)",
        "value": value, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int8/int32 (int64 energy)",
        "data": "synthetic", "config": {"workload": f"cubic{L}_pmJ_h2_tie_{args.sweeps}sweeps",
                                        "n_spins": n, "bonds": inst.m, "sweeps": args.sweeps,
                                        "restarts": 1, "rule": "GREEDY_TIE", "schedule": sched,
                                        "energy": E, "workspace_mb": round(ws_mb, 1)},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
