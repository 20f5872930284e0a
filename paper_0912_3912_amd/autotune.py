"""Measured choice of the schedule and its knobs for a loaded, bound handle.

``SG_SCHED_AUTO`` picks a schedule per instance from fixed rules (lattice
tiles, then the block schedule for many restarts, then the persistent queue,
else per-phase launches) and the knobs' defaults.  ``autotune`` replaces those
defaults by measurement: the first time a workload key is seen (instance
family, size and count buckets, restarts bucket, rule, stopping rule) it
draws the handle's starts and times a short run of every candidate setting
on the handle itself, keeps the fastest, and records it in a table (a JSON
file when a path is given) that later handles of the same key reuse without
measuring.  The knobs change only how sweeps map onto the GPU: every
candidate gives the same spins, energies and counters bit for bit, so the
choice never changes a result.

Calibration draws starts and runs sweeps on the handle: call it before the
handle's real ``init_spins`` (it leaves the handle started from ``seed``,
with the counters of its last calibration run).
"""
from __future__ import annotations

import json
import math
import os
import threading
from typing import Dict, List, Optional

SCHED_AUTO, SCHED_PHASE, SCHED_GRAPH, SCHED_QUEUE = -1, 0, 1, 5

_lock = threading.Lock()
_memory: Dict[str, dict] = {}


def _bucket(v: float) -> int:
    return int(math.floor(math.log2(max(1.0, float(v)))))


def workload_key(h, rule: int, until_converged: bool) -> str:
    """Key of the tuning table: what the schedule choice depends on."""
    ninst = h.query("instances")
    infos = [h.info(q) for q in range(ninst)]
    ns = sorted(i["n"] for i in infos)
    n_med = ns[len(ns) // 2]
    n_max = ns[-1]
    R = max(i["restarts"] for i in infos)
    lattice = all(i["lattice"] for i in infos)
    tri = any(i["t"] > 0 for i in infos)
    fam = "lattice" if lattice else ("graph3" if tri else "graph")
    if h.query("wide_instances"):
        fam += "-wide"
    return (f"{fam}|nmed{_bucket(n_med)}|nmax{_bucket(n_max)}|inst{_bucket(ninst)}|R{_bucket(R)}"
            f"|rule{rule}|uc{int(bool(until_converged))}")


def candidates(h, rule: int, until_converged: bool) -> List[dict]:
    """Settings worth timing for this handle: each is a dict of sg_tune knobs
    plus an optional explicit "schedule"."""
    ninst = h.query("instances")
    infos = [h.info(q) for q in range(ninst)]
    R = max(i["restarts"] for i in infos)
    n_max = max(i["n"] for i in infos)
    lattice = all(i["lattice"] for i in infos)
    out: List[dict] = [{}]  # the defaults
    if lattice and n_max > h.query("lattice_wg_max_n") and not until_converged:
        # one large lattice on the tile kernels: halo widths around the cost model's pick, and the byte kernel
        out += [{"msc_k": k} for k in (3, 4, 6, 8)]
        out += [{"lattice_msc": 0}]
    elif R >= h.query("block_min_restarts") and n_max <= 2048 and rule == 0:
        out += [{"bits_groups": g} for g in (4, 16)]
        out += [{"block_bits": 0}]
    elif h.query("queue_ok") and ninst >= 2:
        out += [{"queue_wave_max_n": w} for w in (128, 256, 512, 1024, 2048)]
        if ninst <= 64:
            # few instances: their per-phase launches, plain or recorded in graphs, instead of the queue
            out += [{"queue_min_items": 1 << 30}]
            out += [{"queue_min_items": 1 << 30, "auto_graph": 1}]
    else:
        out += [{"auto_graph": 1, "graph_sweeps": g} for g in (8, 32, 128)]
    return out


_DEFAULTS = ("msc_k", "lattice_msc", "bits_groups", "block_bits", "queue_wave_max_n", "queue_min_items",
             "auto_graph", "graph_sweeps")


def apply(h, setting: dict, defaults: dict):
    for k in _DEFAULTS:
        h.tune(k, setting.get(k, defaults[k]))


def load_table(path: Optional[str]) -> Dict[str, dict]:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_table(path: str, table: Dict[str, dict]):
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(h, seed: int, rule: int = 0, max_sweeps: int = 10000, until_converged: bool = True,
             table_path: Optional[str] = None, calib_sweeps: int = 64, repeats: int = 2) -> dict:
    """Pick and apply the fastest setting for this handle's workload key.

    Returns the table entry: {"key", "setting", "ms", "measured" (per
    candidate), "calibration_ms" (host wall time spent measuring, 0 when the
    table already held the key), "from_table"}."""
    import time
    key = workload_key(h, rule, until_converged)
    defaults = {k: h.query(k) for k in _DEFAULTS}
    with _lock:
        table = dict(_memory)
        table.update(load_table(table_path))
        hit = table.get(key)
    if hit is not None:
        apply(h, hit["setting"], defaults)
        return dict(hit, key=key, from_table=True, calibration_ms=0.0)
    t0 = time.perf_counter()
    budget = max_sweeps if not until_converged else min(max_sweeps, calib_sweeps)
    measured = []
    for cand in candidates(h, rule, until_converged):
        apply(h, cand, defaults)
        best = None
        for _ in range(max(1, repeats)):
            h.init_spins(seed)
            st = h.run_sweeps(seed=seed, rule=rule, max_sweeps=budget, until_converged=until_converged,
                              schedule=cand.get("schedule", SCHED_AUTO))
            ms = float(st["kernel_ms"])
            best = ms if best is None else min(best, ms)
        measured.append({"setting": cand, "ms": best})
    win = min(measured, key=lambda m: m["ms"])
    apply(h, win["setting"], defaults)
    h.init_spins(seed)
    entry = {"setting": win["setting"], "ms": win["ms"], "measured": measured,
             "calib_sweeps": budget, "calibration_ms": (time.perf_counter() - t0) * 1e3}
    with _lock:
        _memory[key] = entry
        if table_path:
            table = load_table(table_path)
            table[key] = entry
            save_table(table_path, table)
    return dict(entry, key=key, from_table=False)
