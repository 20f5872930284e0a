"""Continuous-batching solve server on top of the C-ABI.

Requests (an instance plus run parameters) arrive over time.  Each request is
ingested on the host (validation, colouring, packing) by a worker pool, then
waits for admission: it is admitted as soon as the device pool has room for
its workspace (its HBM footprint), skipping ahead of earlier requests that do
not fit yet.  An admitted request binds a range of the pool, draws its
starts, and keeps its couplings, fields and spins resident on the device
until it finishes.

Requests run in one of two ways:

* shared (every instance fits the persistent queue kernel and the request
  runs until converged): it joins the running batch.  A scheduler thread
  repeatedly launches one sg_run_group step of at most ``tick_sweeps`` sweeps
  over every shared request resident at that moment, so requests that arrive
  while others are on the GPU join the next launch, converged ones leave
  after it, and small and large requests share the device launch by launch;
* solo (larger instances, fixed sweep budgets): it takes one of ``slots``
  slots with its own HIP stream and host thread and runs sg_run_sweeps on the
  schedule the library picks, overlapping with the shared launches.

A result depends only on its request (instance, instance_id, seed, rule,
budget): never on its slot, its stream, its pool offset, its neighbours or
how its sweeps were split into launches (the sweep index in the random
counter is the replica's absolute sweep count).
"""
from __future__ import annotations

import bisect
import dataclasses
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional

import numpy as np

ALIGN = 256


class Pool:
    """First-fit allocator of aligned byte ranges inside a fixed budget
    (host bookkeeping only; the device memory is one tensor)."""

    def __init__(self, size: int):
        self.size = int(size) // ALIGN * ALIGN
        self.free = [(0, self.size)]  # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        need = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for k, (off, ln) in enumerate(self.free):
            if ln >= need:
                if ln == need:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + need, ln - need)
                self.used += need
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off: int, nbytes: int):
        need = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        self.used -= need
        k = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(k, (off, need))
        # coalesce with neighbours
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    def largest_free(self) -> int:
        return max((ln for _, ln in self.free), default=0)


@dataclasses.dataclass
class Request:
    rid: int
    instance: object
    seed: int = 7
    rule: int = 0
    max_sweeps: int = 10000
    until_converged: bool = True
    arrival: float = 0.0          # seconds after the trace start


@dataclasses.dataclass
class Result:
    rid: int
    status: str                   # "ok", "notconv", "rejected", "cancelled", "error: ..."
    energy: Optional[int] = None  # best energy over restarts
    best_restart: Optional[int] = None
    spins: Optional[np.ndarray] = None
    sweeps_max: int = 0
    flips: int = 0
    attempts: int = 0
    footprint: int = 0
    slot: int = -1
    arrival: float = 0.0
    ingested: float = 0.0         # host ingest finished (validated, coloured, packed)
    admitted: float = 0.0
    started: float = 0.0
    done: float = 0.0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Admission:
    """Admission policy: the earliest ready request that fits the free pool
    (and, unless it joins the shared batch, a free slot); requests larger
    than the whole pool are rejected."""

    def __init__(self, pool: Pool, slots: int):
        self.pool = pool
        self.free_slots = list(range(slots))
        self.ready: List[tuple] = []  # (arrival order, rid, footprint, shared)

    def add(self, order: int, rid: int, footprint: int, shared: bool = False) -> bool:
        if footprint > self.pool.size:
            return False
        bisect.insort(self.ready, (order, rid, footprint, bool(shared)))
        return True

    def cancel(self, rid: int) -> bool:
        for k, it in enumerate(self.ready):
            if it[1] == rid:
                self.ready.pop(k)
                return True
        return False

    def next(self):
        """(rid, slot, offset) of the next admission, or None; slot is -1 for
        a request that joins the shared batch."""
        for k, (order, rid, fp, shared) in enumerate(self.ready):
            if not shared and not self.free_slots:
                continue
            off = self.pool.alloc(fp)
            if off is not None:
                self.ready.pop(k)
                return rid, (-1 if shared else self.free_slots.pop(0)), off
        return None

    def finish(self, slot: int, off: int, footprint: int):
        self.pool.release(off, footprint)
        if slot >= 0:
            self.free_slots.append(slot)
            self.free_slots.sort()


class Server:
    """Runs requests with continuous admission on one GPU.

    budget_bytes   device pool shared by all resident requests
    slots          solo requests resident and running at once (one stream each)
    ingest_workers host threads that validate and pack arriving instances
    tick_sweeps    most sweeps of one shared launch (requests join and leave
                   the shared batch between launches)
    shared         False: every request runs solo (the per-request baseline)
    """

    def __init__(self, budget_bytes: int, slots: int = 4, ingest_workers: int = 4, device: int = 0,
                 keep_spins: bool = False, tick_sweeps: int = 16, shared: bool = True):
        import torch

        import paper_0912_3912_amd as sg
        self.sg = sg
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.pool = Pool(budget_bytes)
        self.mem = torch.empty(self.pool.size, dtype=torch.uint8, device=self.device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.group_stream = torch.cuda.Stream(device=self.device)
        self.adm = Admission(self.pool, slots)
        self.ingest = ThreadPoolExecutor(max_workers=ingest_workers)
        self.slot_exec = ThreadPoolExecutor(max_workers=max(1, slots))
        self.lock = threading.Condition()
        self.handles: Dict[int, object] = {}
        self.requests: Dict[int, Request] = {}
        self.results: Dict[int, Result] = {}
        self.order = 0
        self.t0 = None
        self.keep_spins = keep_spins
        self.timeline: List[tuple] = []  # (time, bytes resident, requests resident)
        self.cancelled = set()
        self.admitted = set()
        self.ingest_done: Dict[int, float] = {}
        self.tick_sweeps = max(1, int(tick_sweeps))
        self.shared_enabled = bool(shared)
        self.paused = False
        self.closing = False
        self.solo_busy = 0
        self.joining: List[tuple] = []      # (rid, offset) admitted to the shared batch, not yet bound
        self.group: Dict[int, dict] = {}    # rid -> state of a resident shared request
        self.scratch = None
        self.shared_launches = 0
        self.shared_batch_sizes: List[int] = []
        # Large lattices under a fixed sweep count use the co-resident tile
        # launch; two such grids must not be resident at once (each could
        # hold CUs the other needs), so they take turns.
        self.coop_lock = threading.Lock()
        self.loop_error: Optional[BaseException] = None
        self.loop = threading.Thread(target=self._group_loop, name="sg-shared-batch", daemon=True)
        self.loop.start()

    # ------------------------------------------------------------------ API
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        """Hand a request to the server (its arrival time is 'now')."""
        if self.t0 is None:
            self.t0 = time.perf_counter()
        req.arrival = self.now()
        with self.lock:
            self.requests[req.rid] = req
            order = self.order
            self.order += 1
        self.ingest.submit(self._ingest, req, order)

    def cancel(self, rid: int) -> bool:
        """Cancel a request that has not been admitted yet.  Returns False
        when it is already running or finished."""
        with self.lock:
            if rid in self.results or rid in self.admitted or rid not in self.requests:
                return False
            if self.adm.cancel(rid):  # ingested, waiting for admission
                h = self.handles.pop(rid, None)
                if h is not None:
                    h.free()
                self._finish_unadmitted(rid, "cancelled")
                return True
            self.cancelled.add(rid)  # still ingesting: dropped when the ingest ends
            return True

    def pause_admission(self):
        """Stop admitting: ingested requests wait (they can still be cancelled)."""
        with self.lock:
            self.paused = True

    def resume_admission(self):
        with self.lock:
            self.paused = False
            self._admit_locked()

    def wait_ingested(self, rids, timeout: float = 60.0):
        """Block until every request is ingested (waiting for admission,
        running or finished)."""
        end = time.perf_counter() + timeout
        with self.lock:
            while True:
                waiting = {it[1] for it in self.adm.ready}
                if all(r in waiting or r in self.admitted or r in self.results for r in rids):
                    return
                left = end - time.perf_counter()
                if left <= 0:
                    raise TimeoutError("requests still ingesting")
                self.lock.wait(timeout=min(left, 0.05))

    def run_trace(self, requests: List[Request], gaps: List[float], time_scale: float = 1.0):
        """Submit requests at cumulative gaps (seconds * time_scale), wait
        for all results and return them in request order."""
        self.t0 = time.perf_counter()
        t = 0.0
        for req, gap in zip(requests, gaps):
            t += gap * time_scale
            dt = t - self.now()
            if dt > 0:
                time.sleep(dt)
            self.submit(req)
        return self.wait([r.rid for r in requests])

    def wait(self, rids, timeout: float = 600.0):
        end = time.perf_counter() + timeout
        with self.lock:
            while any(r not in self.results for r in rids):
                if self.loop_error is not None:
                    raise RuntimeError(f"shared-batch loop failed: {self.loop_error}")
                left = end - time.perf_counter()
                if left <= 0:
                    raise TimeoutError("requests still pending")
                self.lock.wait(timeout=min(left, 1.0))
            return [self.results[r] for r in rids]

    def close(self):
        self.ingest.shutdown(wait=True)
        with self.lock:
            self.closing = True
            self.lock.notify_all()
        self.loop.join()
        self.slot_exec.shutdown(wait=True)

    # ------------------------------------------------------------ internals
    def _resident(self) -> int:
        return len(self.group) + len(self.joining) + self.solo_busy

    def _mark(self):
        self.timeline.append((self.now(), self.pool.used, self._resident()))

    def _finish_unadmitted(self, rid, status):
        req = self.requests[rid]
        self.results[rid] = Result(rid=rid, status=status, arrival=req.arrival, done=self.now())
        self.lock.notify_all()

    def _ingest(self, req: Request, order: int):
        try:
            h = self.sg.load_instance([req.instance])
            fp = h.workspace_bytes()
            shared = (self.shared_enabled and req.until_converged and req.rule == self.sg.GREEDY
                      and h.query("queue_ok") == 1)
            self.ingest_done[req.rid] = self.now()
        except Exception as e:  # invalid instance
            with self.lock:
                self._finish_unadmitted(req.rid, f"error: {e}")
            return
        with self.lock:
            if req.rid in self.cancelled:
                h.free()
                self._finish_unadmitted(req.rid, "cancelled")
                return
            self.handles[req.rid] = h
            if not self.adm.add(order, req.rid, fp, shared=shared):
                h.free()
                self._finish_unadmitted(req.rid, "rejected")
                return
            self.lock.notify_all()
            self._admit_locked()

    def _admit_locked(self):
        while not self.paused:
            nxt = self.adm.next()
            if nxt is None:
                return
            rid, slot, off = nxt
            self.admitted.add(rid)
            if slot < 0:
                self.joining.append((rid, off))
                self.lock.notify_all()
            else:
                self.solo_busy += 1
                self.slot_exec.submit(self._run, rid, slot, off)
            self._mark()

    # -------------------------------------------------------- shared batch
    def _group_loop(self):
        try:
            while True:
                with self.lock:
                    while not self.closing and not self.group and not self.joining:
                        self.lock.wait(timeout=0.05)
                    if self.closing and not self.group and not self.joining:
                        return
                    joins, self.joining = self.joining, []
                    handles = {rid: self.handles.pop(rid) for rid, _ in joins}
                for rid, off in joins:
                    self._join(rid, off, handles[rid])
                if self.group:
                    self._shared_step()
        except BaseException as e:  # surface to waiters instead of hanging them
            with self.lock:
                self.loop_error = e
                self.lock.notify_all()

    def _join(self, rid: int, off: int, h):
        req = self.requests[rid]
        fp = h.workspace_bytes()
        res = Result(rid=rid, status="ok", footprint=fp, slot=-1, arrival=req.arrival, admitted=self.now(),
                     ingested=self.ingest_done.get(rid, req.arrival))
        try:
            h.bind_raw(self.mem.data_ptr() + off, fp, self.group_stream.cuda_stream)
            h.init_spins(req.seed)
            res.started = self.now()
            self.group[rid] = {"h": h, "off": off, "fp": fp, "res": res, "launched": 0, "req": req}
        except Exception as e:
            res.status = f"error: {e}"
            self.group_stream.synchronize()
            h.free()
            self._release(rid, -1, off, fp, res)

    def _shared_step(self):
        rids = list(self.group)
        ent = [self.group[r] for r in rids]
        T = min([self.tick_sweeps] + [e["req"].max_sweeps - e["launched"] for e in ent])
        hs = [e["h"] for e in ent]
        if T > 0:
            need = self.sg.group_scratch_bytes(hs)
            if self.scratch is None or self.scratch.numel() < need:
                self.scratch = self.torch.empty(max(need, 2 * (0 if self.scratch is None else self.scratch.numel())),
                                                dtype=self.torch.uint8, device=self.device)
            _, unc = self.sg.run_group(hs, self.scratch, seed=0, rule=self.sg.GREEDY, max_sweeps=T,
                                       until_converged=True)
            self.shared_launches += 1
            self.shared_batch_sizes.append(len(hs))
        else:
            unc = [e["h"].total_replicas for e in ent]
        for rid, e, u in zip(rids, ent, unc):
            e["launched"] += T
            if u == 0 or e["launched"] >= e["req"].max_sweeps:
                self._finish_shared(rid, e, converged=(u == 0))

    def _finish_shared(self, rid: int, e: dict, converged: bool):
        h, res = e["h"], e["res"]
        try:
            E, r = h.best()
            res.energy, res.best_restart = int(E[0]), int(r[0])
            if self.keep_spins:
                res.spins = h.spins_out(0, int(r[0]))
            sw, fl, _ = h.counters()
            n = h.sizes[0]
            res.sweeps_max, res.flips, res.attempts = int(sw.max()), int(fl.sum()), int(sw.sum()) * n
            if not converged:
                res.status = "notconv"
        except Exception as ex:
            res.status = f"error: {ex}"
        finally:
            self.group_stream.synchronize()
            h.free()
        del self.group[rid]
        self._release(rid, -1, e["off"], e["fp"], res)

    def _release(self, rid: int, slot: int, off: int, fp: int, res: Result):
        res.done = self.now()
        with self.lock:
            self.adm.finish(slot, off, fp)
            if slot >= 0:
                self.solo_busy -= 1
            self.results[rid] = res
            self._mark()
            self.lock.notify_all()
            self._admit_locked()

    # ----------------------------------------------------------- solo path
    def _run(self, rid: int, slot: int, off: int):
        req = self.requests[rid]
        with self.lock:
            h = self.handles.pop(rid)
        fp = h.workspace_bytes()
        res = Result(rid=rid, status="ok", footprint=fp, slot=slot, arrival=req.arrival, admitted=self.now(),
                     ingested=self.ingest_done.get(rid, req.arrival))
        try:
            st = self.streams[slot]
            base = self.mem.data_ptr() + off
            h.bind_raw(base, fp, st.cuda_stream)
            res.started = self.now()
            h.init_spins(req.seed)
            info = h.info(0)
            # a lattice beyond one workgroup runs on the co-resident tile launch
            # (fixed budgets, and GREEDY until converged on the bit-plane kernel)
            coop = info["lattice"] and info["n"] > h.query("lattice_wg_max_n")
            if coop:
                with self.coop_lock:
                    stats = h.run_sweeps(seed=req.seed, rule=req.rule, max_sweeps=req.max_sweeps,
                                         until_converged=req.until_converged)
            else:
                stats = h.run_sweeps(seed=req.seed, rule=req.rule, max_sweeps=req.max_sweeps,
                                     until_converged=req.until_converged)
            E, r = h.best()
            res.energy, res.best_restart = int(E[0]), int(r[0])
            if self.keep_spins:
                res.spins = h.spins_out(0, int(r[0]))
            res.sweeps_max, res.flips, res.attempts = stats["sweeps_max"], stats["flips"], stats["attempts"]
            if stats["status"] == self.sg.SG_ENOTCONV:
                res.status = "notconv"
        except Exception as e:
            res.status = f"error: {e}"
        finally:
            # work still queued on the slot's stream (a start whose run then
            # failed) must end before its pool slice goes to another request
            self.streams[slot].synchronize()
            h.free()
        self._release(rid, slot, off, fp, res)


def summarize(results: List[Result], wall: float) -> dict:
    """Latency (arrival to result on the host) percentiles and throughput,
    with the latency split into host ingest (arrival to packed), waiting for
    admission (packed to admitted) and the run on the device (admitted to
    result, including the start and the readout)."""
    ok = [r for r in results if r.status in ("ok", "notconv")]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    ing = np.array([r.ingested - r.arrival for r in ok]) if ok else np.zeros(1)
    wai = np.array([r.admitted - r.ingested for r in ok]) if ok else np.zeros(1)
    run = np.array([r.done - r.admitted for r in ok]) if ok else np.zeros(1)
    att = sum(r.attempts for r in ok)
    fl = sum(r.flips for r in ok)

    def pct(a, q):
        return float(np.percentile(a, q) * 1e3)

    return {"requests": len(results), "completed": len(ok),
            "rejected": sum(r.status == "rejected" for r in results),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(lat.mean() * 1e3),
            "ingest_p50_ms": pct(ing, 50), "ingest_p99_ms": pct(ing, 99),
            "admission_wait_p50_ms": pct(wai, 50), "admission_wait_p99_ms": pct(wai, 99),
            "device_p50_ms": pct(run, 50), "device_p99_ms": pct(run, 99),
            "shared_requests": sum(r.slot < 0 for r in ok), "solo_requests": sum(r.slot >= 0 for r in ok),
            "wall_s": wall, "attempts_per_s": att / wall, "flips_per_s": fl / wall, "requests_per_s": len(ok) / wall}
