"""Serving loop: continuous batching of check requests on one GPU.

Requests arrive with timestamps (Poisson arrivals from ``workloads.request_stream``).
The loop keeps up to ``slots`` batches in flight, each on its own HIP stream
through ``kc_batch_submit``; whenever a slot is free it admits the longest run
of arrived requests whose device footprint -- as the library accounts it
(``kc_batch_footprint``), plus their memories -- fits in the free part of a
fixed HBM budget (FIFO, a request is never skipped), uploads their memories
and submits them as one batch.  Completed batches are collected with
non-blocking ``kc_poll``; their memory is released and the latency
(completion time - arrival time) recorded.  The request source is replayed in
real time: a request is not admitted before its arrival time.

The scheduler core (`Admission`) is plain Python over sizes and clocks so it
can be unit-tested on the CPU with a fake executor; `Server` drives the real
library.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import kc


def estimate_bytes(job) -> int:
    """Device bytes a request may hold while in flight: its memory, the
    launch-start snapshot, and the access log (records estimated from the
    program shape: 8 B each, 12 accesses per thread per launch as a bound for
    the families served here) plus sort scratch of the same size."""
    mem = 4 * len(job.memory)
    threads = sum(L.n_threads * L.n_blocks for L in job.launches)
    log = 8 * 12 * threads
    return 2 * mem + 2 * log


@dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the run
    job: object
    bytes: int
    admitted: float = -1.0
    done: float = -1.0
    report: Optional[object] = None


class Admission:
    """FIFO admission under a byte budget with a bounded number of slots.

    ``cost(requests)`` gives the device bytes a batch of those requests
    holds (by default the sum of their ``bytes``); a batch is the longest
    prefix of the queue, up to ``max_batch`` requests, whose cost fits in the
    free part of the budget, found by bisection (the cost grows with the
    batch).  A request is never skipped."""

    def __init__(self, budget_bytes: int, slots: int, max_batch: int = 4096,
                 cost: Optional[Callable[[Sequence[Request]], int]] = None):
        self.budget = budget_bytes
        self.slots = slots
        self.max_batch = max_batch
        self.cost = cost or (lambda rs: sum(r.bytes for r in rs))
        self.in_use = 0
        self.inflight = 0
        self.held: Dict[int, int] = {}      # id(batch list) -> its cost
        self.queue: Deque[Request] = collections.deque()

    def arrive(self, r: Request):
        if self.cost([r]) > self.budget:
            raise ValueError(f"request {r.rid} needs {self.cost([r])} B, more than the whole budget")
        self.queue.append(r)

    def take(self) -> List[Request]:
        """Requests for the next batch (empty if no slot or nothing fits)."""
        if self.inflight >= self.slots or not self.queue:
            return []
        free = self.budget - self.in_use
        cand = [self.queue[i] for i in range(min(len(self.queue), self.max_batch))]
        n, used = len(cand), self.cost(cand)
        if used > free:         # the longest fitting prefix, by bisection
            lo, hi, used = 0, n, 0
            while hi - lo > 1:
                mid = (lo + hi) // 2
                c = self.cost(cand[:mid])
                if c <= free:
                    lo, used = mid, c
                else:
                    hi = mid
            n = lo
        if n == 0:
            return []
        batch = [self.queue.popleft() for _ in range(n)]
        self.in_use += used
        self.inflight += 1
        self.held[id(batch)] = used
        return batch

    def finish(self, batch: Sequence[Request]):
        self.in_use -= self.held.pop(id(batch))
        self.inflight -= 1
        assert self.in_use >= 0 and self.inflight >= 0


def simulate(arrivals: Sequence[Tuple[float, int]], service: Callable[[int], float], budget: int, slots: int):
    """Run the admission policy against a fake clock: ``arrivals`` are
    (time, bytes); ``service(n_bytes)`` gives a batch's duration.  Returns the
    per-request (arrival, start, done) and the peak bytes in use."""
    adm = Admission(budget, slots)
    reqs = [Request(i, t, None, b) for i, (t, b) in enumerate(arrivals)]
    pending = list(reqs)
    running: List[Tuple[float, List[Request]]] = []
    now, peak = 0.0, 0
    while pending or adm.queue or running:
        while pending and pending[0].arrival <= now:
            adm.arrive(pending.pop(0))
        while True:
            b = adm.take()
            if not b:
                break
            for r in b:
                r.admitted = now
            running.append((now + service(sum(r.bytes for r in b)), b))
            peak = max(peak, adm.in_use)
        if running:
            running.sort(key=lambda x: x[0])
        nxt = [running[0][0]] if running else []
        if pending:
            nxt.append(pending[0].arrival)
        if not nxt:
            break
        now = max(now, min(nxt))
        while running and running[0][0] <= now:
            t, b = running.pop(0)
            for r in b:
                r.done = t
            adm.finish(b)
    return [(r.arrival, r.admitted, r.done) for r in reqs], peak


class Server:
    """Continuous-batching front end over a kc.Context."""

    def __init__(self, ctx: kc.Context, budget_bytes: int = 64 << 30, slots: int = 4):
        """Admission charges each batch the device bytes the library reports
        for it (kc_batch_footprint) plus its memories and their uploads;
        ``ctx`` should carry the same budget, which the library then
        enforces over all of its buffers."""
        import torch
        self.ctx = ctx
        self._added: Dict[int, int] = {}    # id(job) -> bytes it adds to a batch's footprint
        self._fixed, self._fixed_at = 0, -1.0
        self.adm = Admission(budget_bytes, slots, cost=self._cost)
        self.streams = [torch.cuda.Stream() for _ in range(slots)]   # default priority
        self.free_streams = list(range(slots))
        self.batch = kc.Batch(ctx)

    def _cost(self, reqs: Sequence[Request]) -> int:
        """Library footprint of a batch, bounded by the part of an empty
        batch plus each job's own addition (computed once per job) and the
        jobs' memories."""
        if not reqs:
            return 0
        now = time.perf_counter()
        if now - self._fixed_at > 0.05:         # the part every batch reserves follows the context's hints
            self._fixed, self._fixed_at = kc.jobs_footprint(self.ctx, []), now
        fixed = self._fixed
        total = fixed
        for r in reqs:
            add = self._added.get(id(r.job))
            if add is None:
                add = (kc.jobs_footprint(self.ctx, [r.job]) - kc.jobs_footprint(self.ctx, []) +
                       4 * len(r.job.memory))
                self._added[id(r.job)] = add
            total += add
        return total

    def run(self, stream: Sequence[Tuple[float, object]], keep_reports: bool = False,
            keep_memory: bool = False, pristine: Optional[Dict[int, object]] = None,
            keep_every: int = 0) -> Dict:
        """Serve ``stream`` = [(arrival_s, job)].  ``pristine`` optionally maps
        id(job) to a device tensor holding that job's initial memory; such a
        request's memory is a device-to-device copy of it on the batch's
        stream instead of an upload from the host.  With ``keep_every`` = k,
        every k-th request's (job, report, final memory) is returned under
        "sample"."""
        import torch
        self._added.clear()
        self._fixed_at = -1.0
        reqs = [Request(i, t, j, estimate_bytes(j)) for i, (t, j) in enumerate(stream)]
        pending = collections.deque(reqs)
        inflight: List[Tuple[int, int, List[Request], list]] = []   # (ticket, stream idx, reqs, mems)
        t0 = time.perf_counter()
        records = 0
        busy_batches = 0
        memories: Dict[int, np.ndarray] = {}
        sample = []
        while pending or self.adm.queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                self.adm.arrive(pending.popleft())
            # collect finished batches
            still = []
            for ticket, si, batch, mems in inflight:
                reps = self.batch.poll(ticket, wait=False)
                if reps is None:
                    still.append((ticket, si, batch, mems))
                    continue
                done = time.perf_counter() - t0
                records += int(reps.records.sum())
                for i, (r, m) in enumerate(zip(batch, mems)):
                    r.done = done
                    if keep_reports:
                        r.report = reps[i]
                    if keep_memory:
                        memories[r.rid] = m.cpu().numpy()
                    if keep_every and r.rid % keep_every == 0:
                        sample.append((r.job, reps[i], m.cpu().numpy()))
                self.adm.finish(batch)
                self.free_streams.append(si)
            inflight = still
            # admit and submit
            while self.free_streams:
                batch = self.adm.take()
                if not batch:
                    break
                si = self.free_streams.pop()
                st = self.streams[si]
                with torch.cuda.stream(st):
                    mems = []
                    for r in batch:
                        src = pristine.get(id(r.job)) if pristine else None
                        if src is not None:
                            mems.append(src.clone())
                        else:
                            mems.append(torch.from_numpy(np.ascontiguousarray(r.job.memory)).to(
                                "cuda", non_blocking=False))
                if not pristine:
                    st.synchronize()
                now = time.perf_counter() - t0
                for r in batch:
                    r.admitted = now
                ticket = self.batch.submit([kc.job_item(self.ctx, r.job, m, r.rid)
                                            for r, m in zip(batch, mems)], stream=st)
                inflight.append((ticket, si, batch, mems))
                busy_batches += 1
            if not inflight and pending and not self.adm.queue:
                time.sleep(max(0.0, min(pending[0].arrival - (time.perf_counter() - t0), 0.001)))
            else:
                time.sleep(0.0002)
        wall = time.perf_counter() - t0
        lat = np.array([r.done - r.arrival for r in reqs]) if reqs else np.zeros(1)
        out = {"requests": len(reqs), "records": records, "wall_s": wall,
               "records_per_s": records / wall if wall > 0 else 0.0,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "batches": busy_batches,
               "mean_batch": len(reqs) / busy_batches if busy_batches else 0.0}
        if keep_reports:
            out["reports"] = {r.rid: r.report for r in reqs}
        if keep_memory:
            out["memories"] = memories
        if keep_every:
            out["sample"] = sample
        return out
