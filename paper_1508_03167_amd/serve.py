"""Continuous-batching shuffle server.

Requests (an array of n elements of 4 or 8 bytes and a seed) arrive over
time.  The server admits a request when the HBM it needs fits the budget --
its payload, resident from admission to completion, plus the library scratch
a call of its size needs -- and refuses outright a request that alone exceeds
the budget.  Admitted requests wait in arrival order; whenever one of the
server's `max_inflight` slots (one stream each) is free, the admitted
requests not yet launched go, in arrival order and up to an element cap,
into one batched call on that slot (optionally, requests above the cap
run at most a few at a time, passed meanwhile by smaller ones)
(ms_shuffle_batched_seeds: each request shuffled with its own seed), so
requests that arrive while others run join the next batch and overlap the
batches already on the device.  Completion is seen by polling an event per
batch; the payload space is then recycled.  Each result is exactly what
ms_shuffle would give the request alone (the shuffle depends only on the
request's size and seed).

The scheduling logic (Server) is independent of the device: an executor
provides footprints, payload space, launches and completion checks.
GpuExecutor runs on the GPU through the library; the tests also drive the
server with a simulated executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional

ALIGN = 256


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    elem_bytes: int
    seed: int
    arrival: float
    admitted: Optional[float] = None
    launched: Optional[float] = None
    done: Optional[float] = None
    rejected: bool = False
    batch: int = -1
    offset: int = -1       # payload offset in the executor's pool
    footprint: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Server:
    """The admission / batching / completion logic of the server."""

    def __init__(self, executor, hbm_budget: int, max_inflight: int = 2, max_batch: int = 4096,
                 max_batch_elems: Optional[int] = None, max_large_inflight: Optional[int] = None):
        if max_inflight < 1:
            raise ValueError("max_inflight must be at least 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        # a batch stops before the request that would take its element count
        # past this (it always takes at least one), so that small requests do
        # not wait for the completion of a large one launched with them
        self.max_batch_elems = max_batch_elems
        # requests above the element cap ("large") on the device at once: with
        # a limit, a large request that would exceed it waits and smaller ones
        # behind it may go first (large requests slow one another down when
        # they share the device, small ones barely do)
        self.max_large_inflight = max_large_inflight
        self.used = 0
        self.waiting: collections.deque = collections.deque()   # arrived, not admitted
        self.ready: collections.deque = collections.deque()     # admitted, not launched
        self.inflight = {}                                        # slot -> (handle, [requests], batch id)
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.batches = 0
        self.peak_used = 0

    def submit(self, req: Request, now: float):
        req.footprint = self.ex.footprint(req.n, req.elem_bytes)
        if req.footprint > self.budget:
            req.rejected = True
            req.done = now
            self.rejected.append(req)
            return
        self.waiting.append(req)

    def _admit(self, now: float):
        # in arrival order: the head waits until it fits, so a large request
        # is not overtaken indefinitely by small ones
        while self.waiting:
            r = self.waiting[0]
            if self.used + r.footprint > self.budget:
                break
            off = self.ex.acquire(r)
            if off is None:
                break
            self.waiting.popleft()
            r.offset = off
            r.admitted = now
            self.used += r.footprint
            self.peak_used = max(self.peak_used, self.used)
            self.ready.append(r)

    def _complete(self, now: float):
        for slot in list(self.inflight):
            handle, reqs, _ = self.inflight[slot]
            if self.ex.done(handle):
                del self.inflight[slot]
                for r in reqs:
                    r.done = now
                    self.used -= r.footprint
                    self.ex.release(r)
                    self.finished.append(r)

    def _large(self, r: Request) -> bool:
        return self.max_batch_elems is not None and r.n > self.max_batch_elems

    def _launch(self, now: float):
        free = [s for s in range(self.max_inflight) if s not in self.inflight]
        while free and self.ready:
            large_busy = self.max_large_inflight is not None and sum(
                1 for _, rs, _ in self.inflight.values() if any(self._large(r) for r in rs)) >= self.max_large_inflight
            reqs = []
            elems = 0
            keep = collections.deque()
            while self.ready and len(reqs) < self.max_batch:
                r = self.ready[0]
                if large_busy and self._large(r):
                    keep.append(self.ready.popleft())  # waits for the large slot
                    continue
                if reqs and self.max_batch_elems is not None and elems + r.n > self.max_batch_elems:
                    break
                elems += r.n
                reqs.append(self.ready.popleft())
            keep.extend(self.ready)
            self.ready = keep
            if not reqs:
                break
            slot = free.pop(0)
            for r in reqs:
                r.launched = now
                r.batch = self.batches
            self.inflight[slot] = (self.ex.launch(reqs, slot), reqs, self.batches)
            self.batches += 1

    def step(self, now: float):
        """Complete finished batches, admit what fits, launch on free slots."""
        self._complete(now)
        self._admit(now)
        self._launch(now)

    def idle(self) -> bool:
        return not (self.waiting or self.ready or self.inflight)

    def run(self, requests: List[Request], clock: Callable[[], float], wait: Callable[[float], None]):
        """Serve requests (sorted by arrival, arrival times relative to the
        start) until every one is finished or rejected."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = clock()
        i = 0
        while i < len(reqs) or not self.idle():
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i], now)
                i += 1
            self.step(now)
            if i < len(reqs) and self.idle():
                wait(reqs[i].arrival - now)
            elif not self.ex.poll_is_cheap:
                wait(0.0)
        return self.finished, self.rejected


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


class GpuExecutor:
    """Runs batches through the library on a pool of streams; payloads live
    in one device pool (first-fit ranges, recycled on completion).

    batched=False launches one ms_shuffle call per request instead (with
    max_batch=1 and one slot, the plain one-call-per-request loop).  For the
    request ids in `check`, the input is copied before the launch and the
    result once its batch is done (device copies, no waiting); verify() then
    shuffles each input alone with the request's seed and compares it with
    the result from the mix, after the stream, so that checking adds no
    latency to the requests; `mismatches` lists those that differ."""

    poll_is_cheap = True

    def __init__(self, pool_bytes: int, max_inflight: int = 2, device: str = "cuda:0", fill=None,
                 batched: bool = True, check=()):
        import torch

        from . import _lib

        self.torch = torch
        self.M = _lib
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        if fill is not None:
            fill(self.pool)
        self.pool_bytes = int(pool_bytes)
        self.free = [(0, self.pool_bytes)]          # sorted (start, length)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max_inflight)]
        self.scratch_cache = {}
        self.batched = batched
        self.check = set(check)
        self.saved = {}      # rid -> (input copy, seed)
        self.results = {}    # rid -> result copy
        self.checked = []
        self.mismatches = []

    def footprint(self, n: int, eb: int) -> int:
        key = (n, eb)
        if key not in self.scratch_cache:
            self.scratch_cache[key] = self.M.scratch_bytes(n, eb) if n > 1 else 0
        return -(-n * eb // ALIGN) * ALIGN + self.scratch_cache[key]

    def acquire(self, r: Request):
        need = -(-r.n * r.elem_bytes // ALIGN) * ALIGN
        for i, (s, ln) in enumerate(self.free):
            if ln >= need:
                if ln == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + need, ln - need)
                return s
        return None

    def release(self, r: Request):
        if r.rid in self.saved:
            # the batch's event has completed: copy the result before the
            # range is reused
            self.results[r.rid] = self.view(r).clone()
        need = -(-r.n * r.elem_bytes // ALIGN) * ALIGN
        self.free.append((r.offset, need))
        self.free.sort()
        merged = []
        for s, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((s, ln))
        self.free = merged

    def view(self, r: Request):
        torch = self.torch
        raw = self.pool[r.offset:r.offset + r.n * r.elem_bytes]
        return raw.view(torch.int64 if r.elem_bytes == 8 else torch.int32)

    def launch(self, reqs: List[Request], slot: int):
        torch = self.torch
        st = self.streams[slot]
        # the payloads were written on the caller's stream (or earlier batches)
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            for r in reqs:
                if r.rid in self.check:
                    self.saved[r.rid] = (self.view(r).clone(), r.seed)
        if self.batched:
            self.M.shuffle_batched_seeds_([self.view(r) for r in reqs], [r.seed for r in reqs], stream=st)
        else:
            for r in reqs:
                self.M.shuffle_(self.view(r), r.seed, stream=st)
        ev = torch.cuda.Event()
        ev.record(st)
        return ev

    def done(self, ev) -> bool:
        return ev.query()

    def verify(self):
        """Shuffle each checked input alone and compare it with its result
        from the mix (call after the stream has been served)."""
        torch = self.torch
        torch.cuda.synchronize()
        for rid, (before, seed) in sorted(self.saved.items()):
            if rid not in self.results:
                continue
            self.M.shuffle_(before, seed)
            torch.cuda.synchronize()
            self.checked.append(rid)
            if not bool(torch.equal(before, self.results[rid])):
                self.mismatches.append(rid)
        self.saved.clear()
        self.results.clear()


def serve_stream(requests: List[Request], executor, hbm_budget: int, max_inflight: int = 2,
                 max_batch: int = 4096, max_batch_elems: Optional[int] = None,
                 max_large_inflight: Optional[int] = None):
    """Run a request stream in real time on the executor; returns summary figures."""
    srv = Server(executor, hbm_budget, max_inflight=max_inflight, max_batch=max_batch,
                 max_batch_elems=max_batch_elems, max_large_inflight=max_large_inflight)
    t0 = time.perf_counter()

    def wait(dt):
        if dt > 0:
            time.sleep(min(dt, 0.0005))

    done, rej = srv.run(requests, time.perf_counter, wait)
    span = time.perf_counter() - t0
    lat = [r.latency for r in done]
    elems = sum(r.n for r in done)
    sizes = [len(b) for b in _batches(done)]
    return {"served": len(done), "rejected": len(rej), "batches": srv.batches, "span_s": round(span, 3),
            "p50_ms": round(percentile(lat, 50) * 1e3, 3), "p99_ms": round(percentile(lat, 99) * 1e3, 3),
            "gelem_s": round(elems / span / 1e9, 3), "peak_hbm_bytes": srv.peak_used,
            "mean_batch": round(sum(sizes) / max(len(sizes), 1), 2), "max_batch": max(sizes, default=0)}


def _batches(done: List[Request]):
    by = collections.defaultdict(list)
    for r in done:
        by[r.batch].append(r)
    return list(by.values())
