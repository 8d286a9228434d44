"""Serving loop: continuous batching of Hough-transform requests on one GPU.

Each request brings one image (uint8 edge map or float32, any size) and gets
its four quadrant Hough images back, left on the device.  The loop:

1. plans every arriving request on the library's native planner pool
   (``fht_planner``: C++ worker threads that also copy the plan's programs to
   the device, so the loop only submits and polls and never shares the GIL
   with planning), with an LRU cache of plans by shape, dtype and split;
2. admits requests first come, first served once their plans are made (a
   request whose plan is ready does not wait for an earlier one's), while
   their device footprint (image, outputs, workspace and work-list tables)
   fits the HBM budget; a request larger than the whole budget is rejected,
   not crashed;
3. whenever one of its launch slots (streams x depth) is free, launches the
   admitted requests of the oldest one's dtype (up to the batch limits) as one
   batch on that slot's stream: image uploads, the batch's tables and its
   fused passes, with no device allocation or synchronisation beyond torch's
   caching allocator.  Requests that arrive while batches run join the next
   free slot, so their work overlaps with the batches already on the device;
4. polls the batches' completion events, records each request's latency
   (arrival to observed completion) and returns its budget.

A batch whose enqueue fails is retried request by request; a request that
fails on its own is marked failed and the loop goes on.  The clock and the
executor are parameters, so the scheduling logic runs on the CPU under a fake
clock in tests, and on the GPU with ``GpuExecutor`` and the wall clock.
"""
from __future__ import annotations

import threading
import time
from collections import OrderedDict, deque
from dataclasses import dataclass
from typing import Any, Sequence

import numpy as np

from . import _binding as B

_IN_BYTES = {"u8": 1, "f32": 4, "f64": 8}
_OUT_BYTES = {"u8": 4, "f32": 4, "f64": 8}


def _align(n: int, a: int = 256) -> int:
    return (n + a - 1) // a * a


def _kind(image) -> str:
    name = str(image.dtype)
    if "uint8" in name:
        return "u8"
    if "float32" in name:
        return "f32"
    if "float64" in name:
        return "f64"
    raise ValueError(f"unsupported image dtype {image.dtype}")


# Pending plans the serving loop polls per round (oldest first).
_POLL_WINDOW = 64


@dataclass(eq=False)
class Request:
    """One transform request; the server fills in everything after `split`."""
    rid: int
    image: Any                 # torch tensor (host, ideally pinned, or device) or numpy array
    arrival: float = 0.0       # seconds on the server's clock
    split: str = "S"
    status: str = "new"        # planned, admitted, running, done, rejected, failed
    error: str | None = None
    plan: Any = None
    footprint: int = 0
    t_planned: float | None = None
    t_admit: float | None = None
    t_launch: float | None = None
    t_done: float | None = None
    batch: int | None = None
    out: Any = None            # flat device output (kept when the server keeps outputs)

    @property
    def rows(self) -> int:
        return int(self.image.shape[0])

    @property
    def cols(self) -> int:
        return int(self.image.shape[1])

    @property
    def pixels(self) -> int:
        return self.rows * self.cols

    @property
    def kind(self) -> str:
        return _kind(self.image)

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.arrival

    def result(self) -> list:
        """The four quadrant images, (W, H) device tensors."""
        if self.status != "done" or self.out is None:
            raise RuntimeError(f"request {self.rid} has no result ({self.status})")
        return self.plan.split_out(self.out)


def footprint(plan, kind: str) -> int:
    """Device bytes a request holds while it runs: image, outputs, workspace,
    and a bound on its share of the batch tables."""
    px = plan.rows * plan.cols
    return (px * _IN_BYTES[kind] + plan.out_elems * _OUT_BYTES[kind] + plan.ws_bytes
            + px + (64 << 10))


class PlanFuture:
    """A plan being made by the native planner pool (``done()`` polls it,
    ``result()`` waits for it), shared by every request of its shape."""

    def __init__(self, cache: "PlanCache", ticket: int, args: tuple):
        self._cache, self._ticket, self._args = cache, ticket, args
        self._plan = None
        self._error: Exception | None = None

    def done(self) -> bool:
        with self._cache._lock:
            if self._plan is None and self._error is None:
                if not self._cache._pool:
                    self._error = RuntimeError("the plan cache was closed before this plan was taken")
                    return True
                state, h, st = B.fht_planner_poll(self._cache._pool, self._ticket)
                if state == 0:
                    return False
                if state < 0:
                    self._error = RuntimeError(f"planner ticket {self._ticket} is unknown")
                elif st != 0:
                    self._error = B.FhtError(st, "fht_plan_create")
                else:
                    rows, cols, kind, split = self._args
                    self._plan = B.Plan.adopt(h, rows, cols, kind, split)
            return True

    def result(self):
        while not self.done():
            time.sleep(20e-6)
        if self._error is not None:
            raise self._error
        return self._plan


class PlanCache:
    """Plans made by the library's native planner pool, cached (LRU) by shape,
    dtype and split.  With ``device`` >= 0 the pool also copies each plan's
    programs to that HIP device, on its own threads."""

    def __init__(self, threads: int = 8, capacity: int = 256, schedule: dict | None = None,
                 device: int = -1):
        self._pool = B.fht_planner_create(max(1, min(int(threads), 256)), int(device))
        self._lru: OrderedDict = OrderedDict()
        self._lock = threading.Lock()
        self._capacity = capacity
        self._schedule = B.fht_schedule(**schedule) if schedule else None

    def get(self, rows: int, cols: int, kind: str, split: str) -> PlanFuture:
        key = (rows, cols, kind, split)
        with self._lock:
            fut = self._lru.get(key)
            if fut is not None:
                self._lru.move_to_end(key)
                return fut
            ticket = B.fht_planner_submit(self._pool, rows, cols, B._dtype_code(kind),
                                          B._split_code(split), 15, self._schedule)
            fut = PlanFuture(self, ticket, key)
            self._lru[key] = fut
            while len(self._lru) > self._capacity:
                self._lru.popitem(last=False)
            return fut

    def close(self) -> None:
        """Stops the pool (plans already taken stay valid)."""
        with self._lock:
            pool, self._pool = self._pool, None
        if pool:
            B.fht_planner_destroy(pool)


class WallClock:
    """Seconds since construction; idling yields the CPU briefly."""

    def __init__(self):
        self._t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def sleep_until(self, t: float) -> None:
        while self.now() < t:
            time.sleep(0)

    def idle(self, next_event: float | None) -> None:
        time.sleep(20e-6)


@dataclass(eq=False)
class _Inflight:
    slot: int
    reqs: list
    handle: Any
    bid: int


class GpuExecutor:
    """Runs batches on `streams` HIP streams of one device (default priority)."""

    def __init__(self, device=None, streams: int = 2):
        import torch
        self.torch = torch
        dev = torch.device(device) if device is not None else torch.device("cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self._graveyard: list = []

    @property
    def n_streams(self) -> int:
        return len(self.streams)

    @property
    def plan_device(self) -> int:
        """Device the planner pool copies plan programs to."""
        return self.device.index

    def launch(self, reqs: Sequence[Request], slot: int) -> dict:
        """Enqueues one batch: one device buffer for its images and one for
        its outputs (256-byte aligned slices), the image copies in one call,
        the tables through pinned staging, then the fused passes."""
        torch = self.torch
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            img_off, out_off, ib, ob = [], [], 0, 0
            srcs, held = [], []
            for r in reqs:
                img_off.append(ib)
                ib += _align(r.pixels * _IN_BYTES[r.kind])
                out_off.append(ob)
                ob += _align(r.plan.out_elems * _OUT_BYTES[r.kind])
                img = r.image
                if isinstance(img, np.ndarray):
                    img = torch.from_numpy(img)
                img = img.contiguous()
                held.append(img)
                srcs.append(img.data_ptr())
            imgs = torch.empty(max(ib, 1), dtype=torch.uint8, device=self.device)
            outs = torch.empty(max(ob, 1), dtype=torch.uint8, device=self.device)
            ip, op = imgs.data_ptr(), outs.data_ptr()
            batch = B.Batch.from_pointers([r.plan for r in reqs], [ip + o for o in img_off],
                                          [op + o for o in out_off])
            ws = torch.empty(max(batch.ws_bytes, 1), dtype=torch.uint8, device=self.device)
            tables = torch.empty(batch.tables_bytes, dtype=torch.uint8, device=self.device)
            # pinned staging: the table copy is asynchronous, so the loop never
            # waits here for the batches already on the stream
            staging = torch.empty(batch.tables_bytes, dtype=torch.uint8, pin_memory=True)
            h = {"batch": batch, "imgs": imgs, "outs": outs, "out_off": out_off, "reqs": list(reqs),
                 "held": held, "ws": ws, "tables": tables, "staging": staging}
            try:
                batch.copy_images(srcs, stream)
                batch.upload(tables, stream, staging)
                batch.run(ws, stream)
            except B.FhtError:
                # keep what may already be enqueued alive until the stream passes it
                ev = torch.cuda.Event()
                ev.record(stream)
                h["event"] = ev
                self._graveyard.append(h)
                raise
            ev = torch.cuda.Event()
            ev.record(stream)
            h["event"] = ev
        return h

    def done(self, h) -> bool:
        return h["event"].query()

    def outputs(self, h) -> list:
        """Each request's flat output: a view of the batch's output buffer
        (which it keeps alive)."""
        outs, res = h["outs"], []
        for r, o in zip(h["reqs"], h["out_off"]):
            n = r.plan.out_elems * _OUT_BYTES[r.kind]
            res.append(outs[o:o + n].view(r.plan.out_dtype))
        return res

    def release(self, h) -> None:
        h.clear()
        self._graveyard = [g for g in self._graveyard if not g["event"].query()]

    def next_event(self) -> float | None:
        return None


class Server:
    """Continuous-batching server over an executor (see the module docstring).

    hbm_budget        device bytes the admitted requests may hold together
    max_batch_images  requests per batch at most
    max_batch_px      input pixels per batch at most (a single larger request
                      still runs, alone)
    depth             batches in flight per stream
    keep_outputs      keep each request's device output (else it is dropped
                      when the request completes)
    """

    def __init__(self, executor, hbm_budget: int, max_batch_images: int = 64,
                 max_batch_px: int = 32 << 20, depth: int = 2, plan_threads: int = 8,
                 plan_cache: int = 256, clock=None, keep_outputs: bool = True,
                 schedule: dict | None = None):
        self.executor = executor
        self.budget = int(hbm_budget)
        self.max_batch_images = max(1, int(max_batch_images))
        self.max_batch_px = int(max_batch_px)
        self.depth = max(1, int(depth))
        self.clock = clock or WallClock()
        self.keep_outputs = keep_outputs
        self.plans = PlanCache(plan_threads, plan_cache, schedule,
                               getattr(executor, "plan_device", -1))
        self.in_use = 0
        self.peak_in_use = 0
        self.peak_running = 0
        self.batches = 0
        self.batch_sizes: list = []

    # -- scheduling steps -------------------------------------------------

    def _release(self, r: Request) -> None:
        self.in_use -= r.footprint

    def _finish(self, r: Request, status: str, now: float, error: str | None = None) -> None:
        r.status, r.t_done, r.error = status, now, error

    def _launch(self, group: list, slot: int, now: float) -> None:
        bid = self.batches
        self.batches += 1
        try:
            h = self.executor.launch(group, slot)
        except B.FhtError as e:
            if len(group) == 1:
                r = group[0]
                self._finish(r, "failed", now, str(e))
                self._release(r)
                return
            for r in group:  # retry one by one; only a request failing alone fails
                self._launch([r], slot, now)
            return
        for r in group:
            r.status, r.t_launch, r.batch = "running", now, bid
        self.batch_sizes.append(len(group))
        self.inflight.append(_Inflight(slot, list(group), h, bid))

    def _take_group(self) -> list:
        kind = self.admitted[0].kind
        group, px = [], 0
        for r in self.admitted:
            if r.kind != kind:
                continue
            if group and (len(group) >= self.max_batch_images or px + r.pixels > self.max_batch_px):
                break
            group.append(r)
            px += r.pixels
        for r in group:
            self.admitted.remove(r)
        return group

    def run(self, requests: Sequence[Request]) -> list:
        """Serve `requests` (each with its arrival time on this server's clock)
        until every one is done, rejected or failed; returns them."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        nxt = 0
        planning: deque = deque()
        ready: deque = deque()
        self.admitted: deque = deque()
        self.inflight: list = []
        clock = self.clock
        n_slots = self.executor.n_streams * self.depth
        while nxt < len(reqs) or planning or ready or self.admitted or self.inflight:
            now = clock.now()
            busy = False
            # arrivals -> the planner pool
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                nxt += 1
                try:
                    kind = r.kind
                    if r.rows < 1 or r.cols < 1:
                        raise ValueError("empty image")
                    planning.append((r, self.plans.get(r.rows, r.cols, kind, r.split)))
                except ValueError as e:
                    self._finish(r, "rejected", now, str(e))
                busy = True
            # planned -> admission queue, as plans complete (in arrival order
            # among those completed together): a large plan still being made
            # holds up no request behind it.  The oldest _POLL_WINDOW pending
            # plans are polled per round.
            if planning:
                waiting = deque()
                for i, (r, fut) in enumerate(planning):
                    if i >= _POLL_WINDOW or not fut.done():
                        waiting.append((r, fut))
                        continue
                    busy = True
                    try:
                        r.plan = fut.result()
                    except (B.FhtError, ValueError) as e:
                        self._finish(r, "rejected", now, str(e))
                        continue
                    r.t_planned = now
                    r.footprint = footprint(r.plan, r.kind)
                    if r.footprint > self.budget:
                        self._finish(r, "rejected", now, "larger than the HBM budget")
                        continue
                    r.status = "planned"
                    ready.append(r)
                planning = waiting
            # completions
            for f in list(self.inflight):
                if self.executor.done(f.handle):
                    outs = (self.executor.outputs(f.handle) if self.keep_outputs else None) \
                        or [None] * len(f.reqs)
                    for r, o in zip(f.reqs, outs):
                        self._finish(r, "done", now)
                        r.out = o if self.keep_outputs else None
                        self._release(r)
                    self.executor.release(f.handle)
                    self.inflight.remove(f)
                    busy = True
            # admission, first come first served
            while ready and self.in_use + ready[0].footprint <= self.budget:
                r = ready.popleft()
                self.in_use += r.footprint
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                r.status, r.t_admit = "admitted", now
                self.admitted.append(r)
                busy = True
            # launches into free slots
            while self.admitted:
                load = [0] * self.executor.n_streams
                for f in self.inflight:
                    load[f.slot] += 1
                slot = int(np.argmin(load))
                if load[slot] >= self.depth or sum(load) >= n_slots:
                    break
                self._launch(self._take_group(), slot, now)
                busy = True
            self.peak_running = max(self.peak_running, sum(len(f.reqs) for f in self.inflight))
            if not busy:
                events = [e for e in (self.executor.next_event(),
                                      reqs[nxt].arrival if nxt < len(reqs) else None)
                          if e is not None]
                clock.idle(min(events) if events and not planning else None)
        return list(requests)

    def close(self) -> None:
        self.plans.close()


def summarize(reqs: Sequence[Request]) -> dict:
    """Latency percentiles (ms, arrival to completion) and throughput."""
    done = [r for r in reqs if r.status == "done"]
    out = {"requests": len(reqs), "done": len(done),
           "rejected": sum(r.status == "rejected" for r in reqs),
           "failed": sum(r.status == "failed" for r in reqs)}
    if not done:
        return out
    lat = np.array([r.latency for r in done]) * 1e3
    span = max(r.t_done for r in done) - min(r.arrival for r in reqs)
    px = sum(r.pixels for r in done)
    out.update({
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "mean_ms": round(float(lat.mean()), 3),
        "span_s": round(span, 4),
        "mpixels": round(px / 1e6, 2),
        "mpixel_per_s": round(px / span / 1e6, 1) if span > 0 else None,
        "req_per_s": round(len(done) / span, 1) if span > 0 else None,
    })
    return out
