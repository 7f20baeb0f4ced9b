"""Continuous-batching serving loop for camera-frame requests of mixed resolution.

Requests (one 3xSxS image each) arrive on an open-loop trace.  The scheduler
keeps one FIFO queue per resolution S and a fixed number of execution slots
(one HIP stream each).  Whenever a slot is free it takes the bucket whose
oldest request has waited longest, forms a batch of everything waiting there
(up to ``max_batch``, padded to a power of two so each (batch, S) shape
recurs), reserves the batch's device bytes (activation arena + input + output
from ``dn_arena_bytes``) from an HBM budget and launches it.  Batches on
different slots run concurrently on the GPU; requests that arrive while
others are in flight are admitted as soon as a slot and budget free up.
Completion is detected by polling a per-batch event (no blocking sync), which
frees the slot and the budget and stamps every request's completion time.

With ``fixed_slots`` each slot owns one region of the pool sized for the
largest batch of the largest bucket, so a (slot, batch, size) always runs on
the same addresses and the library replays the forward's captured graph (with
the tiles the autotuner chose for that batch and size) instead of launching
its kernels one by one; the budget is then the slots' regions.  Each batch's
device interval (events at its first and last command) is kept, so that the
overlap of batches on the GPU can be measured (``device_overlap``).

Weights are resident (loaded once), activations live in arenas carved from
one pre-allocated device pool, and each image crosses PCIe once in and its
output once out (the placement of Sec. 3.2 of the paper applied per frame).

The scheduler core is device-independent: ``Executor`` is the interface the
GPU executor (``DnExecutor``, the library through ``dn.py``) and the tests'
fake executor implement.
"""
from __future__ import annotations

import bisect
import gc
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


# ------------------------------------------------------------------ memory budget


class PoolAllocator:
    """First-fit allocator over [0, capacity) with 256-byte alignment; the
    capacity is the HBM budget for in-flight batches."""

    ALIGN = 256

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self._free = [(0, self.capacity)]  # sorted (offset, size)
        self.in_use = 0

    @classmethod
    def _round(cls, n: int) -> int:
        return (int(n) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    def alloc(self, nbytes: int) -> Optional[int]:
        n = self._round(max(nbytes, 1))
        for i, (off, size) in enumerate(self._free):
            if size >= n:
                if size == n:
                    del self._free[i]
                else:
                    self._free[i] = (off + n, size - n)
                self.in_use += n
                return off
        return None

    def free(self, off: int, nbytes: int) -> None:
        n = self._round(max(nbytes, 1))
        self.in_use -= n
        i = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(i, (off, n))
        # coalesce with neighbours
        merged = []
        for o, s in self._free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self._free = merged


# ------------------------------------------------------------------ requests and batches


@dataclass
class Request:
    rid: int
    size: int                 # square side S
    arrival: float            # seconds on the scheduler clock
    completion: Optional[float] = None
    error: Optional[str] = None
    output: Optional[np.ndarray] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.completion is None else self.completion - self.arrival


@dataclass
class Batch:
    slot: int
    size: int
    padded: int
    requests: List[Request]
    offset: int
    nbytes: int
    launched: float
    handle: object = None


class Executor:
    """What the scheduler needs from a device back end."""

    n_slots: int = 1

    def batch_bytes(self, batch: int, size: int) -> int:
        raise NotImplementedError

    def launch(self, slot: int, reqs: Sequence[Request], padded: int, size: int, offset: int):
        """Enqueue the batch (inputs H2D, forward, outputs D2H) on the slot; return a handle."""
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle, reqs: Sequence[Request]) -> None:
        """Called once done(handle): store per-request outputs (or raise)."""
        raise NotImplementedError


def next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


@dataclass
class ServeStats:
    completed: int
    rejected: int
    failed: int
    images_per_s: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    max_inflight: int
    batches: int
    wall_s: float
    extra: Dict[str, float] = field(default_factory=dict)

    def as_dict(self):
        d = dict(self.__dict__)
        d.update(d.pop("extra"))
        return d


class Scheduler:
    """Continuous batching over resolution buckets with HBM-budget admission."""

    def __init__(self, executor: Executor, budget_bytes: int, sizes: Sequence[int],
                 max_batch: int = 64, pad_pow2: bool = True, bucketed: bool = True,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.pool = PoolAllocator(budget_bytes)
        self.sizes = tuple(sizes)
        self.max_batch = int(max_batch)
        self.pad_pow2 = pad_pow2
        self.bucketed = bucketed
        self.clock = clock
        self.queues: Dict[int, deque] = {s: deque() for s in self.sizes}
        self.fifo: deque = deque()  # used when not bucketed (plain FIFO path)
        self.free_slots = list(range(executor.n_slots))
        self.inflight: List[Batch] = []
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self.batches = 0
        self.batch_sizes: List[int] = []
        self.max_inflight = 0

    # -- arrivals
    def submit(self, req: Request) -> None:
        if req.size not in self.queues:
            req.error = "unsupported size %d" % req.size
            self.rejected.append(req)
            return
        if self.ex.batch_bytes(1, req.size) > self.pool.capacity:
            req.error = "request larger than the HBM budget"
            self.rejected.append(req)
            return
        if self.bucketed:
            self.queues[req.size].append(req)
        else:
            self.fifo.append(req)

    def pending(self) -> int:
        return sum(len(q) for q in self.queues.values()) + len(self.fifo)

    # -- completions
    def poll(self) -> int:
        n = 0
        still = []
        for b in self.inflight:
            if self.ex.done(b.handle):
                now = self.clock()
                try:
                    self.ex.finish(b.handle, b.requests)
                except Exception as e:  # a failed batch fails its own requests only
                    for r in b.requests:
                        r.error = "batch failed: %s" % e
                for r in b.requests:
                    r.completion = now
                    self.done.append(r)
                self.pool.free(b.offset, b.nbytes)
                self.free_slots.append(b.slot)
                n += 1
            else:
                still.append(b)
        self.inflight = still
        return n

    # -- admission
    def _pick(self):
        """(size, candidate requests, queue they come from) of the bucket whose
        oldest request has waited longest, or None."""
        if not self.bucketed:
            if not self.fifo:
                return None
            return self.fifo[0].size, [self.fifo[0]], self.fifo
        best = None
        for s, q in self.queues.items():
            if q and (best is None or q[0].arrival < self.queues[best][0].arrival):
                best = s
        if best is None:
            return None
        q = self.queues[best]
        return best, list(q)[: self.max_batch], q

    def _padded(self, n: int) -> int:
        return min(next_pow2(n) if self.pad_pow2 else n, self.max_batch)

    def admit(self) -> int:
        launched = 0
        while self.free_slots:
            pick = self._pick()
            if pick is None:
                break
            size, reqs, queue = pick
            padded = self._padded(len(reqs))
            nbytes = self.ex.batch_bytes(padded, size)
            off = self.pool.alloc(nbytes)
            # Nothing in flight means no completion will free memory: take
            # fewer requests (halving) until the padded batch fits.  One image
            # always fits an idle pool (submit() rejected anything larger).
            while off is None and not self.inflight and len(reqs) > 1:
                reqs = reqs[: (len(reqs) + 1) // 2]
                padded = self._padded(len(reqs))
                nbytes = self.ex.batch_bytes(padded, size)
                off = self.pool.alloc(nbytes)
            if off is None:
                break  # over budget: wait for completions
            for _ in range(len(reqs)):
                queue.popleft()
            slot = self.free_slots.pop(0)
            b = Batch(slot, size, padded, reqs, off, nbytes, self.clock())
            try:
                b.handle = self.ex.launch(slot, reqs, padded, size, off)
            except Exception as e:
                self.pool.free(off, nbytes)
                self.free_slots.append(slot)
                for r in reqs:
                    r.error = "launch failed: %s" % e
                    r.completion = self.clock()
                    self.done.append(r)
                continue
            self.inflight.append(b)
            self.batches += 1
            self.batch_sizes.append(len(reqs))
            self.max_inflight = max(self.max_inflight, len(self.inflight))
            launched += 1
        return launched

    # -- open-loop driver
    def run(self, reqs: Sequence[Request], idle_sleep: float = 0.0, hold_gc: bool = True) -> ServeStats:
        """Feed requests at their arrival times (scheduler clock relative to the
        start) and run until every request completed or was rejected.  With
        hold_gc, Python's cyclic garbage collector is paused for the run (and
        run once after it): a full collection over the run's objects would
        stall the loop for tens of milliseconds."""
        if hold_gc and gc.isenabled():
            gc.disable()
            try:
                return self.run(reqs, idle_sleep, hold_gc=False)
            finally:
                gc.enable()
                gc.collect()
        order = sorted(reqs, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in order:
            r.arrival += t0
        i = 0
        while i < len(order) or self.pending() or self.inflight:
            now = self.clock()
            while i < len(order) and order[i].arrival <= now:
                self.submit(order[i])
                i += 1
            self.poll()
            self.admit()
            if idle_sleep and not self.inflight and i < len(order) and order[i].arrival > self.clock():
                time.sleep(min(idle_sleep, order[i].arrival - self.clock()))
        ok = [r for r in self.done if r.error is None]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        first = min(r.arrival for r in order) if order else t0
        last = max((r.completion for r in ok), default=first)
        wall = max(last - first, 1e-9)
        for r in order:  # back to trace-relative times
            r.arrival -= t0
            if r.completion is not None:
                r.completion -= t0
        return ServeStats(completed=len(ok), rejected=len(self.rejected),
                          failed=len(self.done) - len(ok), images_per_s=len(ok) / wall,
                          p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                          mean_batch=float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
                          max_inflight=self.max_inflight, batches=self.batches, wall_s=wall)


# ------------------------------------------------------------------ GPU executor


class DnExecutor(Executor):
    """Runs batches through libdn (``dn_forward_arena``) on per-slot streams.

    Device memory: one pool of ``budget_bytes`` allocated up front; every batch
    gets a contiguous region [arena | input NCHW FP32 | output NCHW FP32]
    carved by the scheduler's allocator.  With ``fixed_slots`` the pool is
    instead n_slots regions of ``slot_bytes()`` (budget_bytes is ignored), and
    a batch always runs at the start of its slot's region, so its addresses
    repeat and the net's captured graph for (batch, size) on that slot is
    replayed.  Host images come from ``image_of`` (request -> float32
    [3, S, S], numpy or a pinned torch tensor): numpy images are copied into
    a per-slot pinned staging buffer and sent with one H2D copy per batch,
    pinned tensors with one H2D copy each.  Region sizes come from the net's
    plans when the executor is created: tune the net first.
    """

    def __init__(self, net, torch, budget_bytes: int, n_slots: int, image_of: Callable[[Request], np.ndarray],
                 max_batch: int, max_size: int, keep_outputs: bool = True, fixed_slots: bool = False,
                 sizes: Sequence[int] = ()):
        self.net = net
        self.torch = torch
        self.n_slots = n_slots
        self.image_of = image_of
        self.keep = keep_outputs
        self.fixed = fixed_slots
        self._layout = {}
        # an input_u8 net takes its frames as 8-bit pixels
        self.in_u8 = bool(getattr(net, "input_u8", False))
        self.in_dtype = torch.uint8 if self.in_u8 else torch.float32
        self.in_bytes = 1 if self.in_u8 else 4
        if fixed_slots:
            self.region = max(self._bytes(max_batch, s) for s in (sizes or (max_size,)))
            budget_bytes = self.region * n_slots
        self.pool = torch.empty(budget_bytes, dtype=torch.uint8, device="cuda")
        self.base = self.pool.data_ptr()
        self.intervals = []  # (start event, end event, padded batch) of every launched batch
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        c = net.in_c
        self.stage_in = [torch.empty((max_batch, c, max_size, max_size), dtype=self.in_dtype).pin_memory()
                         for _ in range(n_slots)]
        oc, oh, ow = net.output_shape(max_size, max_size)
        self.stage_out = [torch.empty((max_batch * oc * oh * ow,), dtype=torch.float32).pin_memory()
                          for _ in range(n_slots)]

    def _regions(self, batch: int, size: int):
        key = (batch, size)
        if key not in self._layout:
            ab = self.net.arena_bytes(batch, size, size)
            ab = (ab + 255) // 256 * 256
            xb = batch * self.net.in_c * size * size * self.in_bytes
            xb = (xb + 255) // 256 * 256
            oc, oh, ow = self.net.output_shape(size, size)
            yb = batch * oc * oh * ow * 4
            self._layout[key] = (ab, xb, yb, (oc, oh, ow))
        return self._layout[key]

    def _bytes(self, batch: int, size: int) -> int:
        ab, xb, yb, _ = self._regions(batch, size)
        return (ab + xb + yb + 255) // 256 * 256

    def batch_bytes(self, batch: int, size: int) -> int:
        # a fixed slot's whole region: the allocator then hands out whole regions
        return self.region if self.fixed else self._bytes(batch, size)

    def launch(self, slot, reqs, padded, size, offset):
        torch = self.torch
        ab, xb, yb, oshape = self._regions(padded, size)
        s = self.streams[slot]
        c = self.net.in_c
        imgs = [self.image_of(r) for r in reqs]
        # images already in pinned host memory (a capture pipeline's frame
        # buffers) go to the device one copy each; others are gathered into
        # the slot's pinned staging buffer first and sent with one copy
        direct = all(isinstance(im, torch.Tensor) and im.is_pinned() for im in imgs)
        if not direct:
            hx = self.stage_in[slot].view(-1)[: padded * c * size * size].view(padded, c, size, size)
            for j, im in enumerate(imgs):
                hx[j].copy_(torch.from_numpy(im))
            if padded > len(imgs):
                hx[len(imgs):].zero_()
        if self.fixed:
            offset = slot * self.region
        arena = self.base + offset
        x_ptr = arena + ab
        y_ptr = x_ptr + xb
        n = padded * c * size * size
        dx = self.pool.narrow(0, offset + ab, n * self.in_bytes).view(self.in_dtype)
        dy = self.pool.narrow(0, offset + ab + xb, yb).view(torch.float32)
        ho = self.stage_out[slot][: yb // 4]
        with torch.cuda.stream(s):
            t0 = torch.cuda.Event(enable_timing=True)
            t0.record(s)
            if direct:
                dxv = dx.view(padded, c, size, size)
                for j, im in enumerate(imgs):
                    dxv[j].copy_(im, non_blocking=True)
                if padded > len(imgs):
                    dxv[len(imgs):].zero_()
            else:
                dx.copy_(hx.view(-1), non_blocking=True)
            self.net.forward_arena(arena, ab, x_ptr, padded, size, size, y_ptr, s)
            ho.copy_(dy, non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        self.intervals.append((t0, ev, padded))
        return (ev, slot, padded, size, oshape)

    def done(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle, reqs):
        ev, slot, padded, size, (oc, oh, ow) = handle
        if self.keep:
            out = self.stage_out[slot][: padded * oc * oh * ow].view(padded, oc, oh, ow)
            for j, r in enumerate(reqs):
                r.output = out[j].numpy().copy()


def device_overlap(intervals, ref_event) -> Dict[str, float]:
    """Overlap of batches on the GPU from their event timestamps (all events
    complete): each batch's interval runs from the event before its input copy
    to the event after its output copy, in ms after ``ref_event`` (recorded
    before any of them).  Returns the time the GPU held at least one batch
    (busy_ms), the sum of the intervals, their ratio (mean batches in flight
    while busy), the share of busy time with two or more batches in flight,
    and the largest number in flight at once."""
    ev = []
    for t0, t1, _ in intervals:
        a, b = ref_event.elapsed_time(t0), ref_event.elapsed_time(t1)
        ev.append((a, 1))
        ev.append((b, -1))
    if not ev:
        return {"busy_ms": 0.0, "sum_batch_ms": 0.0, "mean_in_flight": 0.0, "overlap_frac": 0.0, "max_in_flight": 0}
    ev.sort(key=lambda e: (e[0], e[1]))  # an end before a start at the same instant
    busy = multi = total = 0.0
    depth = peak = 0
    last = ev[0][0]
    for t, d in ev:
        if depth >= 1:
            busy += t - last
            total += (t - last) * depth
        if depth >= 2:
            multi += t - last
        depth += d
        peak = max(peak, depth)
        last = t
    return {"busy_ms": busy, "sum_batch_ms": total, "mean_in_flight": total / busy if busy else 0.0,
            "overlap_frac": multi / busy if busy else 0.0, "max_in_flight": peak}


def make_requests(trace, count: Optional[int] = None) -> List[Request]:
    n = len(trace.arrival_s) if count is None else min(count, len(trace.arrival_s))
    return [Request(i, int(trace.size[i]), float(trace.arrival_s[i])) for i in range(n)]
