"""Continuous-batching decode server over a resident list pool.

Requests arrive over time; each asks for a set of lists of the pool to be
decoded into a device buffer that the caller owns (the caller hands it over
when the request is admitted and gets it back, filled, on completion). The
loop admits arrived requests while the output bytes of the requests in
flight stay within an HBM budget and the caller has a buffer for them,
groups every admitted request not yet launched into one micro-batch, and
launches it (one batched decode launch, each list straight into its
request's buffer) on the next free stream, so batches overlap on the device
while new requests keep arriving. A request is complete when its batch's
completion event has fired; its latency is completion minus arrival (host
clock, polled).

The device work is the batched decoder of the C library; this module only
schedules it (host bookkeeping, no decoding).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import BatchPlan


@dataclass
class Request:
    rid: int
    arrival: float           # seconds since the start of the run
    lists: np.ndarray        # pool list ids
    n: int = 0               # output elements (lists at 4-aligned offsets)
    ints: int = 0            # integers decoded (the lists' lengths)
    out: object = None       # the caller's device buffer (int32/uint32 tensor, >= n elements)
    launched: float = -1.0
    done: float = -1.0
    offsets: list = field(default_factory=list)  # each list's first element in `out`


class RingArena:
    """Allocations in arrival order from a ring of `size` elements. Each
    allocation is contiguous; space comes back when the oldest live
    allocation is freed (requests finish roughly in order, and an
    out-of-order free waits for its elders)."""

    def __init__(self, size: int):
        self.size = int(size)
        self.blocks = collections.deque()  # [start, n, freed], oldest first
        self.tail = 0                      # end of the newest block

    @property
    def head(self) -> int:
        return self.blocks[0][0] if self.blocks else self.tail

    def alloc(self, n: int):
        n = max(4, (int(n) + 3) & ~3)
        if n > self.size:
            return None
        if not self.blocks:
            return self._place(0, n)
        head = self.head
        if self.tail > head:                    # live data in [head, tail)
            if self.tail + n <= self.size:
                return self._place(self.tail, n)
            if n <= head:                       # wrap: the end of the ring is skipped
                self.blocks.append([self.tail, self.size - self.tail, True])
                return self._place(0, n)
            return None
        # wrapped: live data in [head, size) and [0, tail); free is [tail, head)
        if self.tail + n <= head:
            return self._place(self.tail, n)
        return None

    def _place(self, start, n):
        self.blocks.append([start, n, False])
        self.tail = start + n
        return start

    def free(self, start: int):
        for b in self.blocks:
            if b[0] == start and not b[2]:
                b[2] = True
                break
        else:
            raise KeyError(start)
        while self.blocks and self.blocks[0][2]:
            self.blocks.popleft()
        if not self.blocks:
            self.tail = 0


class ArenaBuffers:
    """A caller's output buffers carved from one device tensor it owns (a
    ring): get(request) returns a view of at least request.n elements or
    None when the ring is full; put(request) gives the space back."""

    def __init__(self, arena):
        self.arena = arena
        self.ring = RingArena(arena.numel() - 4)
        self.start = {}

    def get(self, r):
        s = self.ring.alloc(r.n)
        if s is None:
            return None
        self.start[r.rid] = s
        return self.arena[s:s + max(4, (r.n + 3) & ~3)]

    def put(self, r):
        self.ring.free(self.start.pop(r.rid))


class CheckingCaller:
    """A caller that owns one zeroed device arena, hands out buffers from
    it (get) and checks every completed request (done) against the pool's
    resident input values on a stream of its own: the request's buffer must
    equal its lists' values, each list zero-padded to 4 elements as the
    server lays them out. The buffer is zeroed again and given back once the
    check has run. finish() waits for the checks and returns the number of
    wrong elements."""

    def __init__(self, pool, arena_elems: int, device="cuda"):
        import torch
        if pool.values is None:
            raise ValueError("checking needs the pool's input values")
        self.pool = pool
        self.arena = torch.zeros(int(arena_elems) + 4, dtype=torch.int32, device=device)
        self.bufs = ArenaBuffers(self.arena)
        self.stream = torch.cuda.Stream()  # default priority
        self.bad = torch.zeros(1, dtype=torch.int64, device=device)
        self.pending = collections.deque()
        self.checked = 0

    def _reap(self):
        while self.pending and self.pending[0][0].query():
            _, r = self.pending.popleft()
            self.bufs.put(r)
            self.checked += 1

    def get(self, r):
        self._reap()
        return self.bufs.get(r)

    def done(self, r):
        import torch
        vals = self.pool.values
        rows = self.pool.rows
        with torch.cuda.stream(self.stream):
            want = torch.cat([vals[rows[li][2]:rows[li][2] + ((rows[li][3] + 3) & ~3)] for li in r.lists])
            got = r.out[:r.n]
            self.bad += (got != want).sum()
            got.zero_()
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.pending.append((ev, r))

    def finish(self) -> int:
        self.stream.synchronize()
        self._reap()
        return int(self.bad.item())


class Server:
    """Continuous batching of decode requests over a ListPool, into caller
    buffers, under an HBM budget for the output bytes in flight."""

    def __init__(self, pool, budget_bytes: int = 64 << 30, streams: int = 4, max_batch: int = 512, tune=None):
        import torch
        self.pool = pool
        self.budget_bytes = int(budget_bytes)
        self.in_flight_bytes = 0
        self.peak_bytes = 0
        self.streams = [torch.cuda.Stream() for _ in range(streams)]  # default priority
        self.tune = dict(tune or {})
        self.tune.setdefault("use_graph", 0)
        self.plans = [BatchPlan(pool.pool, None, [], tune=self.tune) for _ in range(streams)]
        self.events = [torch.cuda.Event() for _ in range(streams)]
        self.busy = [None] * streams
        self.max_batch = max_batch
        self.waited_for_budget = 0
        self.waited_for_buffer = 0

    def _launch(self, slot, batch, now):
        rows = []
        for r in batch:
            base = r.out.data_ptr()
            for li, o in zip(r.lists, r.offsets):
                co, cw, _, n, codec = self.pool.rows[li]
                rows.append((co, cw, 0, n, codec, base + 4 * o))
            r.launched = now
        st = self.streams[slot]
        self.plans[slot].replan(self.pool.pool, None, rows, stream=st)
        self.plans[slot].decode(stream=st)
        self.events[slot].record(st)
        self.busy[slot] = batch

    def run(self, times, reqs, get_out, on_done=None, idle_sleep=20e-6):
        """Serves requests with arrival times `times` (seconds) and list ids
        `reqs`. get_out(request) returns the caller's buffer for it (a
        device tensor of at least request.n elements) or None if the caller
        has none free yet (the request then waits); on_done(request) is
        called when its output is complete (the caller checks and takes the
        buffer back). Returns the list of completed Request objects."""
        lens = self.pool.lens
        pending = collections.deque()
        for i, (t, ids) in enumerate(zip(times, reqs)):
            ids = np.asarray(ids, dtype=np.int64)
            r = Request(i, float(t), ids)
            offs, o = [], 0
            for li in ids:
                offs.append(o)
                o += (int(lens[li]) + 3) & ~3
            r.offsets, r.n, r.ints = offs, o, int(sum(int(lens[li]) for li in ids))
            if 4 * r.n > self.budget_bytes:
                raise ValueError(f"request {i} needs {4 * r.n} output bytes, beyond the budget")
            pending.append(r)
        waiting = collections.deque()
        admitted = collections.deque()
        done = []
        total = len(pending)
        t0 = time.perf_counter()
        while len(done) < total:
            now = time.perf_counter() - t0
            progressed = False
            for s in range(len(self.streams)):
                b = self.busy[s]
                if b is not None and self.events[s].query():
                    tdone = time.perf_counter() - t0
                    for r in b:
                        r.done = tdone
                        self.in_flight_bytes -= 4 * r.n
                        if on_done is not None:
                            on_done(r)
                        done.append(r)
                    self.busy[s] = None
                    progressed = True
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                r = waiting[0]
                if self.in_flight_bytes + 4 * r.n > self.budget_bytes:
                    self.waited_for_budget += 1
                    break
                out = get_out(r)
                if out is None:
                    self.waited_for_buffer += 1
                    break
                if out.numel() < r.n:
                    raise ValueError(f"request {r.rid}: the caller's buffer holds {out.numel()} < {r.n} elements")
                waiting.popleft()
                r.out = out
                self.in_flight_bytes += 4 * r.n
                self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
                admitted.append(r)
            if admitted:
                for s in range(len(self.streams)):
                    if self.busy[s] is None:
                        batch = [admitted.popleft() for _ in range(min(self.max_batch, len(admitted)))]
                        self._launch(s, batch, now)
                        progressed = True
                        break
            if not progressed:
                nxt = pending[0].arrival - (time.perf_counter() - t0) if pending else 0.0
                time.sleep(min(max(nxt, 0.0), idle_sleep) if nxt > 0 else idle_sleep)
        self.wall = time.perf_counter() - t0
        return done

    def close(self):
        for p in self.plans:
            p.free()


def summarize(done, wall):
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    ints = sum(r.ints for r in done)
    return {
        "requests": len(done),
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "max_ms": float(lat.max()) if len(lat) else None,
        "mean_ms": float(lat.mean()) if len(lat) else None,
        "wall_s": wall,
        "gints_per_s": ints / wall / 1e9 if wall > 0 else None,
        "mean_lists_per_request": float(np.mean([len(r.lists) for r in done])) if done else None,
    }
