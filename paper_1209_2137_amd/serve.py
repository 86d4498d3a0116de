"""Continuous-batching decode server over a resident list pool.

Requests arrive over time; each asks for a set of lists of the pool to be
decoded into the caller's buffer. The loop admits arrived requests while
the output arena (an HBM budget) has room, groups every admitted request
not yet launched into one micro-batch, and launches it (one batched
decode launch) on the next free stream, so batches overlap on the device
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
    n: int = 0               # output integers
    out_off: int = -1        # start in the arena (elements)
    launched: float = -1.0
    done: float = -1.0
    offsets: list = field(default_factory=list)


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


class Server:
    """Continuous batching of decode requests over a ListPool."""

    def __init__(self, pool, arena_elems: int, budget_bytes: int = 64 << 30, streams: int = 4,
                 max_batch: int = 512, tune=None):
        import torch
        self.pool = pool
        self.arena_elems = int(min(arena_elems, budget_bytes // 4))
        self.arena = torch.empty(self.arena_elems + 4, dtype=torch.int32, device="cuda")
        self.alloc = RingArena(self.arena_elems)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]  # default priority
        self.tune = dict(tune or {})
        self.tune.setdefault("use_graph", 0)
        self.plans = [BatchPlan(pool.pool, self.arena, [], tune=self.tune) for _ in range(streams)]
        self.events = [torch.cuda.Event() for _ in range(streams)]
        self.busy = [None] * streams
        self.max_batch = max_batch

    def _launch(self, slot, batch, now):
        rows = []
        for r in batch:
            rows.extend(self.pool.rows_for(r.lists, [r.out_off + o for o in r.offsets]))
            r.launched = now
        st = self.streams[slot]
        self.plans[slot].replan(self.pool.pool, self.arena, rows, stream=st)
        self.plans[slot].decode(stream=st)
        self.events[slot].record(st)
        self.busy[slot] = batch

    def run(self, times, reqs, check=None, idle_sleep=20e-6):
        """Serves requests with arrival times `times` (seconds) and list ids
        `reqs`. check(request, arena) is called on completion (optional).
        Returns the list of completed Request objects."""
        lens = self.pool.lens
        pending = collections.deque()
        for i, (t, ids) in enumerate(zip(times, reqs)):
            ids = np.asarray(ids, dtype=np.int64)
            r = Request(i, float(t), ids)
            offs, o = [], 0
            for li in ids:
                offs.append(o)
                o += (int(lens[li]) + 3) & ~3
            r.offsets, r.n = offs, o
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
                        if check is not None:
                            check(r, self.arena)
                        self.alloc.free(r.out_off)
                        done.append(r)
                    self.busy[s] = None
                    progressed = True
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                start = self.alloc.alloc(waiting[0].n)
                if start is None:
                    break
                r = waiting.popleft()
                r.out_off = start
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
    ints = sum(r.n for r in done)
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
