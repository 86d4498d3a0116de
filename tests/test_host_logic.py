"""Host-side logic that needs no GPU: the serving arena allocator and the
batch planner's registry checks (through the C library, no device work)."""
import ctypes
import random

import numpy as np

import paper_1209_2137_amd as wp
from paper_1209_2137_amd import datagen
from paper_1209_2137_amd.serve import RingArena


def test_ring_arena_never_overlaps_and_stays_in_bounds():
    rng = random.Random(1)
    for trial in range(150):
        size = rng.choice([64, 100, 1000, 4096])
        arena = RingArena(size)
        occ = np.zeros(size, dtype=bool)
        live = []
        for _ in range(400):
            if live and rng.random() < 0.45:
                k = rng.randrange(len(live)) if rng.random() < 0.3 else 0  # mostly in order
                st, n = live.pop(k)
                arena.free(st)
                occ[st:st + n] = False
            else:
                n = rng.randint(1, size // 3)
                st = arena.alloc(n)
                if st is not None:
                    n4 = (n + 3) & ~3
                    assert 0 <= st and st + n4 <= size and st % 4 == 0
                    assert not occ[st:st + n4].any()
                    occ[st:st + n4] = True
                    live.append((st, n4))
        for st, _ in list(live):
            arena.free(st)
        assert not arena.blocks and arena.alloc(size) == 0


def test_ring_arena_fills_completely_in_fifo_use():
    arena = RingArena(64)
    starts = [arena.alloc(16) for _ in range(4)]
    assert starts == [0, 16, 32, 48] and arena.alloc(4) is None
    arena.free(16)                 # out of order: nothing comes back yet
    assert arena.alloc(4) is None
    arena.free(0)                  # now [0, 32) is free
    assert arena.alloc(32) == 0


def test_poisson_arrivals_shape():
    times, reqs = datagen.poisson_arrivals(rate=2000.0, duration=2.0, pool=1000, seed=6)
    assert 3500 < len(times) < 4500 and (np.diff(times) > 0).all()
    assert all(1 <= len(r) <= 32 and r.max() < 1000 for r in reqs)
