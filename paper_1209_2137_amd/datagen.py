"""Seeded synthetic inputs for the decoder workloads.

This module only draws numbers: sorted uint32 arrays, gap sequences and list
lengths. It holds none of the codec's arithmetic (no delta coding, no bit
widths, no packing), so both the CPU oracle and the GPU path may consume it.

All generators use numpy's PCG64 (``numpy.random.default_rng(seed)``).

Workloads (the shapes follow the paper's synthetic and posting-list data:
Section 6.4, synthetic data sets, ClusterData and Uniform; Section 6.5,
realistic data sets, posting lists):

* ``single_geometric``   x_1 ~ U[0,1000), gaps ~ Geom(mean) on {1,2,...}.
* ``cluster_sorted``     distinct sorted values from a recursive-cluster
                         splitter (dense and sparse stretches mixed).
* ``uniform_sorted``     distinct sorted values uniform in [0, 2^32).
* ``patched_gaps``       gaps: Geom(mean 4) with Bernoulli(0.1) positions
                         replaced by U[2^8, 2^24) "exceptions"; the array is
                         their running sum modulo 2^32.
* ``posting_lists``      many lists with rank-size Zipf lengths and per-list
                         geometric gaps of log-uniform mean.
* ``poisson_arrivals``   request arrival times and list picks for serving.
"""
from __future__ import annotations

import numpy as np

U32 = np.uint32
MOD32 = 1 << 32


def _wrap_cumsum(gaps: np.ndarray, start: int = 0) -> np.ndarray:
    """Running sum of ``gaps`` (plus ``start``) reduced modulo 2^32.

    uint64 accumulation wraps at 2^64, and 2^32 divides 2^64, so casting the
    uint64 running sum down to uint32 is the exact running sum mod 2^32."""
    acc = np.cumsum(gaps.astype(np.uint64), dtype=np.uint64)
    if start:
        acc += np.uint64(start)
    return acc.astype(U32)


def geometric_gaps(rng: np.random.Generator, n: int, mean: float) -> np.ndarray:
    """n i.i.d. geometric gaps on {1, 2, ...} with the given mean (p = 1/mean)."""
    p = 1.0 / float(mean)
    g = rng.geometric(p, size=n)
    return np.minimum(g, MOD32 - 1).astype(U32)


def single_geometric(n: int = 1 << 20, mean: float = 8.0, seed: int = 1) -> np.ndarray:
    """Sorted uint32: x_1 ~ U[0,1000), then i.i.d. geometric gaps (>= 1)."""
    rng = np.random.default_rng(seed)
    if n == 0:
        return np.zeros(0, dtype=U32)
    x1 = int(rng.integers(0, 1000))
    gaps = geometric_gaps(rng, n, mean)
    gaps[0] = 0
    return _wrap_cumsum(gaps, x1)


def _sorted_distinct_in_ranges(rng, lo, hi, cnt):
    """For each interval [lo_j, hi_j) draw cnt_j distinct sorted integers.

    Uses the order-statistics bijection: cnt values drawn with replacement
    from [0, hi-lo-cnt+1), sorted, plus 0..cnt-1, are distinct and lie in
    [0, hi-lo). Vectorised over all intervals at once."""
    lo = lo.astype(np.int64)
    hi = hi.astype(np.int64)
    cnt = cnt.astype(np.int64)
    total = int(cnt.sum())
    seg = np.repeat(np.arange(len(cnt)), cnt)
    room = (hi - lo - cnt + 1)[seg]
    draws = (rng.random(total) * room).astype(np.int64)
    draws = np.minimum(draws, room - 1)
    # sort inside each segment: the segment index in the high bits keeps
    # segments apart (draws < 2^32 here, segments < 2^31)
    if len(cnt) >= (1 << 31) or (total and int(room.max()) > (1 << 32)):
        raise ValueError("interval too wide for the packed sort key")
    key = (seg.astype(np.int64) << 32) | draws
    key.sort()
    draws = key & np.int64(0xFFFFFFFF)
    starts = np.concatenate(([0], np.cumsum(cnt)[:-1]))
    rank = np.arange(total) - np.repeat(starts, cnt)
    return lo[seg] + draws + rank


def cluster_sorted(n: int = 1 << 26, lo: int = 0, hi: int = 1 << 30,
                   max_depth: int = 20, leaf: int = 64, seed: int = 2) -> np.ndarray:
    """Distinct sorted values from a recursive-cluster splitter.

    Each interval holding cnt > leaf values (and above max_depth levels) is
    split at a point s uniform in [lo + cnt_left, hi - cnt_right] with
    cnt_left = floor(cnt/2): each side keeps room for its distinct values.
    Leaves draw their values uniformly (distinct) inside their interval.
    Vectorised level by level."""
    rng = np.random.default_rng(seed)
    if n > hi - lo:
        raise ValueError("more values than room in the range")
    los = np.array([lo], dtype=np.int64)
    his = np.array([hi], dtype=np.int64)
    cnts = np.array([n], dtype=np.int64)
    done_lo, done_hi, done_cnt = [], [], []
    for _depth in range(max_depth + 1):
        is_leaf = (cnts <= leaf) | (_depth == max_depth)
        done_lo.append(los[is_leaf])
        done_hi.append(his[is_leaf])
        done_cnt.append(cnts[is_leaf])
        keep = ~is_leaf
        if not keep.any():
            break
        los, his, cnts = los[keep], his[keep], cnts[keep]
        nl = cnts // 2
        nr = cnts - nl
        smin = los + nl
        smax = his - nr
        s = smin + (rng.random(len(cnts)) * (smax - smin + 1)).astype(np.int64)
        s = np.minimum(s, smax)
        los = np.concatenate([los, s])
        his = np.concatenate([s, his])
        cnts = np.concatenate([nl, nr])
        # keep intervals in ascending order
        order = np.argsort(los, kind="stable")
        los, his, cnts = los[order], his[order], cnts[order]
    L = np.concatenate(done_lo)
    H = np.concatenate(done_hi)
    C = np.concatenate(done_cnt)
    order = np.argsort(L, kind="stable")
    L, H, C = L[order], H[order], C[order]
    nz = C > 0
    vals = _sorted_distinct_in_ranges(rng, L[nz], H[nz], C[nz])
    return vals.astype(U32)


def uniform_sorted(n: int = 1 << 26, seed: int = 3) -> np.ndarray:
    """n distinct uint32 uniform in [0, 2^32), sorted.

    Draws in rounds, de-duplicating, until at least n distinct values exist,
    then drops a seeded random surplus."""
    rng = np.random.default_rng(seed)
    have = np.zeros(0, dtype=U32)
    while have.size < n:
        need = n - have.size
        extra = rng.integers(0, MOD32, size=need + need // 64 + 16, dtype=np.uint64).astype(U32)
        have = np.unique(np.concatenate([have, extra]))
    if have.size > n:
        drop = rng.choice(have.size, size=have.size - n, replace=False)
        mask = np.ones(have.size, dtype=bool)
        mask[drop] = False
        have = have[mask]
    return have


def patched_gaps(n: int = 1 << 28, mean: float = 4.0, p_exc: float = 0.1,
                 exc_lo: int = 1 << 8, exc_hi: int = 1 << 24, seed: int = 4) -> np.ndarray:
    """Array whose gaps are mostly geometric with rare large 'exceptions'.

    gaps ~ Geom(mean) on {1,...}; each position independently (prob p_exc)
    takes a gap uniform in [exc_lo, exc_hi) instead. Returns the running sum
    of the gaps modulo 2^32 (x_1 = g_1)."""
    rng = np.random.default_rng(seed)
    gaps = geometric_gaps(rng, n, mean)
    where = rng.random(n) < p_exc
    k = int(where.sum())
    gaps[where] = rng.integers(exc_lo, exc_hi, size=k, dtype=np.int64).astype(U32)
    return _wrap_cumsum(gaps)


def zipf_lengths(n_lists: int = 100_000, s: float = 1.1, total: float = 1.2e9,
                 lmin: int = 128, lmax: int = 1 << 22, seed: int = 5) -> np.ndarray:
    """Rank-size Zipf list lengths L_r = clip(C r^-s, lmin, lmax), r = 1..n,
    with C solved (bisection) so that sum L_r ~= total; shuffled by the seed."""
    r = np.arange(1, n_lists + 1, dtype=np.float64)
    w = r ** (-s)

    def tot(c):
        return np.clip(np.floor(c * w), lmin, lmax).sum()

    lo_c, hi_c = 0.0, 1.0
    while tot(hi_c) < total:
        hi_c *= 2.0
        if hi_c > 1e30:
            break
    for _ in range(200):
        mid = 0.5 * (lo_c + hi_c)
        if tot(mid) < total:
            lo_c = mid
        else:
            hi_c = mid
    lens = np.clip(np.floor(hi_c * w), lmin, lmax).astype(np.int64)
    rng = np.random.default_rng(seed)
    rng.shuffle(lens)
    return lens


def posting_lists(n_lists: int = 100_000, total: float = 1.2e9, seed: int = 5,
                  lmin: int = 128, lmax: int = 1 << 22, s: float = 1.1):
    """Posting-list pool: returns (lengths, codec, means, generator-of-arrays).

    codec[i] is 0 (binary packing) or 1 (patched) from a fair seeded coin;
    means[i] = 2^U[1,12]; list i is the running sum (mod 2^32) of
    geometric gaps of that mean, x_1 = its first gap. Arrays are produced
    on demand by ``list_array(i)`` so that huge pools need not sit in memory.
    """
    lens = zipf_lengths(n_lists, s=s, total=total, lmin=lmin, lmax=lmax, seed=seed)
    rng = np.random.default_rng(seed + 1000)
    codec = rng.integers(0, 2, size=n_lists).astype(np.int32)
    means = 2.0 ** rng.uniform(1.0, 12.0, size=n_lists)
    list_seeds = rng.integers(0, 2**63 - 1, size=n_lists, dtype=np.int64)

    def list_array(i: int) -> np.ndarray:
        g = geometric_gaps(np.random.default_rng(int(list_seeds[i])), int(lens[i]), means[i])
        return _wrap_cumsum(g)

    return lens, codec, means, list_array


def poisson_arrivals(rate: float = 2000.0, duration: float = 60.0, pool: int = 100_000,
                     max_lists: int = 32, seed: int = 6):
    """Poisson request arrivals: returns (times_s, list_ids per request)."""
    rng = np.random.default_rng(seed)
    times = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        times.append(t)
    reqs = [rng.integers(0, pool, size=int(rng.integers(1, max_lists + 1))) for _ in times]
    return np.array(times), reqs


def random_widths_array(n: int, seed: int, max_bits: int = 32) -> np.ndarray:
    """uint32 values whose bit counts are spread uniformly over 0..max_bits."""
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, max_bits + 1, size=n)
    hi = np.where(bits == 0, 0, (np.uint64(1) << bits.astype(np.uint64)) - np.uint64(1))
    v = (rng.integers(0, 2**63 - 1, size=n, dtype=np.int64).astype(np.uint64)) & hi
    return v.astype(U32)
