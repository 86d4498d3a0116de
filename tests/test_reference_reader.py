"""An independent pure-Python reader of the stream layout, checked against
the oracle's streams.

The reader below is written from the layout alone (header, directory with
unit offsets and bases, SIMD-BP128 meta-blocks in the sequential and in the
four-lane block layout, BP32 meta-blocks, FastPFOR pages with exception
arrays padded to 128 or to 32 values, FastPFOR pages in the paper's own
layout with the counted byte array, SimplePFOR pages with one Simple-8b
array of exception high parts, Variable Byte remainder), with bit fields
read from Python big integers; it shares nothing with the oracle but the
layout. Every stream the oracle writes for small inputs (every length
0..300, every stride, every codec) and for a few multi-unit inputs must read
back to the input: a mistake in either one's reading of the layout shows.
No GPU.
"""
import numpy as np
import pytest

import oracle
from paper_1209_2137_amd import datagen

MAGIC = {"bp": 0x31425057, "fp": 0x31465057, "bp32": 0x32335057, "fp32": 0x33465057, "bpv": 0x31565057,
         "sp": 0x31535057, "fpi": 0x31495057}
ENC = {"bp": oracle.bp_encode, "fp": oracle.fp_encode, "bp32": oracle.bp32_encode, "fp32": oracle.fp32_encode,
       "bpv": oracle.bpv_encode, "sp": oracle.sp_encode, "fpi": oracle.fpi_encode}
# Simple-8b modes (Section 2): selector -> (integers per word, bits each)
S8 = [(240, 0), (120, 0), (60, 1), (30, 2), (20, 3), (15, 4), (12, 5), (10, 6), (8, 7), (7, 8), (6, 10), (5, 12),
      (4, 15), (3, 20), (2, 30), (1, 60)]


def _big(words):
    """The words as one little-endian integer (word 0 lowest)."""
    v = 0
    for i, w in enumerate(words):
        v |= int(w) << (32 * i)
    return v


def _fields(words, count, b):
    big = _big(words)
    m = (1 << b) - 1
    return [(big >> (i * b)) & m for i in range(count)]


def _fields_four_lanes(words, count, b):
    """Four 32-bit lanes, word w of lane l at 4w + l; value i is field i // 4
    of lane i % 4."""
    lanes = [_big(words[l::4]) for l in range(4)]
    m = (1 << b) - 1
    return [(lanes[i % 4] >> ((i // 4) * b)) & m for i in range(count)]


def _vbyte(data, count):
    out, v, shift = [], 0, 0
    for byte in data:
        v |= (byte & 0x7F) << shift
        shift += 7
        if byte & 0x80:
            out.append(v)
            v, shift = 0, 0
            if len(out) == count:
                break
    assert len(out) == count
    return out


def _bp_unit(w, nblocks, four_lanes):
    desc = [(int(w[j // 4]) >> (8 * (j % 4))) & 255 for j in range(16)]
    assert all(b == 0 for b in desc[nblocks:])
    at, out = 4, []
    for j in range(nblocks):
        b = desc[j]
        blk = w[at:at + 4 * b]
        out += _fields_four_lanes(blk, 128, b) if four_lanes else _fields(blk, 128, b)
        at += 4 * b
    assert at == len(w)
    return out


def _bp32_unit(w, nmeta):
    at, out = 0, []
    for _ in range(nmeta):
        d = int(w[at])
        at += 1
        for j in range(4):
            b = (d >> (8 * j)) & 255
            out += _fields(w[at:at + b], 32, b)
            at += b
    assert -(-at // 4) * 4 == len(w) and not any(int(v) for v in w[at:])
    return out


def _fp_page(w, nblocks, pad, S):
    """Patched page: (deltas, segment bases). After the counts, the header
    holds S words for every 64-block segment but the first: the values just
    before that segment."""
    nb, packed, meta_bytes, bitset = (int(v) for v in w[:4])
    assert nb == nblocks
    ks = [k for k in range(1, 33) if bitset >> (k - 1) & 1]
    counts = {k: int(w[4 + i]) for i, k in enumerate(ks)}
    nseg = -(-nb // 64)
    segb = [int(v) for v in w[4 + len(ks):4 + len(ks) + S * (nseg - 1)]]
    at = -(-(4 + len(ks) + S * (nseg - 1)) // 4) * 4
    packed_at = at
    at += packed
    meta = bytes(np.asarray(w[at:at + -(-meta_bytes // 16) * 4], dtype=np.uint32).tobytes())[:meta_bytes]
    at += -(-meta_bytes // 16) * 4
    b, mb, c = meta[:nb], meta[nb:2 * nb], meta[2 * nb:3 * nb]
    pos = meta[3 * nb:]
    arrays = {}
    for k in ks:
        cnt = counts[k]
        words = -(-cnt // pad) * pad * k // 32
        arrays[k] = _fields(w[at:at + words], cnt, k)
        at += words
    assert -(-at // 4) * 4 == len(w)
    taken = {k: 0 for k in ks}
    out, p_at, blk_at = [], 0, packed_at
    for t in range(nb):
        vals = _fields(w[blk_at:blk_at + 4 * b[t]], 128, b[t])
        blk_at += 4 * b[t]
        k = mb[t] - b[t]
        for j in range(c[t]):
            vals[pos[p_at + j]] |= arrays[k][taken[k]] << b[t]
            taken[k] += 1
        p_at += c[t]
        out += vals
    assert all(taken[k] == counts[k] for k in ks)
    return out, segb


def _fpi_page(w, nblocks):
    """The paper's page: offset word -> counter of the byte array, whose
    records are b, maxb and, when maxb > b, c and c positions; after the
    byte array a bitset, then each array behind its counter, padded to 32
    values."""
    at = int(w[0])
    nba = int(w[at])
    ba = bytes(np.asarray(w[at + 1:at + 1 + -(-nba // 4)], dtype=np.uint32).tobytes())
    xp = at + 1 + -(-nba // 4)
    bitset = int(w[xp])
    xp += 1
    arrays = {}
    for k in range(1, 33):
        if bitset >> (k - 1) & 1:
            cnt = int(w[xp])
            words = -(-cnt // 32) * k
            arrays[k] = _fields(w[xp + 1:xp + 1 + words], cnt, k)
            xp += 1 + words
    assert -(-xp // 4) * 4 == len(w)
    taken = {k: 0 for k in arrays}
    out, r, pk = [], 0, 1
    for _ in range(nblocks):
        b, mb = ba[r], ba[r + 1]
        r += 2
        vals = _fields(w[pk:pk + 4 * b], 128, b)
        pk += 4 * b
        if mb > b:
            c = ba[r]
            for p_ in ba[r + 1:r + 1 + c]:
                vals[p_] |= arrays[mb - b][taken[mb - b]] << b
                taken[mb - b] += 1
            r += 1 + c
        out += vals
    assert pk == at and r == nba and not any(ba[nba:])
    assert all(taken[k] == len(arrays[k]) for k in arrays)
    return out


def _sp_page(w, nblocks, S):
    """SimplePFOR page: FastPFOR's packed values and metadata, the
    exceptions' high parts as one Simple-8b array (selector in the top four
    bits of each 64-bit word, low 32-bit half first); after the 4 header
    words, S bases and then one Simple-8b entry for each 64-block segment
    after the first (the word holding the segment's first high part | the
    values of that word before it << 24). Returns the deltas and the
    segment bases."""
    nb, packed, meta_bytes, s8_words = (int(v) for v in w[:4])
    assert nb == nblocks
    nseg = -(-nb // 64)
    segb = [int(v) for v in w[4:4 + S * (nseg - 1)]]
    entries = [int(v) for v in w[4 + S * (nseg - 1):4 + (S + 1) * (nseg - 1)]]
    at = -(-(4 + (S + 1) * (nseg - 1)) // 4) * 4
    assert not any(int(v) for v in w[4 + (S + 1) * (nseg - 1):at])
    packed_at = at
    at += packed
    meta = bytes(np.asarray(w[at:at + -(-meta_bytes // 16) * 4], dtype=np.uint32).tobytes())[:meta_bytes]
    at += -(-meta_bytes // 16) * 4
    b, mb, c = meta[:nb], meta[nb:2 * nb], meta[2 * nb:3 * nb]
    pos = meta[3 * nb:]
    high, word_of = [], []
    for i in range(0, s8_words, 2):
        word = int(w[at + i]) | (int(w[at + i + 1]) << 32)
        cnt, bits = S8[word >> 60]
        word_of += [(i // 2) | (j << 24) for j in range(cnt)]
        high += [(word >> (j * bits)) & ((1 << bits) - 1) if bits else 0 for j in range(cnt)]
    at += s8_words
    assert -(-at // 4) * 4 == len(w) and len(high) == len(pos)
    for g in range(1, nseg):
        e = sum(c[:64 * g])
        assert entries[g - 1] == (word_of[e] if e < len(high) else s8_words // 2)
    out, p_at, blk_at = [], 0, packed_at
    for t in range(nb):
        vals = _fields(w[blk_at:blk_at + 4 * b[t]], 128, b[t])
        blk_at += 4 * b[t]
        for j in range(c[t]):
            assert 0 < high[p_at + j] < (1 << (mb[t] - b[t]))
            vals[pos[p_at + j]] |= high[p_at + j] << b[t]
        p_at += c[t]
        out += vals
    return out, segb


def read(stream, codec):
    """The integers the stream holds (deltas undone from the stored bases)."""
    s = np.asarray(stream, dtype=np.uint32)
    assert int(s[0]) == MAGIC[codec]
    n = int(s[1]) | (int(s[2]) << 32)
    S, units, tail_bytes, tail_off, total = (int(v) for v in s[3:8])
    assert total == s.size
    per = 512 if codec in ("fp", "fp32", "sp", "fpi") else 16
    nfull, tail = n // 128, n % 128
    assert units == -(-nfull // per)
    ndir = units + (1 if tail else 0)
    offs = [int(v) for v in s[8:8 + ndir]]
    out = []
    for u in range(ndir):
        start = u * per * 128 if u < units else nfull * 128
        bases = [int(v) for v in s[8 + ndir + u * S:8 + ndir + (u + 1) * S]]
        end = offs[u + 1] if u + 1 < units else tail_off
        if u < units:
            nb = min(per, nfull - u * per)
            w = s[offs[u]:end]
            if codec in ("bp", "bpv"):
                d = _bp_unit(w, nb, codec == "bpv")
            elif codec == "bp32":
                d = _bp32_unit(w, nb)
            elif codec == "sp":
                d, segb = _sp_page(w, nb, S)
            elif codec == "fpi":
                d = _fpi_page(w, nb)
            else:
                d, segb = _fp_page(w, nb, 32 if codec == "fp32" else 128, S)
        else:
            assert offs[u] == tail_off
            d = _vbyte(s[tail_off:total].tobytes()[:tail_bytes], tail)
        # Section 3: x_i = d_i + x_{i-S}, the unit's bases standing in before it
        x = []
        for i, v in enumerate(d):
            prev = (x[i - S] if i >= S else bases[i]) if S else 0
            x.append((v + prev) & 0xFFFFFFFF)
        if u < units and codec in ("fp", "fp32", "sp"):
            # segment g's stored bases are the values just before it
            for i, v in enumerate(segb):
                g, t = 1 + i // S, i % S
                assert x[g * 64 * 128 - S + t] == v
        out += x
        assert len(out) == start + len(d)
    assert len(out) == n
    return np.asarray(out, dtype=np.uint32)


@pytest.mark.parametrize("codec", sorted(MAGIC))
@pytest.mark.parametrize("stride", [0, 1, 4])
def test_reader_agrees_on_every_small_length(codec, stride):
    rng = np.random.default_rng(11 * stride + len(codec))
    for n in range(0, 301):
        kind = n % 3
        if kind == 0:
            x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        elif kind == 1:
            x = np.cumsum(rng.integers(1, 1 << int(rng.integers(1, 20)), size=n)).astype(np.uint32)
        else:
            x = (rng.integers(0, 16, size=n) | (rng.random(n) < 0.1) * rng.integers(1 << 10, 1 << 28, size=n)
                 ).astype(np.uint32)
        s = ENC[codec](x, stride)
        got = read(s, codec)
        assert np.array_equal(got, x), (codec, stride, n)


@pytest.mark.parametrize("codec", sorted(MAGIC))
def test_reader_agrees_on_multi_unit_lists(codec):
    # more than one unit of each kind (meta-blocks of 2048, pages of 65536),
    # a partial last unit and a tail; exceptions of many widths
    x = datagen.patched_gaps(65536 + 2048 * 3 + 128 * 5 + 77, seed=91)
    for stride in (1, 4):
        s = ENC[codec](x, stride)
        assert np.array_equal(read(s, codec), x), (codec, stride)
