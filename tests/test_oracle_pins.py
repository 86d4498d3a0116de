"""Pins of the CPU oracle against what the paper and plain mathematics fix.

Each test checks the oracle against something other than itself: a worked
example printed in the paper (fixtures under tests/golden/), a closed form,
an invariant, a library routine or brute force on tiny inputs. No GPU.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1209_2137_amd import datagen
from tests.conftest import GOLDEN


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _bitlen(v):
    return int(v).bit_length()


# ---------------------------------------------------------------- widths

def test_bits_binary_notation():
    # Section 2: a positive integer x needs ceil(log2(x+1)) binary digits
    for x in list(range(0, 5000)) + [2**k + d for k in range(1, 32) for d in (-1, 0, 1)] + [2**32 - 1]:
        x &= 0xFFFFFFFF
        assert oracle.bits(x) == _bitlen(x)
        if x < 2**20:
            assert oracle.bits(x) == math.ceil(math.log2(x + 1))


# ---------------------------------------------------------------- bit packing

def test_bitfield_b4_layout():
    g = _golden("bitfield_layout.json")["b4"]
    vals = [3, 14, 0, 9, 15, 1, 7, 12]
    w = oracle.pack(vals, 4)
    assert w.size == g["words"]
    for v, start in zip(vals, g["field_start_bits"]):
        assert (int(w[0]) >> start) & 15 == v
    assert list(oracle.unpack(w, 8, 4)) == vals


def test_bitfield_b5_straddle():
    g = _golden("bitfield_layout.json")["b5"]
    rng = np.random.default_rng(0)
    for _ in range(200):
        vals = [int(v) for v in rng.integers(0, 32, size=8)]
        w = oracle.pack(vals, 5)
        assert w.size == g["words"]
        w0, w1 = int(w[0]), int(w[1])
        for i in range(6):
            assert (w0 >> g["field_start_bits"][i]) & 31 == vals[i]
        # the 7th integer: bits 30-31 of word 0 are its low bits, bits 0-2 of
        # word 1 its high bits
        lo = sum(((w0 >> b) & 1) << j for j, b in enumerate(g["int7_low_bits_from_word0"]))
        hi = sum(((w1 >> b) & 1) << j for j, b in enumerate(g["int7_high_bits_from_word1"]))
        assert lo | (hi << 2) == vals[6]
        v8 = sum(((w1 >> b) & 1) << j for j, b in enumerate(g["int8_bits_from_word1"]))
        assert v8 == vals[7]
        assert w1 >> 8 == 0  # the 24 unused bits are left clear by this packer
        assert list(oracle.unpack(w, 8, 5)) == vals


@pytest.mark.parametrize("b", range(0, 33))
def test_pack_layout_as_big_integer(b):
    # field i occupies bits [i*b, i*b + b) of the little-endian word string
    rng = np.random.default_rng(b)
    vals = rng.integers(0, 2**32, size=128, dtype=np.uint64).astype(np.uint32)
    w = oracle.pack(vals, b)
    assert w.size == 128 * b // 32  # 128 * b is divisible by 32
    big = 0
    for i, word in enumerate(w):
        big |= int(word) << (32 * i)
    mask = (1 << b) - 1
    for i in range(128):
        assert (big >> (i * b)) & mask == int(vals[i]) & mask
    assert np.array_equal(oracle.unpack(w, 128, b), vals & np.uint32(mask))


# ---------------------------------------------------------------- Variable Byte

def test_vbyte_paper_example():
    g = _golden("vbyte_example.json")
    assert int(g["binary"], 2) == g["value"]
    enc = oracle.vbyte_encode([g["value"]])
    assert list(enc) == g["bytes_memory_order"]
    vals, used = oracle.vbyte_decode(enc, 1)
    assert int(vals[0]) == g["value"] and used == 2


def test_vbyte_lengths_and_flags():
    vals = [0, 1, 127, 128, 2**14 - 1, 2**14, 2**21 - 1, 2**21, 2**28 - 1, 2**28, 2**32 - 1]
    for v in vals:
        enc = oracle.vbyte_encode([v])
        assert len(enc) == max(1, math.ceil(_bitlen(v) / 7))
        assert all(byte < 128 for byte in enc[:-1]) and enc[-1] >= 128
        # low-order group first
        assert sum((byte & 127) << (7 * i) for i, byte in enumerate(enc)) == v
    enc = oracle.vbyte_encode(vals)
    out, used = oracle.vbyte_decode(enc, len(vals))
    assert list(out) == vals and used == len(enc)


def test_vbyte_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.vbyte_decode(bytes([0x01, 0x02]), 1)        # no terminating byte
    with pytest.raises(ValueError):
        oracle.vbyte_decode(bytes([0, 0, 0, 0, 0, 0x81]), 1)  # six bytes
    with pytest.raises(ValueError):
        oracle.vbyte_decode(bytes([0x7F, 0x7F, 0x7F, 0x7F, 0x9F]), 1)  # > 2^32 - 1


# ---------------------------------------------------------------- differential coding

def test_delta_inplace_paper_example():
    g = _golden("delta_examples.json")["inplace"]
    a = np.array(g["original"], dtype=np.uint32)
    oracle.delta_encode_inplace(a, 0, 1)
    assert list(a) == g["deltas"]
    oracle.delta_decode_inplace(a, 0, 1)
    assert list(a) == g["original"]


def test_delta_stride4_rule():
    g = _golden("delta_examples.json")["stride4"]
    a = np.array(g["original"], dtype=np.uint32)
    oracle.delta_encode_inplace(a, 0, 4)
    assert list(a) == g["deltas"]
    oracle.delta_decode_inplace(a, 0, 4)
    assert list(a) == g["original"]


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_delta_decode_is_prefix_sum(stride):
    rng = np.random.default_rng(stride)
    d = rng.integers(0, 2**32, size=10001, dtype=np.uint64).astype(np.uint32)
    init = 0xFFFFFFF0
    a = d.copy()
    oracle.delta_decode_inplace(a, init, stride)
    if stride == 0:
        ref = d
    else:
        ref = np.empty_like(d)
        for r in range(stride):
            ref[r::stride] = (np.cumsum(d[r::stride].astype(np.uint64)) + init).astype(np.uint32)
    assert np.array_equal(a, ref)
    oracle.delta_encode_inplace(a, init, stride)
    assert np.array_equal(a, d)


# ---------------------------------------------------------------- FastPFOR width choice

def _example_block():
    g = _golden("fastpfor_example.json")
    return g, [int(s, 2) for s in g["values_binary"]]


def test_fastpfor_worked_example_choice():
    g, vals = _example_block()
    hist = {}
    for v in vals:
        hist[_bitlen(v)] = hist.get(_bitlen(v), 0) + 1
    assert {str(k): v for k, v in hist.items()} == g["histogram"]
    maxb = max(hist)
    assert maxb == g["max_width"]
    # the paper's cost for B=16: b*16 + (8 + maxb - b)*c
    for b, cost in g["costs"].items():
        b = int(b)
        c = sum(n for w, n in hist.items() if w > b)
        assert b * 16 + (8 + maxb - b) * c == cost
    b, mb, c = oracle.fp_choose(vals)
    assert (b, mb, c) == (g["chosen_b"], g["max_width"], g["exceptions"])
    assert [vals[i] for i in g["exception_positions"]] == [int(s, 2) for s in g["exception_values_binary"]]
    assert [vals[i] >> b for i in g["exception_positions"]] == [int(s, 2) for s in g["exception_high_bits_binary"]]
    assert [v & ((1 << b) - 1) for v in vals] == [int(s, 2) for s in g["truncated_binary"]]
    # 16*b truncated bits + byte array + (maxb-b) bits per exception = 92 bits
    total = 16 * b + 8 * len(g["byte_array"]) + c * (mb - b)
    assert total == g["total_bits"] and total / 16 == g["bits_per_int"]


def test_fastpfor_worked_example_page_bytes():
    """The example block, extended to 128 values with more '10's (which keeps
    b = 2), encoded as a one-block page: the metadata bytes are the paper's
    byte array, the exception array k = 4 holds the printed high bits, and
    the packed data holds the printed truncated values."""
    g, vals = _example_block()
    block = np.array(vals + [2] * 112, dtype=np.uint32)
    assert oracle.fp_choose(block) == (2, 6, 3)
    s = oracle.fp_encode(block, stride=0)
    n_units = int(s[4])
    assert n_units == 1
    page = int(s[8])  # directory entry 0, stride 0: just the offset
    nblocks, packed_words, meta_bytes, bitset = (int(v) for v in s[page:page + 4])
    assert (nblocks, packed_words, meta_bytes) == (1, 128 * 2 // 32, 6)
    assert bitset == 1 << (g["exception_array_width"] - 1)
    assert int(s[page + 4]) == 3
    hdr = 8  # 4 + one count, padded to 4 words
    packed = s[page + hdr: page + hdr + packed_words]
    trunc = oracle.unpack(packed, 16, 2)
    assert [int(v) for v in trunc] == [int(t, 2) for t in g["truncated_binary"]]
    meta = s[page + hdr + packed_words: page + hdr + packed_words + 4].view(np.uint8)
    assert list(meta[:6]) == g["byte_array"] and not meta[6:].any()
    exc = s[page + hdr + packed_words + 4:]
    assert exc.size == 128 * 4 // 32  # one group of 128 at k = 4 bits
    assert [int(v) for v in oracle.unpack(exc, 3, 4)] == [int(t, 2) for t in g["exception_high_bits_binary"]]
    assert np.array_equal(oracle.fp_decode(s, 128), block)


def _cost_table(vals):
    widths = np.array([_bitlen(v) for v in vals])
    maxb = int(widths.max()) if widths.size else 0
    out = []
    for b in range(maxb + 1):
        c = int((widths > b).sum())
        out.append((len(vals) * b + c * (8 + maxb - b), b, c))
    return maxb, out


def test_fastpfor_choice_is_the_minimum():
    rng = np.random.default_rng(7)
    for trial in range(400):
        kind = trial % 4
        if kind == 0:
            v = rng.geometric(1 / 4, size=128)
            v[rng.random(128) < 0.1] = rng.integers(256, 1 << 24)
        elif kind == 1:
            v = datagen.random_widths_array(128, trial)
        elif kind == 2:
            v = rng.integers(0, 1 << int(rng.integers(0, 33)), size=128, dtype=np.uint64)
        else:
            v = np.zeros(128, dtype=np.uint64)
            v[rng.integers(0, 128, size=int(rng.integers(0, 130)))] = rng.integers(0, 2**32, dtype=np.uint64)
        v = np.asarray(v, dtype=np.uint64).astype(np.uint32)
        b, mb, c = oracle.fp_choose(v)
        maxb, table = _cost_table(v)
        best = min(t[0] for t in table)
        winners = [t for t in table if t[0] == best]
        # equal costs: the widest candidate is kept
        assert (b, c) == (winners[-1][1], winners[-1][2]) and mb == maxb
        assert c < 128


# ---------------------------------------------------------------- stream structure

def _bp_widths(stream):
    n_units = int(stream[4])
    widths = []
    for u in range(n_units):
        off = int(stream[8 + u])  # the directory's offsets come first
        desc = stream[off:off + 4].view(np.uint8)
        widths.append([int(b) for b in desc])
    return widths


def _block_max_widths(x, stride):
    x = np.asarray(x, dtype=np.uint64)
    d = x.copy()
    if stride:
        d[stride:] = (x[stride:] - x[:-stride]) % (1 << 32)
    nfull = x.size // 128
    return [_bitlen(int(m)) for m in d[:nfull * 128].reshape(-1, 128).max(axis=1)] if nfull else []


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_bp_widths_are_block_max_bits(stride):
    x = datagen.single_geometric(40000, mean=37, seed=11)
    s = oracle.bp_encode(x, stride)
    flat = [b for unit in _bp_widths(s) for b in unit]
    ref = _block_max_widths(x, stride)
    assert flat[:len(ref)] == ref and not any(flat[len(ref):])


def test_or_shortcut_counterexample():
    # the OR-of-(x+1) formula printed in Section 6.2 gives 3 bits for {3, 0};
    # the widest value needs 2: the width used is bits(OR of the values)
    x = np.zeros(128, dtype=np.uint32)
    x[0] = 3
    assert math.ceil(math.log2((3 + 1) | (0 + 1))) == 3
    s = oracle.bp_encode(x, 0)
    assert _bp_widths(s)[0][0] == 2
    assert np.array_equal(oracle.bp_decode(s, 128), x)


def _vbyte_len(v):
    return max(1, math.ceil(_bitlen(v) / 7))


@pytest.mark.parametrize("stride", [0, 1, 4])
@pytest.mark.parametrize("n", [0, 5, 128, 2048 * 3 + 127, 40000])
def test_bp_size_closed_form(n, stride):
    x = datagen.single_geometric(n, mean=100, seed=n + stride)
    s = oracle.bp_encode(x, stride)
    nfull, tail = n // 128, n % 128
    units = -(-nfull // 16)
    ndir = units + (1 if tail else 0)
    widths = _block_max_widths(x, stride)
    d = np.asarray(x, dtype=np.uint64)
    if stride:
        d = d.copy()
        d[stride:] = (np.asarray(x, np.uint64)[stride:] - np.asarray(x, np.uint64)[:-stride]) % (1 << 32)
    tail_bytes = sum(_vbyte_len(int(v)) for v in d[nfull * 128:])
    dir_words = -(-(1 + stride) * ndir // 4) * 4
    words = 8 + dir_words + 4 * units + sum(4 * b for b in widths) + -(-tail_bytes // 4)
    assert s.size == words
    assert int(s[7]) == words and int(s[5]) == tail_bytes


def test_appendix_a_bound_on_sorted_distinct_arrays():
    # Appendix A: binary packing of the deltas of n sorted distinct 32-bit
    # integers costs less than 8/B + 1 + log2(B) + log2(2^32/n) bits per
    # integer (B = 128); the stream adds a 32-byte header and an 8-byte
    # directory entry per 2048 integers.
    n = 1 << 18
    for x in (datagen.cluster_sorted(n, hi=1 << 32, max_depth=12, seed=21),
              datagen.uniform_sorted(n, seed=22)):
        s = oracle.bp_encode(x, 1)
        bound = 8 / 128 + 1 + 7 + math.log2(2**32 / n)
        extra = (32 * 8 + 8 * 8 * (n / 2048)) / n
        assert s.size * 32 / n <= bound + extra


# ---------------------------------------------------------------- round trips

_ENC = {"bp": oracle.bp_encode, "fp": oracle.fp_encode, "bp32": oracle.bp32_encode, "fp32": oracle.fp32_encode,
        "bpv": oracle.bpv_encode, "sp": oracle.sp_encode, "fpi": oracle.fpi_encode}
_DEC = {"bp": oracle.bp_decode, "fp": oracle.fp_decode, "bp32": oracle.bp32_decode, "fp32": oracle.fp32_decode,
        "bpv": oracle.bpv_decode, "sp": oracle.sp_decode, "fpi": oracle.fpi_decode}
_RC = {"bp": oracle.bp_decode_rc, "fp": oracle.fp_decode_rc, "bp32": oracle.bp32_decode_rc,
       "fp32": oracle.fp32_decode_rc, "bpv": oracle.bpv_decode_rc, "sp": oracle.sp_decode_rc,
       "fpi": oracle.fpi_decode_rc}


@pytest.mark.parametrize("codec", ["bp", "fp", "bp32", "fp32", "bpv", "sp", "fpi"])
@pytest.mark.parametrize("stride", [0, 1, 4])
def test_roundtrip_every_small_length(codec, stride):
    enc, dec = _ENC[codec], _DEC[codec]
    rng = np.random.default_rng(stride)
    for n in range(0, 301):
        x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        if n % 3 == 0:
            x = np.sort(x)
        s = enc(x, stride)
        assert np.array_equal(dec(s, n), x), n


@pytest.mark.parametrize("b", range(0, 33))
def test_single_block_every_width(b):
    rng = np.random.default_rng(100 + b)
    hi = (1 << b) - 1
    x = (rng.integers(0, 2**32, size=128, dtype=np.uint64) & hi).astype(np.uint32)
    x[int(rng.integers(0, 128))] = hi
    s = oracle.bp_encode(x, 0)
    assert _bp_widths(s)[0][0] == b
    assert np.array_equal(oracle.bp_decode(s, 128), x)
    s = oracle.fp_encode(x, 0)
    assert np.array_equal(oracle.fp_decode(s, 128), x)


@pytest.mark.parametrize("stride", [1, 4])
def test_patched_wraparound_roundtrip(stride):
    x = datagen.patched_gaps(3 * 65536 + 1000, seed=5)
    # gaps up to 2^24 make the running sum wrap modulo 2^32
    assert (np.diff(x.astype(np.int64)) < 0).any()
    for enc, dec in ((oracle.fp_encode, oracle.fp_decode), (oracle.bp_encode, oracle.bp_decode)):
        s = enc(x, stride)
        assert np.array_equal(dec(s, x.size), x)


def test_patched_page_counts_match_blocks():
    x = datagen.patched_gaps(65536 + 3 * 128, seed=9)
    s = oracle.fp_encode(x, 1)
    page = int(s[8])
    nblocks, packed_words, meta_bytes, bitset = (int(v) for v in s[page:page + 4])
    assert nblocks == 512
    # after the counts: the value before each of the page's segments of 64
    # blocks but the first (stride 1: one word each), taken from the input
    nset = bin(bitset).count("1")
    assert [int(v) for v in s[page + 4 + nset:page + 4 + nset + 7]] == [int(x[g * 8192 - 1]) for g in range(1, 8)]
    meta_at = page + (-(-(4 + nset + 7) // 4) * 4) + packed_words
    meta = s[meta_at:].view(np.uint8)
    b, mb, c = meta[:512].astype(int), meta[512:1024].astype(int), meta[1024:1536].astype(int)
    assert meta_bytes == 3 * 512 + c.sum()
    assert packed_words == 4 * b.sum()
    counts = {}
    for t in range(512):
        if c[t]:
            counts[mb[t] - b[t]] = counts.get(mb[t] - b[t], 0) + c[t]
    ks = [k for k in range(1, 33) if bitset >> (k - 1) & 1]
    assert ks == sorted(counts)
    assert [int(v) for v in s[page + 4:page + 4 + len(ks)]] == [counts[k] for k in ks]
    # exception positions lie in [0, 127] and each block's are ascending
    pos = meta[1536:1536 + c.sum()]
    at = 0
    for t in range(512):
        p = pos[at:at + c[t]].astype(int)
        assert (p < 128).all() and (np.diff(p) > 0).all()
        at += c[t]


# ---------------------------------------------------------------- corrupt input

@pytest.mark.parametrize("codec", ["bp", "fp", "bp32", "fp32", "bpv"])
def test_corrupt_streams_are_rejected(codec):
    enc, rc = _ENC[codec], _RC[codec]
    x = datagen.single_geometric(5000, seed=3)
    s = enc(x, 1)
    assert rc(s, 5000) == oracle.OK
    assert rc(s[:-1], 5000) == oracle.ERR_CORRUPT              # truncated
    assert rc(s, 4999) == oracle.ERR_CORRUPT                   # wrong length
    bad = s.copy(); bad[0] ^= 1
    assert rc(bad, 5000) == oracle.ERR_CORRUPT                 # magic
    bad = s.copy(); bad[3] = 2
    assert rc(bad, 5000) == oracle.ERR_CORRUPT                 # stride
    bad = s.copy(); bad[8] = 0xFFFFFF
    assert rc(bad, 5000) == oracle.ERR_CORRUPT                 # unit offset
    unit = int(s[8])
    bad = s.copy()
    if codec in ("bp", "bp32", "bpv"):
        bad[unit] = (int(bad[unit]) & ~0xFF) | 33              # width 33
    else:
        bad[unit] = 7                                          # block count
    assert rc(bad, 5000) == oracle.ERR_CORRUPT


def test_max_words_bounds_worst_case():
    rng = np.random.default_rng(1)
    for n in (0, 1, 128, 2048, 65536 + 129):
        x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        for codec, enc in ((0, oracle.bp_encode), (1, oracle.fp_encode), (2, oracle.bp32_encode),
                           (3, oracle.fp32_encode), (4, oracle.bpv_encode)):
            for stride in (0, 1, 4):
                assert enc(x, stride).size <= oracle.max_words(codec, n)


# ---------------------------------------------------------------- generators

def test_generators_shapes_and_determinism():
    a = datagen.single_geometric(1 << 12, seed=1)
    assert np.array_equal(a, datagen.single_geometric(1 << 12, seed=1))
    assert a[0] < 1000 and (np.diff(a.astype(np.int64)) >= 1).all()
    c = datagen.cluster_sorted(1 << 16, max_depth=10, seed=2)
    assert c.size == 1 << 16 and (np.diff(c.astype(np.int64)) > 0).all() and int(c[-1]) < 1 << 30
    u = datagen.uniform_sorted(1 << 16, seed=3)
    assert u.size == 1 << 16 and (np.diff(u.astype(np.int64)) > 0).all()
    lens = datagen.zipf_lengths(1000, total=1.2e7)
    assert lens.min() >= 128 and lens.max() <= 1 << 22 and abs(int(lens.sum()) - 1.2e7) < 2000


# ---------------------------------------------------------------------------
# Intersection of posting lists (the consumer of decoded lists): pinned by
# brute force, the set definition on small inputs, and special cases.

def _sorted_unique(rng, n, hi):
    return np.unique(rng.integers(0, hi, size=n, dtype=np.uint64)).astype(np.uint32)


def test_intersect_matches_set_definition():
    rng = np.random.default_rng(71)
    for trial in range(300):
        hi = int(rng.choice([8, 100, 5000, 2**32]))
        a = _sorted_unique(rng, int(rng.integers(0, 60)), hi)
        b = _sorted_unique(rng, int(rng.integers(0, 60)), hi)
        want = np.array(sorted(set(a.tolist()) & set(b.tolist())), dtype=np.uint32)
        got = oracle.intersect(a, b)
        assert got.dtype == np.uint32 and np.array_equal(got, want), (trial, a, b)


def test_intersect_special_cases():
    e = np.zeros(0, np.uint32)
    x = np.array([0, 1, 7, 2**31, 2**32 - 1], dtype=np.uint32)
    assert oracle.intersect(e, x).size == 0 and oracle.intersect(x, e).size == 0
    assert np.array_equal(oracle.intersect(x, x), x)
    assert oracle.intersect(np.array([1, 3, 5], np.uint32), np.array([2, 4, 6], np.uint32)).size == 0
    sub = x[[1, 3]]
    assert np.array_equal(oracle.intersect(sub, x), sub) and np.array_equal(oracle.intersect(x, sub), sub)
    # symmetric in its arguments
    rng = np.random.default_rng(5)
    a, b = _sorted_unique(rng, 500, 2000), _sorted_unique(rng, 300, 2000)
    assert np.array_equal(oracle.intersect(a, b), oracle.intersect(b, a))


# ---------------------------------------------------------------- BP32 (Section 6.2)

def _deltas(x, stride):
    x = np.asarray(x, dtype=np.uint64)
    d = x.copy()
    if stride:
        d[stride:] = (x[stride:] - x[:-stride]) % (1 << 32)
    return d


def _pack_big(vals, b):
    """Fields of b bits end to end, least significant first (Section 4),
    written as one big integer and cut into 32-bit words."""
    big = 0
    for i, v in enumerate(vals):
        big |= (int(v) & ((1 << b) - 1)) << (i * b)
    return [(big >> (32 * k)) & 0xFFFFFFFF for k in range(len(vals) * b // 32)]


def test_bp32_meta_block_layout():
    # one meta-block: a descriptor word of four 8-bit widths, then the four
    # 32-integer blocks, each in exactly b words (32 fields of b bits)
    rng = np.random.default_rng(7)
    widths = [3, 0, 32, 17]
    x = np.zeros(128, dtype=np.uint32)
    for j, b in enumerate(widths):
        if b:
            blk = rng.integers(0, 1 << b, size=32, dtype=np.uint64)
            blk[5] = (1 << b) - 1
            x[32 * j:32 * j + 32] = blk.astype(np.uint32)
    s = oracle.bp32_encode(x, 0)
    unit = int(s[8])
    assert int(s[0]) == 0x32335057 and int(s[4]) == 1
    desc = int(s[unit])
    assert [(desc >> (8 * j)) & 255 for j in range(4)] == widths
    at = unit + 1
    for j, b in enumerate(widths):
        assert [int(w) for w in s[at:at + b]] == _pack_big(x[32 * j:32 * j + 32], b)
        at += b
    # the unit is zero-padded to a multiple of 4 words, then the stream ends
    used = 1 + sum(widths)
    assert s.size == unit + -(-used // 4) * 4 and not s[unit + used:].any()
    assert np.array_equal(oracle.bp32_decode(s, 128), x)


@pytest.mark.parametrize("stride", [0, 1, 4])
@pytest.mark.parametrize("n", [0, 5, 128, 2048 * 3 + 127, 40000])
def test_bp32_size_closed_form(n, stride):
    x = datagen.single_geometric(n, mean=100, seed=n + stride + 50)
    s = oracle.bp32_encode(x, stride)
    d = _deltas(x, stride)
    nfull, tail = n // 128, n % 128
    units = -(-nfull // 16)
    ndir = units + (1 if tail else 0)
    w32 = [_bitlen(int(m)) for m in d[:nfull * 128].reshape(-1, 32).max(axis=1)] if nfull else []
    words = 8 + -(-(1 + stride) * ndir // 4) * 4
    for u in range(units):
        metas = min(16, nfull - 16 * u)
        used = metas + sum(w32[64 * u:64 * u + 4 * metas])
        words += -(-used // 4) * 4
        # the descriptor of every meta-block holds its four block widths
        at = int(s[8 + u])
        for m in range(metas):
            desc = int(s[at])
            got = [(desc >> (8 * j)) & 255 for j in range(4)]
            assert got == w32[64 * u + 4 * m:64 * u + 4 * m + 4]
            at += 1 + sum(got)
    tail_bytes = sum(_vbyte_len(int(v)) for v in d[nfull * 128:])
    words += -(-tail_bytes // 4)
    assert s.size == words and int(s[7]) == words and int(s[5]) == tail_bytes
    assert np.array_equal(oracle.bp32_decode(s, n), x)


@pytest.mark.parametrize("b", range(0, 33))
def test_bp32_single_block_every_width(b):
    # widths differ block by block: blocks 0..3 of the meta-block get b,
    # 32 - b, b // 2 and 0
    rng = np.random.default_rng(300 + b)
    ws = [b, 32 - b, b // 2, 0]
    x = np.zeros(128, dtype=np.uint32)
    for j, w in enumerate(ws):
        if w:
            blk = rng.integers(0, 1 << w, size=32, dtype=np.uint64)
            blk[int(rng.integers(0, 32))] = (1 << w) - 1
            x[32 * j:32 * j + 32] = blk.astype(np.uint32)
    s = oracle.bp32_encode(x, 0)
    desc = int(s[int(s[8])])
    assert [(desc >> (8 * j)) & 255 for j in range(4)] == ws
    assert np.array_equal(oracle.bp32_decode(s, 128), x)


def test_appendix_a_bound_bp32():
    # Appendix A with B = 32: fewer than 8/32 + 1 + log2(32) + log2(2^32/n)
    # bits per integer for the deltas of n sorted distinct integers, plus the
    # stream's header, directory (8 bytes per 2048 integers) and unit padding
    # (at most 3 words per 2048 integers)
    n = 1 << 18
    for x in (datagen.cluster_sorted(n, hi=1 << 32, max_depth=12, seed=23),
              datagen.uniform_sorted(n, seed=24)):
        s = oracle.bp32_encode(x, 1)
        bound = 8 / 32 + 1 + 5 + math.log2(2**32 / n)
        extra = (32 * 8 + (8 + 12) * 8 * (n / 2048)) / n
        assert s.size * 32 / n <= bound + extra


def test_bp32_never_wider_than_bp128_plus_descriptors():
    # a 32-integer block's width never exceeds that of the 128-integer block
    # holding it, so BP32 spends at most the extra descriptor words (one per
    # 128 integers instead of a quarter) and the unit padding more
    for seed, x in enumerate((datagen.cluster_sorted(1 << 16, max_depth=10, seed=31),
                              datagen.patched_gaps(1 << 16, seed=32))):
        a, b = oracle.bp32_encode(x, 1), oracle.bp_encode(x, 1)
        metas, units = (1 << 16) // 128, (1 << 16) // 2048
        assert a.size <= b.size + metas - metas // 4 + 3 * units


# ---------------------------------------------------------------- FastPFOR, arrays padded to 32 (Section 5)

def _fp_hdr_words(nb, nset, stride):
    """Words of a patched page's header: 4 fixed words, a count per set k,
    stride words per 64-block segment after the first, padded to 4."""
    return -(-(4 + nset + stride * (-(-nb // 64) - 1)) // 4) * 4


def _fp_pages(s):
    """(offset, words, nblocks, packed_words, meta_bytes, counts by k) of each page."""
    units = int(s[4])
    ends = [int(s[8 + u]) for u in range(1, units)] + [int(s[6])]
    pages = []
    for u in range(units):
        at = int(s[8 + u])
        nb, packed, meta, bitset = (int(v) for v in s[at:at + 4])
        ks = [k for k in range(1, 33) if bitset >> (k - 1) & 1]
        counts = dict(zip(ks, (int(v) for v in s[at + 4:at + 4 + len(ks)])))
        pages.append((at, ends[u] - at, nb, packed, meta, counts))
    return pages


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_fastpfor_32_padding_against_128(stride):
    # FastPFOR and SIMD-FastPFOR differ only in how far each exception array
    # is padded (32 values against 128): same headers, packed values and
    # metadata; array k of the first is the first ceil(c/32)*k words of
    # array k of the second (the same LSB-first stream of k-bit fields)
    x = datagen.patched_gaps(3 * 65536 + 5000, seed=40 + stride)
    a, b = oracle.fp32_encode(x, stride), oracle.fp_encode(x, stride)
    assert int(a[0]) == 0x33465057 and int(b[0]) == 0x31465057
    pa, pb = _fp_pages(a), _fp_pages(b)
    assert len(pa) == len(pb) == 4
    saved = 0
    for (oa, wa, nba, pka, ma, ca), (ob, wb, nbb, pkb, mb_, cb) in zip(pa, pb):
        assert (nba, pka, ma, ca) == (nbb, pkb, mb_, cb)
        hdr = _fp_hdr_words(nba, len(ca), stride)
        meta_w = -(-ma // 16) * 4
        fixed = hdr + pka + meta_w
        assert np.array_equal(a[oa:oa + fixed], b[ob:ob + fixed])
        xa, xb = oa + fixed, ob + fixed
        for k in sorted(ca):
            c = ca[k]
            wa_k, wb_k = -(-c // 32) * k, -(-c // 128) * 4 * k
            assert np.array_equal(a[xa:xa + wa_k], b[xb:xb + wa_k])
            assert not b[xb + wa_k:xb + wb_k].any()  # the rest of the 128-padding is zero
            xa += wa_k
            xb += wb_k
            saved += wb_k - wa_k
        # FastPFOR pages end zero-padded to 4 words (units start on 16 bytes)
        assert -(-(xa - oa) // 4) * 4 == wa and not a[xa:oa + wa].any() and xb == ob + wb
    assert 0 < b.size - a.size <= saved
    assert np.array_equal(oracle.fp32_decode(a, x.size), x)


# ---------------------------------------------------------------- vectorized (four-lane) layout (Section 4)

def _words_of_field(i, count, b):
    # the words that field i occupies: pack a lone all-ones field
    v = np.zeros(count, dtype=np.uint32)
    v[i] = (1 << b) - 1
    w = oracle.pack_vertical(v, b)
    return [k for k in range(w.size) if w[k]]


def test_vertical_layout_paper_example():
    g = _golden("vertical_layout.json")
    b, count = g["b"], g["count"]
    assert oracle.pack_vertical(np.zeros(count, np.uint32), b).size == 8  # two series of four words
    lo, hi = g["whole_in_first_row"]
    for i in range(lo, hi + 1):
        ws = _words_of_field(i - 1, count, b)
        assert len(ws) == 1 and ws[0] < 4 and ws[0] == (i - 1) % 4, i
    lo, hi = g["split_between_rows"]
    for i in range(lo, hi + 1):
        assert _words_of_field(i - 1, count, b) == [(i - 1) % 4, 4 + (i - 1) % 4], i
    lo, hi = g["whole_in_second_row"]
    for i in range(lo, hi + 1):
        assert _words_of_field(i - 1, count, b) == [4 + (i - 1) % 4], i
    firsts = [_words_of_field(i - 1, count, b)[0] for i in g["first_four_in_different_words"]]
    assert sorted(firsts) == [0, 1, 2, 3]
    a, c = g["adjacent_in_one_word"]
    wa, wc = _words_of_field(a - 1, count, b), _words_of_field(c - 1, count, b)
    assert wa == wc
    # Int 5 starts where Int 1 ends
    v = np.zeros(count, np.uint32); v[c - 1] = 1
    assert int(oracle.pack_vertical(v, b)[wa[0]]) == 1 << b


@pytest.mark.parametrize("b", range(0, 33))
def test_vertical_lanes_are_horizontal_packings(b):
    # lane l (words l, l+4, l+8, ...) is the plain packing of values l, l+4, ...
    rng = np.random.default_rng(700 + b)
    vals = rng.integers(0, 2**32, size=128, dtype=np.uint64).astype(np.uint32)
    w = oracle.pack_vertical(vals, b)
    assert w.size == 4 * b
    mask = np.uint32((1 << b) - 1) if b < 32 else np.uint32(0xFFFFFFFF)
    for lane in range(4):
        assert np.array_equal(w[lane::4], oracle.pack(vals[lane::4], b)), lane
    assert np.array_equal(oracle.unpack_vertical(w, 128, b), vals & mask)


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_vertical_stream_differs_from_bp_only_inside_blocks(stride):
    # same header, directory, descriptors, sizes and tail; each block's
    # words are the four-lane packing of the same deltas
    x = datagen.single_geometric(2048 * 3 + 128 * 5 + 77, mean=300, seed=60 + stride)
    a, h = oracle.bpv_encode(x, stride), oracle.bp_encode(x, stride)
    assert a.size == h.size and int(a[0]) == 0x31565057 and np.array_equal(a[1:8], h[1:8])
    d = _deltas(x, stride).astype(np.uint32)
    for u, widths in enumerate(_bp_widths(h)):
        off = int(h[8 + u])
        assert np.array_equal(a[off:off + 4], h[off:off + 4])
        at = off + 4
        for j, b in enumerate(widths):
            if 128 * (16 * u + j) >= x.size // 128 * 128:
                break
            blk = d[128 * (16 * u + j):128 * (16 * u + j + 1)]
            assert np.array_equal(a[at:at + 4 * b], oracle.pack_vertical(blk, b))
            assert np.array_equal(h[at:at + 4 * b], oracle.pack(blk, b))
            at += 4 * b
    tail = int(h[6])
    assert np.array_equal(a[tail:], h[tail:])
    assert np.array_equal(oracle.bpv_decode(a, x.size), x)


# ---------------------------------------------------------------------------
# Simple-8b (Section 2) and SimplePFOR (Section 5)

def test_simple8b_modes_are_the_papers_table():
    g = _golden("simple8b_modes.json")
    for sel, cnt, bits in zip(g["selector"], g["integers_coded"], g["bits_per_integer"]):
        assert oracle.s8_mode(sel) == (cnt, bits), sel
        assert cnt * bits <= g["data_bits"]


def _word(sel, vals, bits):
    w = sel << 60
    for j, v in enumerate(vals):
        w |= int(v) << (j * bits)
    return w


def test_simple8b_greedy_special_cases():
    # worked by hand from the table and the greedy rule (selectors tried
    # from 0 upward, the first that fits the next integers is taken)
    assert [int(w) for w in oracle.s8_encode(np.zeros(240, np.uint32))] == [0]
    # 239 zeros: 120 (selector 1), then 60, 30, 20 (selectors 2, 3, 4), 8
    # (selector 8: 9 left, too few for selectors 5..7), 1 (selector 15)
    w = oracle.s8_encode(np.zeros(239, np.uint32))
    assert [int(x) >> 60 for x in w] == [1, 2, 3, 4, 8, 15]
    assert [int(x) for x in oracle.s8_encode(np.ones(60, np.uint32))] == [_word(2, [1] * 60, 1)]
    v = np.array([(1 << 20) - 1, 5, (1 << 20) - 2], np.uint32)
    assert [int(x) for x in oracle.s8_encode(v)] == [_word(13, v, 20)]
    assert [int(x) for x in oracle.s8_encode(np.array([0xFFFFFFFF], np.uint32))] == [_word(15, [0xFFFFFFFF], 60)]
    # one value of 2 bits among 60 small ones: two words of 30 two-bit values
    v = np.array([1] * 59 + [2], np.uint32)
    assert [int(x) >> 60 for x in oracle.s8_encode(v)] == [3, 3]
    # values of 31 bits: one per word (30 bits are too few)
    assert [int(x) >> 60 for x in oracle.s8_encode(np.array([1 << 30, 1 << 30], np.uint32))] == [15, 15]


def test_simple8b_roundtrip_and_errors():
    rng = np.random.default_rng(81)
    for n in (0, 1, 2, 59, 60, 61, 239, 240, 241, 1000):
        for hi in (1, 2, 1 << 7, 1 << 20, 1 << 31):
            v = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
            v[rng.random(n) < 0.3] = 0
            w = oracle.s8_encode(v)
            k, back = oracle.s8_decode(w, n)
            assert k == n and np.array_equal(back, v), (n, hi)
    w = oracle.s8_encode(np.zeros(240, np.uint32))
    assert oracle.s8_decode(w, 239)[0] == oracle.ERR_CORRUPT  # more values than room
    assert oracle.s8_decode(np.array([(15 << 60) | (1 << 40)], np.uint64), 1)[0] == oracle.ERR_CORRUPT  # > 32 bits


def _sp_hdr_words(nb, stride):
    """Words of a SimplePFOR page's header: 4 fixed words, then for each
    64-block segment after the first `stride` bases and one Simple-8b
    entry, padded to 4."""
    return -(-(4 + (stride + 1) * (-(-nb // 64) - 1)) // 4) * 4


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_simplepfor_pages_are_fastpfor_pages_but_for_the_exceptions(stride):
    # Section 5: SimplePFOR and FastPFOR differ only in how the high parts
    # of the exceptions are stored: same widths, packed values, metadata and
    # segment bases
    x = datagen.patched_gaps(2 * 65536 + 128 * 9 + 40, seed=83)
    fp, sp = oracle.fp_encode(x, stride), oracle.sp_encode(x, stride)
    assert np.array_equal(oracle.sp_decode(sp, x.size), x)
    units = int(fp[4])
    for u in range(units):
        fo, so = int(fp[8 + u]), int(sp[8 + u])
        nb, packed, meta_bytes, bitset = (int(v) for v in fp[fo:fo + 4])
        assert [int(v) for v in sp[so:so + 3]] == [nb, packed, meta_bytes]
        nset = bin(bitset).count("1")
        nseg = -(-nb // 64)
        assert np.array_equal(fp[fo + 4 + nset:fo + 4 + nset + stride * (nseg - 1)],
                              sp[so + 4:so + 4 + stride * (nseg - 1)])
        fh, sh = _fp_hdr_words(nb, nset, stride), _sp_hdr_words(nb, stride)
        meta_w = (meta_bytes + 15) // 16 * 4
        assert np.array_equal(fp[fo + fh:fo + fh + packed + meta_w], sp[so + sh:so + sh + packed + meta_w])
        # the Simple-8b array holds one high part per exception, in block order
        s8w = int(sp[so + 3])
        words = sp[so + sh + packed + meta_w:so + sh + packed + meta_w + s8w].astype(np.uint64)
        w64 = words[0::2] | (words[1::2] << np.uint64(32))
        k, hv = oracle.s8_decode(w64, meta_bytes - 3 * nb)
        assert k == meta_bytes - 3 * nb and (hv > 0).all()


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_simplepfor_segment_entries_locate_each_segments_first_exception(stride):
    # each segment's entry names the Simple-8b word holding the high part
    # of its first exception (the exceptions of the blocks before it,
    # counted from the metadata) and how many of that word's values come
    # before it; counted here from the selectors with Section 2's table
    count_of = _golden("simple8b_modes.json")["integers_coded"]
    x = datagen.patched_gaps(3 * 65536 + 128 * 70 + 9, seed=86)
    s = oracle.sp_encode(x, stride)
    checked = 0
    for u in range(int(s[4])):
        so = int(s[8 + u])
        nb, packed, meta_bytes, s8w = (int(v) for v in s[so:so + 4])
        nseg = -(-nb // 64)
        sh = _sp_hdr_words(nb, stride)
        meta = s[so + sh + packed:].view(np.uint8)
        counts = [int(c) for c in meta[2 * nb:3 * nb]]
        meta_w = (meta_bytes + 15) // 16 * 4
        words = s[so + sh + packed + meta_w:so + sh + packed + meta_w + s8w].astype(np.uint64)
        sel = [int(w >> np.uint64(28)) for w in words[1::2]]
        starts = np.concatenate([[0], np.cumsum([count_of[q] for q in sel])])
        for g in range(1, nseg):
            e = sum(counts[:64 * g])
            ent = int(s[so + 4 + stride * (nseg - 1) + g - 1])
            if e == starts[-1]:
                assert ent == len(sel)
            else:
                w = int(np.searchsorted(starts, e, side="right")) - 1
                assert ent == w | ((e - int(starts[w])) << 24), (u, g)
            checked += 1
    assert checked >= 3 * 7
    # a wrong entry is rejected
    so = int(s[8])
    bad = s.copy()
    bad[so + 4 + stride * 7] ^= 1
    assert oracle.sp_decode_rc(bad, x.size) == oracle.ERR_CORRUPT


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_simplepfor_roundtrip_and_size(stride):
    rng = np.random.default_rng(84 + stride)
    for n in (0, 1, 127, 128, 129, 1000, 65536, 65536 + 128 * 3 + 5):
        d = np.where(rng.random(n) < 0.05, rng.integers(1 << 16, 1 << 28, size=n), rng.integers(0, 16, size=n))
        x = (d if stride == 0 else np.cumsum(d)).astype(np.uint32)
        s = oracle.sp_encode(x, stride)
        assert s.size <= oracle.max_words(oracle.CODEC_SP, n)
        assert np.array_equal(oracle.sp_decode(s, n), x), n


def test_simplepfor_corrupt_streams_are_rejected():
    x = datagen.patched_gaps(65536 + 500, seed=85)
    s = oracle.sp_encode(x, 1)
    assert oracle.sp_decode_rc(s, x.size) == oracle.OK
    unit = int(s[8])
    for at, val in ((0, int(s[0]) ^ 1), (unit, 7), (unit + 2, int(s[unit + 2]) + 1), (unit + 3, int(s[unit + 3]) + 2)):
        bad = s.copy()
        bad[at] = val & 0xFFFFFFFF
        assert oracle.sp_decode_rc(bad, x.size) == oracle.ERR_CORRUPT, at
    assert oracle.sp_decode_rc(oracle.fp_encode(x, 1), x.size) == oracle.ERR_CORRUPT


# ---------------------------------------------------------------- segment bases of patched pages

@pytest.mark.parametrize("stride", [1, 4])
@pytest.mark.parametrize("codec", ["fp", "fp32"])
def test_patched_segment_bases_are_the_inputs_before_each_segment(stride, codec):
    # after the per-array counts, a page header holds, for each 64-block
    # segment but the first, the `stride` input values just before it; a
    # page of nb blocks has ceil(nb / 64) segments
    enc, rc = ((oracle.fp_encode, oracle.fp_decode_rc) if codec == "fp"
               else (oracle.fp32_encode, oracle.fp32_decode_rc))
    x = datagen.patched_gaps(2 * 65536 + 200 * 128 + 33, seed=60 + stride)
    s = enc(x, stride)
    units = int(s[4])
    assert units == 3
    for u in range(units):
        at = int(s[8 + u])
        nb, _, _, bitset = (int(v) for v in s[at:at + 4])
        nseg = -(-nb // 64)
        assert nseg == (8 if u < 2 else 4)
        h = at + 4 + bin(bitset).count("1")
        got = [int(v) for v in s[h:h + stride * (nseg - 1)]]
        first = u * 65536
        want = [int(x[first + g * 8192 - stride + t]) for g in range(1, nseg) for t in range(stride)]
        assert got == want
        # a wrong segment base is rejected (it disagrees with the decoded values)
        bad = s.copy()
        bad[h + stride * (nseg - 1) - 1] ^= np.uint32(1 << 7)
        assert rc(bad, x.size) == oracle.ERR_CORRUPT
    assert rc(s, x.size) == oracle.OK


def test_patched_stride0_pages_hold_no_segment_bases():
    x = datagen.patched_gaps(65536, seed=66)
    s = oracle.fp_encode(x, 0)
    at = int(s[8])
    nb, packed, _, bitset = (int(v) for v in s[at:at + 4])
    assert nb == 512 and _fp_hdr_words(nb, bin(bitset).count("1"), 0) == -(-(4 + bin(bitset).count("1")) // 4) * 4
    assert np.array_equal(oracle.fp_decode(s, x.size), x)


# ---------------------------------------------------------------- the paper's own page layout

def test_paper_layout_worked_example_page():
    """Section 5's running example (the block extended to 128 values with
    more '10's, keeping b = 2) as a one-block page in the layout of the
    page-layout figure: the offset word points at the byte array's counter,
    which sits right after the truncated values and holds 6; the byte array
    is the printed 2, 6, 3, 4, 9, 11, zero-padded to 8 bytes; then the
    bitset (array 4 only), array 4's counter 3 and its three 4-bit high
    parts 1001, 1000, 1101, padded to 32 values (4 words)."""
    g, vals = _example_block()
    block = np.array(vals + [2] * 112, dtype=np.uint32)
    s = oracle.fpi_encode(block, stride=0)
    assert int(s[0]) == 0x31495057 and int(s[4]) == 1
    page = s[int(s[8]):int(s[6])]
    packed_words = 128 * 2 // 32
    assert int(page[0]) == 1 + packed_words
    trunc = oracle.unpack(page[1:1 + packed_words], 16, 2)
    assert [int(v) for v in trunc] == [int(t, 2) for t in g["truncated_binary"]]
    assert int(page[1 + packed_words]) == len(g["byte_array"])
    ba = page[2 + packed_words:4 + packed_words].view(np.uint8)
    assert list(ba[:6]) == g["byte_array"] and not ba[6:].any()
    at = 4 + packed_words
    assert int(page[at]) == 1 << (g["exception_array_width"] - 1)
    assert int(page[at + 1]) == 3
    exc = page[at + 2:at + 2 + 4]
    assert [int(v) for v in oracle.unpack(exc, 3, 4)] == [int(t, 2) for t in g["exception_high_bits_binary"]]
    assert not oracle.unpack(exc, 32, 4)[3:].any()
    assert page.size == at + 2 + 4 + 2  # zero words to a multiple of 4
    assert np.array_equal(oracle.fpi_decode(s, 128), block)


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_paper_layout_holds_the_fastpfor_page_inline(stride):
    # the same page as the FastPFOR (32-padded) page of the same input,
    # arranged as the paper arranges it: its packed words, its b / maxb / c
    # bytes interleaved per block (c and the positions only when maxb > b),
    # its arrays each behind a counter instead of all counts in the header
    x = datagen.patched_gaps(2 * 65536 + 128 * 3 + 9, seed=90 + stride)
    a, f = oracle.fpi_encode(x, stride), oracle.fp32_encode(x, stride)
    units = int(a[4])
    assert units == int(f[4]) == 3
    ends_a = [int(a[8 + u]) for u in range(1, units)] + [int(a[6])]
    ends_f = [int(f[8 + u]) for u in range(1, units)] + [int(f[6])]
    for u in range(units):
        pa = a[int(a[8 + u]):ends_a[u]]
        pf = f[int(f[8 + u]):ends_f[u]]
        nb, packed, meta_bytes, bitset = (int(v) for v in pf[:4])
        ks = [k for k in range(1, 33) if bitset >> (k - 1) & 1]
        hdr = -(-(4 + len(ks) + stride * (-(-nb // 64) - 1)) // 4) * 4
        cpos = int(pa[0])
        assert cpos == 1 + packed
        assert np.array_equal(pa[1:cpos], pf[hdr:hdr + packed])
        meta = pf[hdr + packed:].view(np.uint8)[:meta_bytes]
        b, mb, c, pos = meta[:nb], meta[nb:2 * nb], meta[2 * nb:3 * nb], meta[3 * nb:]
        want, at = [], 0
        for t in range(nb):
            want += [int(b[t]), int(mb[t])]
            if mb[t] > b[t]:
                want += [int(c[t])] + [int(v) for v in pos[at:at + int(c[t])]]
            at += int(c[t])
        nba = int(pa[cpos])
        assert nba == len(want) == 3 * nb + len(pos) - int((mb == b).sum())
        ba = pa[cpos + 1:cpos + 1 + -(-nba // 4)].view(np.uint8)
        assert list(ba[:nba]) == want and not ba[nba:].any()
        xp = cpos + 1 + -(-nba // 4)
        assert int(pa[xp]) == bitset
        xp += 1
        xf = hdr + packed + -(-meta_bytes // 16) * 4
        counts = [int(v) for v in pf[4:4 + len(ks)]]
        for k, cnt in zip(ks, counts):
            words = -(-cnt // 32) * k
            assert int(pa[xp]) == cnt
            assert np.array_equal(pa[xp + 1:xp + 1 + words], pf[xf:xf + words])
            xp += 1 + words
            xf += words
        assert -(-xp // 4) * 4 == pa.size and not pa[xp:].any()
    assert np.array_equal(oracle.fpi_decode(a, x.size), x)


def test_paper_layout_corrupt_pages_are_rejected():
    x = datagen.patched_gaps(65536 + 700, seed=95)
    s = oracle.fpi_encode(x, 1)
    assert oracle.fpi_decode_rc(s, x.size) == oracle.OK
    p0 = int(s[8])
    cpos = p0 + int(s[p0])
    nba = int(s[cpos])
    bad_cases = {
        "offset": (p0, int(s[p0]) + 4),
        "counter": (cpos, nba + 1),
        "bitset": (cpos + 1 + -(-nba // 4), int(s[cpos + 1 + -(-nba // 4)]) ^ 1),
        "first_width": (cpos + 1, (int(s[cpos + 1]) & ~0xFF) | 33),
    }
    for what, (at, val) in bad_cases.items():
        bad = s.copy()
        bad[at] = val & 0xFFFFFFFF
        assert oracle.fpi_decode_rc(bad, x.size) == oracle.ERR_CORRUPT, what
    assert oracle.fpi_decode_rc(oracle.fp32_encode(x, 1), x.size) == oracle.ERR_CORRUPT

