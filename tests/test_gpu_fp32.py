"""GPU parity for FastPFOR pages whose exception arrays are padded to 32
values (Section 5) instead of SIMD-FastPFOR's 128: the HIP decoder against
the generators' arrays and the oracle's streams, the HIP encoder against
the oracle's encoder byte for byte. Exact comparisons (integer work);
outputs sit between canary fences to catch writes outside [out, out + n)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1209_2137_amd as wp
from paper_1209_2137_amd import autotune
from paper_1209_2137_amd import datagen

pytestmark = pytest.mark.gpu

CANARY = 0x5A5A5A5A
PAD = 64
WAVES = (8, 4, 2)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    wp.lib()
    yield
    autotune.apply()


def to_dev(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if a.size == 0:
        return torch.zeros(4, dtype=torch.int32, device="cuda")[:0]
    return torch.from_numpy(a.view(np.int32)).to("cuda")


def to_host(t):
    return t.cpu().numpy().view(np.uint32)


def gpu_decode(stream_np, n):
    comp = to_dev(stream_np)
    buf = torch.full((n + 2 * PAD,), CANARY, dtype=torch.int32, device="cuda")
    out = buf[PAD:PAD + n]
    wp.fastpfor32_decode(comp, n, out)
    rc = wp.check_code()
    h = to_host(buf)
    assert (h[:PAD] == CANARY).all() and (h[PAD + n:] == CANARY).all(), "write outside [out, out + n)"
    return rc, h[PAD:PAD + n]


def assert_same(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[0]}: "
                             f"got {got[bad[0]]} want {want[bad[0]]}")


LENGTHS = [0, 1, 5, 127, 128, 129, 1000, 2049, 8192 + 3, 65535, 65536, 65537, 2 * 65536 + 3 * 128 + 77]


def _case(rng, n):
    kind = n % 3
    if kind == 0:
        return rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    if kind == 1:
        return datagen.single_geometric(n, mean=float(rng.integers(2, 5000)), seed=n)
    return datagen.patched_gaps(n, seed=n) if n else np.zeros(0, np.uint32)


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_decode_lengths_strides_shapes(stride):
    rng = np.random.default_rng(5200 + stride)
    cases = [(n, x, oracle.fp32_encode(x, stride)) for n, x in ((n, _case(rng, n)) for n in LENGTHS)]
    for waves in WAVES:
        wp.set_decode_tune(wp.CODEC_FP32, waves, 4)
        for n, x, s in cases:
            print(f"fp32 stride={stride} waves={waves} n={n}", flush=True)
            rc, got = gpu_decode(s, n)
            assert rc == wp.OK
            assert_same(got, x, f"n={n} waves={waves}")


@pytest.mark.parametrize("wide_frac", [0.001, 0.05, 0.4])
@pytest.mark.parametrize("stride", [0, 1])
def test_encode_matches_oracle_and_decodes(wide_frac, stride):
    # few to many exceptions: arrays of every length modulo 32
    rng = np.random.default_rng(int(wide_frac * 1000) + stride)
    n = 3 * 65536 + 128 * 7 + 5
    small = rng.integers(0, 16, size=n, dtype=np.uint64)
    wide = rng.integers(1 << 20, 1 << 24, size=n, dtype=np.uint64)
    d = np.where(rng.random(n) < wide_frac, wide, small)
    x = (d if stride == 0 else np.cumsum(d)).astype(np.uint32)
    print(f"fp32 encode wide_frac={wide_frac} stride={stride}", flush=True)
    want = oracle.fp32_encode(x, stride)
    got = to_host(wp.encode_trimmed(to_dev(x), wp.CODEC_FP32, stride))
    assert got.size == want.size
    assert_same(got, want, f"wide_frac={wide_frac}")
    rc, back = gpu_decode(got, n)
    assert rc == wp.OK
    assert_same(back, x)
    # never longer than the SIMD-FastPFOR stream of the same input
    assert got.size <= oracle.fp_encode(x, stride).size


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_encode_small_lengths_match_oracle(stride):
    rng = np.random.default_rng(5300 + stride)
    for n in LENGTHS:
        x = _case(rng, n)
        print(f"fp32 encode stride={stride} n={n}", flush=True)
        got = to_host(wp.encode_trimmed(to_dev(x), wp.CODEC_FP32, stride))
        want = oracle.fp32_encode(x, stride)
        assert got.size == want.size and np.array_equal(got, want), f"n={n}"


def test_full_size_patched_list():
    # the 2^28 patched workload: GPU encode, GPU decode, exact round trip;
    # a sampled page of the GPU stream equals the oracle's page
    x = datagen.patched_gaps()
    xd = to_dev(x)
    comp = wp.encode_trimmed(xd, wp.CODEC_FP32, 1)
    out = torch.empty(xd.numel(), dtype=torch.int32, device="cuda")
    autotune.apply()
    wp.fastpfor32_decode(comp, xd.numel(), out)
    assert wp.check_code() == wp.OK
    assert torch.equal(out, xd)
    full = wp.encode_trimmed(xd, wp.CODEC_FP, 1)
    assert comp.numel() < full.numel()
    # page 1000 of the stream against the oracle's encoding of its values
    # (with stride 1 its deltas depend on the value before the page only)
    s = to_host(comp[:8 + 4096 * 2 + 8])
    off, end = int(s[8 + 1000]), int(s[8 + 1001])
    page = to_host(comp[off:end])
    lo = 1000 * 65536
    seg = x[lo:lo + 65536].astype(np.uint64)
    d = np.empty(65536, np.uint64)
    d[0] = (seg[0] - np.uint64(x[lo - 1])) % (1 << 32)
    d[1:] = (seg[1:] - seg[:-1]) % (1 << 32)
    ref = oracle.fp32_encode(d.astype(np.uint32), 0)
    ref = ref[int(ref[8]):int(ref[6])]
    # the stride-1 page holds, after the counts, the value before each of
    # its 64-block segments but the first (the stride-0 page holds none)
    nset = bin(int(page[3])).count("1")
    sb = [int(v) for v in page[4 + nset:4 + nset + 7]]
    assert sb == [int(x[lo + g * 8192 - 1]) for g in range(1, 8)]
    h_ref, h_got = (4 + nset + 3) // 4 * 4, (4 + nset + 7 + 3) // 4 * 4
    assert np.array_equal(page[:4 + nset], ref[:4 + nset])
    assert np.array_equal(page[h_got:], ref[h_ref:])


def test_corrupt_streams_flagged_without_stray_writes():
    n = 2 * 65536 + 300
    x = datagen.patched_gaps(n, seed=79)
    s = oracle.fp32_encode(x, 1)
    rc, got = gpu_decode(s, n)
    assert rc == wp.OK and np.array_equal(got, x)
    unit = int(s[8])
    mutations = {
        "magic": (0, int(s[0]) ^ 1),
        "units": (4, int(s[4]) + 1),
        "total": (7, int(s[7]) + 100),
        "unit_offset": (8, 0xFFFFFF),
        "nblocks": (unit, 7),
        "packed_words": (unit + 1, int(s[unit + 1]) + 4),
        "bitset": (unit + 3, int(s[unit + 3]) ^ 0x80000000),
        "count": (unit + 4, int(s[unit + 4]) + 200),
    }
    for what, (at, val) in mutations.items():
        bad = s.copy()
        bad[at] = val & 0xFFFFFFFF
        print("fp32 corruption", what, flush=True)
        rc, _ = gpu_decode(bad, n)
        assert rc == wp.ERR_CORRUPT, what
        assert oracle.fp32_decode_rc(bad, n) == oracle.ERR_CORRUPT, what
    # a SIMD-FastPFOR stream is not a FastPFOR-32 stream
    rc, _ = gpu_decode(oracle.fp_encode(x, 1), n)
    assert rc == wp.ERR_CORRUPT
    rc, got = gpu_decode(s, n)
    assert rc == wp.OK and np.array_equal(got, x)
