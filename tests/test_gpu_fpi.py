"""GPU parity for FastPFOR pages in the paper's own layout (Section 5 and
its page-layout figure: offset word, truncated values, counted byte array,
bitset and counted exception arrays): the HIP decoder against the
generators' arrays and the oracle's streams (byte arrays held in LDS and,
when too long for it, read from the page), the HIP encoder against the
oracle's encoder word for word. Exact comparisons (integer work); outputs
sit between canary fences to catch writes outside [out, out + n)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1209_2137_amd as wp
from paper_1209_2137_amd import datagen

pytestmark = pytest.mark.gpu

CANARY = 0x5A5A5A5A
PAD = 64


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    wp.lib()


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
    wp.fastpfor_inline_decode(comp, n, out)
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
def test_decode_and_encode_lengths_strides(stride):
    rng = np.random.default_rng(7200 + stride)
    for n in LENGTHS:
        x = _case(rng, n)
        want = oracle.fpi_encode(x, stride)
        print(f"fpi stride={stride} n={n}", flush=True)
        rc, got = gpu_decode(want, n)
        assert rc == wp.OK
        assert_same(got, x, f"decode n={n}")
        enc = to_host(wp.encode_trimmed(to_dev(x), wp.CODEC_FPI, stride))
        assert enc.size == want.size, f"n={n}: {enc.size} words, oracle {want.size}"
        assert_same(enc, want, f"encode n={n}")


@pytest.mark.parametrize("wide_frac", [0.001, 0.05, 0.3])
def test_byte_arrays_in_lds_and_from_the_page(wide_frac):
    # few to many exceptions: at 30 % a full page's byte array (512 records
    # of 3 + c bytes, c about 38) outgrows the 12 KB the decoder holds in
    # LDS, and is read from the page instead
    rng = np.random.default_rng(int(wide_frac * 1000))
    n = 3 * 65536 + 128 * 7 + 5
    small = rng.integers(0, 16, size=n, dtype=np.uint64)
    wide = rng.integers(1 << 20, 1 << 24, size=n, dtype=np.uint64)
    x = np.cumsum(np.where(rng.random(n) < wide_frac, wide, small)).astype(np.uint32)
    want = oracle.fpi_encode(x, 1)
    p0 = int(want[8])
    nba = int(want[p0 + int(want[p0])])
    print(f"fpi wide_frac={wide_frac}: first page byte array {nba} bytes", flush=True)
    if wide_frac >= 0.3:
        assert nba > 12 * 1024
    elif wide_frac <= 0.05:
        assert nba <= 12 * 1024
    rc, got = gpu_decode(want, n)
    assert rc == wp.OK
    assert_same(got, x)
    enc = to_host(wp.encode_trimmed(to_dev(x), wp.CODEC_FPI, 1))
    assert_same(enc, want, "encode")


def test_full_size_patched_list():
    # the 2^28 patched workload in the paper's layout: GPU encode, GPU
    # decode, exact round trip; a sampled page equals the oracle's page
    x = datagen.patched_gaps()
    xd = to_dev(x)
    comp = wp.encode_trimmed(xd, wp.CODEC_FPI, 1)
    out = torch.empty(xd.numel(), dtype=torch.int32, device="cuda")
    wp.fastpfor_inline_decode(comp, xd.numel(), out)
    assert wp.check_code() == wp.OK
    assert torch.equal(out, xd)
    s = to_host(comp[:8 + 4096 * 2 + 8])
    off, end = int(s[8 + 1000]), int(s[8 + 1001])
    page = to_host(comp[off:end])
    lo = 1000 * 65536
    seg = x[lo:lo + 65536].astype(np.uint64)
    d = np.empty(65536, np.uint64)
    d[0] = (seg[0] - np.uint64(x[lo - 1])) % (1 << 32)
    d[1:] = (seg[1:] - seg[:-1]) % (1 << 32)
    ref = oracle.fpi_encode(d.astype(np.uint32), 0)
    assert np.array_equal(page, ref[int(ref[8]):int(ref[6])])


def test_corrupt_streams_flagged_without_stray_writes():
    n = 2 * 65536 + 300
    x = datagen.patched_gaps(n, seed=83)
    s = oracle.fpi_encode(x, 1)
    rc, got = gpu_decode(s, n)
    assert rc == wp.OK and np.array_equal(got, x)
    p0 = int(s[8])
    cpos = p0 + int(s[p0])
    nba = int(s[cpos])
    xp = cpos + 1 + -(-nba // 4)
    mutations = {
        "magic": (0, int(s[0]) ^ 1),
        "unit_offset": (8, 0xFFFFFF),
        "offset_word": (p0, int(s[p0]) + 4),
        "byte_counter": (cpos, nba + 1),
        "first_width": (cpos + 1, (int(s[cpos + 1]) & ~0xFF) | 40),
        "bitset": (xp, int(s[xp]) ^ 0x80000000),
        "array_counter": (xp + 1, int(s[xp + 1]) + 40),
    }
    for what, (at, val) in mutations.items():
        bad = s.copy()
        bad[at] = val & 0xFFFFFFFF
        print("fpi corruption", what, flush=True)
        rc, _ = gpu_decode(bad, n)
        assert rc == wp.ERR_CORRUPT, what
        assert oracle.fpi_decode_rc(bad, n) == oracle.ERR_CORRUPT, what
    rc, _ = gpu_decode(oracle.fp32_encode(x, 1), n)
    assert rc == wp.ERR_CORRUPT
    rc, got = gpu_decode(s, n)
    assert rc == wp.OK and np.array_equal(got, x)
