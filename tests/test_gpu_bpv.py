"""GPU parity for SIMD-BP128 streams in the paper's four-lane (vectorized)
block layout (Section 4): the HIP decoder against the generators' arrays and
the oracle's streams, the HIP encoder against the oracle's encoder byte for
byte. Exact comparisons (integer work); outputs sit between canary fences
to catch writes outside [out, out + n)."""
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
# (waves, vpl, runs per CU, depth)
TUNES = [(4, 4, 28, 2), (1, 4, 4, 3), (2, 4, 64, 4), (8, 4, 16, 2), (4, 4, 1, 3)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    wp.lib()
    yield
    autotune.apply()


def to_dev(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if a.size == 0:
        return torch.zeros(0, dtype=torch.int32, device="cuda")
    return torch.from_numpy(a.view(np.int32)).to("cuda")


def to_host(t):
    return t.cpu().numpy().view(np.uint32)


def gpu_decode(stream_np, n):
    comp = to_dev(stream_np)
    buf = torch.full((n + 2 * PAD,), CANARY, dtype=torch.int32, device="cuda")
    out = buf[PAD:PAD + n]
    wp.bp_vertical_decode(comp, n, out)
    rc = wp.check_code()
    h = to_host(buf)
    assert (h[:PAD] == CANARY).all() and (h[PAD + n:] == CANARY).all(), "write outside [out, out + n)"
    return rc, h[PAD:PAD + n]


def assert_same(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[0]}: "
                             f"got {got[bad[0]]} want {want[bad[0]]}")


LENGTHS = [0, 1, 3, 4, 5, 31, 32, 33, 100, 127, 128, 129, 255, 256, 1000, 2047, 2048, 2049, 4096 + 127,
           3 * 2048 + 5, 65535, 65536, 65537, 2 * 65536 + 3 * 128 + 77]


def _case(rng, n):
    kind = n % 3
    if kind == 0:
        return rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    if kind == 1:
        return datagen.single_geometric(n, mean=float(rng.integers(2, 5000)), seed=n)
    return datagen.patched_gaps(n, seed=n) if n else np.zeros(0, np.uint32)


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_decode_lengths_strides_tunes(stride):
    rng = np.random.default_rng(4200 + stride)
    cases = []
    for n in LENGTHS:
        x = _case(rng, n)
        cases.append((n, x, oracle.bpv_encode(x, stride)))
    for waves, vpl, wpc, depth in TUNES:
        wp.set_decode_tune(wp.CODEC_BPV, waves, vpl, wpc, depth)
        for n, x, s in cases:
            print(f"bpv stride={stride} tune=({waves},{vpl},{wpc},{depth}) n={n}", flush=True)
            rc, got = gpu_decode(s, n)
            assert rc == wp.OK
            assert_same(got, x, f"n={n} tune=({waves},{vpl},{wpc},{depth})")


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_mixed_widths_every_offset(stride):
    # 150 meta-blocks whose 128-integer blocks take widths 0..32 in random
    # order, with stretches of 32-bit and of empty blocks (every row offset
    # and ring wrap-around), plus a tail
    rng = np.random.default_rng(191 + stride)
    nblk = 150 * 16
    widths = rng.integers(0, 33, size=nblk)
    widths[100:180] = 32
    widths[300:420] = 0
    widths[1000:1006] = [32, 0, 32, 1, 31, 32]
    d = []
    for j, b in enumerate(widths):
        hi = (1 << int(b)) - 1
        v = (rng.integers(0, 2**32, size=128, dtype=np.uint64) & hi).astype(np.uint32)
        v[j % 128] = hi
        d.append(v)
    d.append(rng.integers(0, 2**32, size=77, dtype=np.uint64).astype(np.uint32))
    d = np.concatenate(d)
    x = d if stride == 0 else np.cumsum(d.astype(np.uint64)).astype(np.uint32)
    if stride == 4:
        x = d.astype(np.uint64)
        for r in range(4):
            x[r::4] = np.cumsum(d[r::4].astype(np.uint64))
        x = x.astype(np.uint32)
    s = oracle.bpv_encode(x, stride)
    for waves, vpl, wpc, depth in TUNES:
        wp.set_decode_tune(wp.CODEC_BPV, waves, vpl, wpc, depth)
        print(f"bpv mixed stride={stride} tune=({waves},{vpl},{wpc},{depth})", flush=True)
        rc, got = gpu_decode(s, x.size)
        assert rc == wp.OK
        assert_same(got, x)


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_encode_matches_oracle(stride):
    rng = np.random.default_rng(4300 + stride)
    for n in LENGTHS + [(1 << 20) + 77]:
        x = _case(rng, n) if n < (1 << 20) else datagen.cluster_sorted(n, max_depth=14, seed=5)
        print(f"bpv encode stride={stride} n={n}", flush=True)
        want = oracle.bpv_encode(x, stride)
        got = to_host(wp.encode_trimmed(to_dev(x), wp.CODEC_BPV, stride)) if n else \
            to_host(wp.encode_trimmed(torch.zeros(4, dtype=torch.int32, device="cuda")[:0], wp.CODEC_BPV, stride))
        assert got.size == want.size and np.array_equal(got, want), f"n={n}"
        # and the GPU decodes its own stream
        rc, back = gpu_decode(got, n)
        assert rc == wp.OK and np.array_equal(back, x)


@pytest.mark.parametrize("stride", [1, 4])
def test_full_size_cluster_list(stride):
    # the 2^26 recursive-cluster list: GPU stream == oracle stream, decode == input
    x = datagen.cluster_sorted()
    want = oracle.bpv_encode(x, stride)
    xd = to_dev(x)
    comp = wp.encode_trimmed(xd, wp.CODEC_BPV, stride)
    assert comp.numel() == want.size and np.array_equal(to_host(comp), want)
    out = torch.empty(x.size, dtype=torch.int32, device="cuda")
    autotune.apply()
    wp.bp_vertical_decode(comp, x.size, out)
    assert wp.check_code() == wp.OK
    assert torch.equal(out, xd)


def test_corrupt_streams_flagged_without_stray_writes():
    n = 2 * 2048 * 5 + 300
    x = datagen.patched_gaps(n, seed=78)
    s = oracle.bpv_encode(x, 1)
    rc, got = gpu_decode(s, n)
    assert rc == wp.OK and np.array_equal(got, x)
    unit = int(s[8])
    mutations = {
        "magic": (0, int(s[0]) ^ 1),
        "stride": (3, 2),
        "units": (4, int(s[4]) + 1),
        "total": (7, int(s[7]) + 100),
        "unit_offset": (8, 0xFFFFFF),
        "tail_bytes": (5, int(s[5]) + 1),
        "width33": (unit, (int(s[unit]) & ~0xFF) | 33),
        "width_plus1": (unit, int(s[unit]) + 1),
    }
    for what, (at, val) in mutations.items():
        bad = s.copy()
        bad[at] = val & 0xFFFFFFFF
        print("bpv corruption", what, flush=True)
        rc, _ = gpu_decode(bad, n)
        assert rc == wp.ERR_CORRUPT, what
        assert oracle.bpv_decode_rc(bad, n) == oracle.ERR_CORRUPT, what
    # a sequential-layout SIMD-BP128 stream is not a four-lane one
    rc, _ = gpu_decode(oracle.bp_encode(x, 1), n)
    assert rc == wp.ERR_CORRUPT
    rc, _ = gpu_decode(s, n - 1)
    assert rc == wp.ERR_CORRUPT
    rc, got = gpu_decode(s, n)
    assert rc == wp.OK and np.array_equal(got, x)


def test_capacity_and_max_words():
    for n in (0, 1, 128, 2048, 65536 + 129, 10**6):
        assert wp.max_compressed_words(wp.CODEC_BPV, n) == oracle.max_words(oracle.CODEC_BPV, n)
    x = to_dev(np.arange(5000, dtype=np.uint32))
    small = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(wp.WavepackError):
        wp.bp_vertical_encode(x, 1, out=small)
