"""GPU parity: the HIP decoders against the CPU oracle and the generators.

Streams are produced by the oracle's encoder; the expected output is the
generator's array itself (decoding is lossless, so decode(encode(x)) == x is
the plain definition of the result). Comparisons are exact (integer work).
Outputs sit between canary fences to catch writes outside [out, out + n).
"""
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
# (waves, vpl, runs or workgroups per CU, depth)
BP_TUNES = [(4, 4, 28, 2), (1, 4, 4, 3), (2, 4, 64, 4), (8, 4, 16, 2), (4, 4, 1, 3)]
FP_TUNES = [(8, 4, 0, 0), (4, 4, 0, 0), (2, 4, 0, 0), (1, 4, 0, 0)]


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


def gpu_decode(codec, stream_np, n):
    comp = to_dev(stream_np)
    buf = torch.full((n + 2 * PAD,), CANARY, dtype=torch.int32, device="cuda")
    out = buf[PAD:PAD + n]
    (wp.bp_decode if codec == wp.CODEC_BP else wp.fastpfor_decode)(comp, n, out)
    rc = wp.check_code()
    h = to_host(buf)
    assert (h[:PAD] == CANARY).all() and (h[PAD + n:] == CANARY).all(), "write outside [out, out + n)"
    return rc, h[PAD:PAD + n]


def encode(codec, x, stride):
    return (oracle.bp_encode if codec == wp.CODEC_BP else oracle.fp_encode)(x, stride)


def assert_same(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[0]}: "
                             f"got {got[bad[0]]} want {want[bad[0]]}")


LENGTHS = [0, 1, 3, 4, 5, 100, 127, 128, 129, 255, 256, 1000, 2047, 2048, 2049, 4096 + 127,
           3 * 2048 + 5, 65535, 65536, 65537, 2 * 65536 + 3 * 128 + 77]


@pytest.mark.parametrize("codec,tunes", [(wp.CODEC_BP, BP_TUNES), (wp.CODEC_FP, FP_TUNES)])
@pytest.mark.parametrize("stride", [0, 1, 4])
def test_lengths_strides_tunes(codec, tunes, stride):
    rng = np.random.default_rng(1000 * codec + stride)
    cases = []
    for n in LENGTHS:
        kind = n % 3
        if kind == 0:
            x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        elif kind == 1:
            x = datagen.single_geometric(n, mean=float(rng.integers(2, 5000)), seed=n)
        else:
            x = datagen.patched_gaps(n, seed=n) if n else np.zeros(0, np.uint32)
        cases.append((n, x, encode(codec, x, stride)))
    for waves, vpl, wpc, depth in tunes:
        wp.set_decode_tune(codec, waves, vpl, wpc, depth)
        for n, x, s in cases:
            print(f"codec={codec} stride={stride} tune=({waves},{vpl},{wpc},{depth}) n={n}", flush=True)
            rc, got = gpu_decode(codec, s, n)
            assert rc == wp.OK
            assert_same(got, x, f"n={n} tune=({waves},{vpl},{wpc},{depth})")


@pytest.mark.parametrize("codec", [wp.CODEC_BP, wp.CODEC_FP])
def test_every_block_width(codec):
    # 33 blocks, block j holds values of exactly j bits (one at 2^j - 1), stride 0
    rng = np.random.default_rng(5)
    blocks = []
    for b in range(33):
        hi = (1 << b) - 1
        v = (rng.integers(0, 2**32, size=128, dtype=np.uint64) & hi).astype(np.uint32)
        v[int(rng.integers(0, 128))] = hi
        blocks.append(v)
    x = np.concatenate(blocks + [np.array([7, 1 << 31, 5], dtype=np.uint32)])
    tunes = BP_TUNES if codec == wp.CODEC_BP else FP_TUNES
    for waves, vpl, wpc, depth in tunes:
        wp.set_decode_tune(codec, waves, vpl, wpc, depth)
        rc, got = gpu_decode(codec, encode(codec, x, 0), x.size)
        assert rc == wp.OK
        assert_same(got, x)


@pytest.mark.parametrize("stride", [0, 1])
def test_mixed_block_widths_long_runs(stride):
    # 150 meta-blocks whose blocks take widths 0..32 in random order, with
    # stretches of 32-bit and of empty blocks: passes that read 0..256 words,
    # ring wrap-around at every offset, runs of every length; plus a tail
    rng = np.random.default_rng(77 + stride)
    nblk = 150 * 16
    widths = rng.integers(0, 33, size=nblk)
    widths[100:180] = 32
    widths[300:420] = 0
    widths[1000:1003] = [32, 0, 32]
    d = []
    for j, b in enumerate(widths):
        hi = (1 << int(b)) - 1
        v = (rng.integers(0, 2**32, size=128, dtype=np.uint64) & hi).astype(np.uint32)
        v[j % 128] = hi
        d.append(v)
    d.append(rng.integers(0, 2**32, size=77, dtype=np.uint64).astype(np.uint32))
    d = np.concatenate(d)
    x = d if stride == 0 else np.cumsum(d.astype(np.uint64)).astype(np.uint32)
    s = encode(wp.CODEC_BP, x, stride)
    for waves, vpl, wpc, depth in BP_TUNES:
        wp.set_decode_tune(wp.CODEC_BP, waves, vpl, wpc, depth)
        print(f"stride={stride} tune=({waves},{vpl},{wpc},{depth}) n={x.size}", flush=True)
        rc, got = gpu_decode(wp.CODEC_BP, s, x.size)
        assert rc == wp.OK
        assert_same(got, x, f"tune=({waves},{vpl},{wpc},{depth})")


def test_config_small_single_list():
    # 2^20 sorted integers, x_1 ~ U[0,1000), geometric gaps of mean 8
    x = datagen.single_geometric(1 << 20, mean=8.0, seed=1)
    for codec in (wp.CODEC_BP, wp.CODEC_FP):
        for stride in (1, 4):
            rc, got = gpu_decode(codec, encode(codec, x, stride), x.size)
            assert rc == wp.OK
            assert_same(got, x)


def test_full_size_binary_packing_lists():
    # the 2^26 single-list workloads: recursive-cluster and uniform distinct values
    for x in (datagen.cluster_sorted(), datagen.uniform_sorted()):
        s = oracle.bp_encode(x, 1)
        comp = to_dev(s)
        out = torch.empty(x.size, dtype=torch.int32, device="cuda")
        autotune.apply()  # the tuned launch shape, as timed by the benchmark
        wp.bp_decode(comp, x.size, out)
        assert wp.check_code() == wp.OK
        assert torch.equal(out, to_dev(x))


def test_full_size_patched_list():
    # the 2^28 patched workload (wraps modulo 2^32)
    x = datagen.patched_gaps()
    s = oracle.fp_encode(x, 1)
    comp = to_dev(s)
    xd = to_dev(x)
    del x
    out = torch.empty(xd.numel(), dtype=torch.int32, device="cuda")
    autotune.apply()
    wp.fastpfor_decode(comp, xd.numel(), out)
    assert wp.check_code() == wp.OK
    assert torch.equal(out, xd)


@pytest.mark.parametrize("codec", [wp.CODEC_BP, wp.CODEC_BPV, wp.CODEC_BP32])
def test_full_size_binary_packing_every_shape(codec):
    # the 2^26 cluster list in every binary-packing layout, decoded with
    # every launch shape of the tests above (wavefronts per workgroup, runs
    # per compute unit, loads in flight), twice each, at full occupancy
    x = datagen.cluster_sorted()
    xd = to_dev(x)
    del x
    comp = wp.encode_trimmed(xd, codec, 1)
    dec = {wp.CODEC_BP: wp.bp_decode, wp.CODEC_BPV: wp.bp_vertical_decode, wp.CODEC_BP32: wp.bp32_decode}[codec]
    out = torch.empty(xd.numel(), dtype=torch.int32, device="cuda")
    for waves, vpl, wpc, depth in BP_TUNES + [(4, 4, 256, 3), (4, 4, 128, 2)]:
        wp.set_decode_tune(codec, waves, vpl, wpc, depth)
        for rep in range(2):
            out.fill_(-1)
            dec(comp, xd.numel(), out)
            assert wp.check_code() == wp.OK
            bad = int((out != xd).sum().item())
            print(f"codec={codec} tune=({waves},{vpl},{wpc},{depth}) run {rep}: {bad} mismatches", flush=True)
            assert bad == 0
    autotune.apply()


def test_full_size_patched_list_every_shape():
    # the 2^28 patched list with two, four and eight wavefronts per page:
    # with two, the 16-byte output stores once took a register overwritten
    # right behind them (element 2 of the last four lanes of each row held
    # the block width) -- only at this size, where many workgroups share
    # each compute unit
    x = datagen.patched_gaps()
    xd = to_dev(x)
    del x
    comp = wp.encode_trimmed(xd, wp.CODEC_FP, 1)
    out = torch.empty(xd.numel(), dtype=torch.int32, device="cuda")
    for waves in (2, 4, 8):
        wp.set_decode_tune(wp.CODEC_FP, waves, 4)
        for rep in range(2):
            out.fill_(-1)
            wp.fastpfor_decode(comp, xd.numel(), out)
            assert wp.check_code() == wp.OK
            bad = int((out != xd).sum().item())
            print(f"waves={waves} run {rep}: {bad} mismatches", flush=True)
            assert bad == 0
    autotune.apply()


@pytest.mark.parametrize("codec", [wp.CODEC_BP, wp.CODEC_FP])
def test_corrupt_streams_flagged_without_stray_writes(codec):
    n = 2 * 65536 + 300
    x = datagen.patched_gaps(n, seed=77)
    s = encode(codec, x, 1)
    rc, got = gpu_decode(codec, s, n)
    assert rc == wp.OK and np.array_equal(got, x)
    unit = int(s[8])
    mutations = {
        "magic": (0, int(s[0]) ^ 1),
        "stride": (3, 2),
        "units": (4, int(s[4]) + 1),
        "total": (7, int(s[7]) + 100),
        "unit_offset": (8, 0xFFFFFF),
        "tail_bytes": (5, int(s[5]) + 1),
    }
    if codec == wp.CODEC_BP:
        mutations["width33"] = (unit, (int(s[unit]) & ~0xFF) | 33)
    else:
        mutations["nblocks"] = (unit, 7)
        mutations["packed_words"] = (unit + 1, int(s[unit + 1]) + 4)
        mutations["bitset"] = (unit + 3, int(s[unit + 3]) ^ 0x80000000)
    for what, (at, val) in mutations.items():
        bad = s.copy()
        bad[at] = val & 0xFFFFFFFF
        print("corruption", what, flush=True)
        rc, _ = gpu_decode(codec, bad, n)
        assert rc == wp.ERR_CORRUPT, what
        # the oracle agrees that the stream is bad
        assert (oracle.bp_decode_rc if codec == wp.CODEC_BP else oracle.fp_decode_rc)(bad, n) == oracle.ERR_CORRUPT
    # wrong n: flagged as well
    rc, _ = gpu_decode(codec, s, n - 1)
    assert rc == wp.ERR_CORRUPT
    # a good decode afterwards is clean again
    rc, got = gpu_decode(codec, s, n)
    assert rc == wp.OK and np.array_equal(got, x)


def dense_exception_deltas(rng, nblocks, per_block):
    """Deltas whose blocks hold `per_block[j]` values of 20..24 bits among
    zeros: the cost rule then keeps b = 0 and makes every one of them an
    exception (up to about 90 per block), so a pass of four blocks can hold
    far more than 64."""
    d = np.zeros(nblocks * 128, dtype=np.uint32)
    for j in range(nblocks):
        c = int(per_block[j])
        pos = rng.choice(128, size=c, replace=False)
        d[j * 128 + pos] = rng.integers(1 << 19, 1 << 24, size=c).astype(np.uint32)
    return d


@pytest.mark.parametrize("stride", [0, 1, 4])
def test_patched_dense_exceptions(stride):
    # passes with 0..360 exceptions (one per lane, then rounds of 64 more),
    # blocks of up to 90, on pages of every fill; plus a tail
    rng = np.random.default_rng(900 + stride)
    nblocks = 512 + 200
    per = rng.integers(0, 91, size=nblocks)
    per[:8] = 90
    per[8:16] = 0
    per[40:44] = [1, 90, 2, 89]
    d = np.concatenate([dense_exception_deltas(rng, nblocks, per), np.arange(1, 51, dtype=np.uint32)])
    if stride == 0:
        x = d
    elif stride == 1:
        x = np.cumsum(d.astype(np.uint64)).astype(np.uint32)
    else:
        x = d.astype(np.uint64).copy()
        for c in range(4):
            x[c::4] = np.cumsum(x[c::4])
        x = x.astype(np.uint32)
    s = encode(wp.CODEC_FP, x, stride)
    for waves, vpl, wpc, depth in FP_TUNES:
        wp.set_decode_tune(wp.CODEC_FP, waves, vpl, wpc, depth)
        print(f"dense exceptions stride={stride} waves={waves}", flush=True)
        rc, got = gpu_decode(wp.CODEC_FP, s, x.size)
        assert rc == wp.OK
        assert_same(got, x, f"waves={waves}")
    autotune.apply()


def _page_meta(s, n):
    """Word offset of the first page, its block count and the byte offset
    (from the stream start) of its metadata."""
    unit = int(s[8])
    stride = int(s[3])
    nb, packed, bitset = int(s[unit]), int(s[unit + 1]), int(s[unit + 3])
    # 4 words, a count per non-empty array, the segment bases, padded to 4
    hdr = (4 + bin(bitset).count("1") + stride * (-(-nb // 64) - 1) + 3) & ~3
    return unit, nb, 4 * (unit + hdr + packed)


def test_patched_corrupt_metadata_flagged():
    # exception positions out of order or past the block, and a block whose
    # exception count disagrees with its widths: the GPU and the oracle both
    # reject the stream, and the decode stays inside [out, out + n)
    n = 2 * 65536 + 300
    x = datagen.patched_gaps(n, seed=78)
    s = encode(wp.CODEC_FP, x, 1)
    unit, nb, meta = _page_meta(s, n)
    by = s.view(np.uint8)
    c = by[meta + 2 * nb: meta + 3 * nb].astype(np.int64)
    t = int(np.nonzero(c >= 2)[0][3])           # a block with at least two exceptions
    p0 = meta + 3 * nb + int(c[:t].sum())        # its first position byte
    cases = {}
    b = s.copy(); bb = b.view(np.uint8); bb[p0], bb[p0 + 1] = bb[p0 + 1], bb[p0]; cases["positions_swapped"] = b
    b = s.copy(); bb = b.view(np.uint8); bb[p0 + 1] = bb[p0]; cases["position_repeated"] = b
    b = s.copy(); bb = b.view(np.uint8); bb[p0] = 200; cases["position_past_block"] = b
    b = s.copy(); bb = b.view(np.uint8); bb[meta + 2 * nb + t] = 0; cases["count_without_width_gap"] = b
    b = s.copy(); bb = b.view(np.uint8); bb[meta + t] = 40; cases["width_40"] = b
    for what, bad in cases.items():
        print("corruption", what, flush=True)
        for waves in (1, 4):
            wp.set_decode_tune(wp.CODEC_FP, waves, 4)
            rc, _ = gpu_decode(wp.CODEC_FP, bad, n)
            assert rc == wp.ERR_CORRUPT, (what, waves)
        assert oracle.fp_decode_rc(bad, n) == oracle.ERR_CORRUPT, what
    autotune.apply()
    rc, got = gpu_decode(wp.CODEC_FP, s, n)
    assert rc == wp.OK and np.array_equal(got, x)


DELTA_SIZES = [1, 3, 4, 5, 4095, 4096, 4097, 12345, 32767, 32768, 32769, 3 * 32768 + 5, 1 << 20, (1 << 22) + 3]


@pytest.mark.parametrize("stride", [1, 4])
def test_delta_decode_inplace_matches_oracle(stride):
    rng = np.random.default_rng(stride)
    for n in DELTA_SIZES:
        for init in (0, 0xFFFFFFF0):
            d = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
            want = d.copy()
            oracle.delta_decode_inplace(want, init, stride)
            t = to_dev(d)
            wp.delta_decode_inplace(t, init, stride)
            torch.cuda.synchronize()
            print(f"delta n={n} stride={stride} init={init:#x}", flush=True)
            assert_same(to_host(t), want, f"n={n}")


def test_delta_decode_inplace_paper_example():
    t = to_dev(np.array([1, 3, 9], dtype=np.uint32))
    wp.delta_decode_inplace(t, 0, 1)
    assert list(to_host(t)) == [1, 4, 13]


def test_delta_decode_inplace_large_repeatable():
    n = (1 << 26) + 1
    rng = np.random.default_rng(9)
    d = rng.integers(0, 1 << 8, size=n, dtype=np.uint64).astype(np.uint32)
    want = (np.cumsum(d.astype(np.uint64)) & 0xFFFFFFFF).astype(np.uint32)
    for _ in range(2):
        t = to_dev(d)
        wp.delta_decode_inplace(t, 0, 1)
        torch.cuda.synchronize()
        assert_same(to_host(t), want)


def test_time_next_launch_brackets_the_kernel():
    # the timing hook records the caller's events around the decoder's own
    # kernel; the decode is unchanged and the hook is consumed by one call
    x = datagen.single_geometric(1 << 20, mean=8.0, seed=11)
    comp = to_dev(oracle.bp_encode(x, 1))
    out = torch.empty(x.size, dtype=torch.int32, device="cuda")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    stop.record()
    torch.cuda.synchronize()
    wp.time_next_launch(start, stop)
    wp.bp_decode(comp, x.size, out)
    stop.synchronize()
    ms = start.elapsed_time(stop)
    assert wp.check_code() == wp.OK
    assert_same(out.cpu().numpy().view(np.uint32), x)
    assert 0.0 < ms < 100.0
    wp.bp_decode(comp, x.size, out)  # no events pending: a plain launch
    torch.cuda.synchronize()
    assert wp.check_code() == wp.OK
