"""GPU encoders against the CPU oracle: the streams must be identical word
for word (every width choice, offset, padding byte and exception array)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1209_2137_amd as wp
from paper_1209_2137_amd import datagen
from tests.test_gpu_decode import LENGTHS, assert_same, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    wp.lib()


def gpu_encode(codec, x, stride):
    t = to_dev(x)
    if t.numel() == 0:
        t = torch.zeros(4, dtype=torch.int32, device="cuda")[:0]
    buf, words = (wp.bp_encode if codec == wp.CODEC_BP else wp.fastpfor_encode)(t, stride)
    assert wp.check_code() == wp.OK
    w = int(words.item())
    return to_host(buf[:w])


def oracle_encode(codec, x, stride):
    return (oracle.bp_encode if codec == wp.CODEC_BP else oracle.fp_encode)(x, stride)


@pytest.mark.parametrize("codec", [wp.CODEC_BP, wp.CODEC_FP])
@pytest.mark.parametrize("stride", [0, 1, 4])
def test_encode_matches_oracle(codec, stride):
    rng = np.random.default_rng(50 + 10 * codec + stride)
    for n in LENGTHS:
        for kind in range(3):
            if kind == 0:
                x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
            elif kind == 1:
                x = datagen.single_geometric(n, mean=float(rng.integers(2, 5000)), seed=n + 1)
            else:
                x = datagen.patched_gaps(n, seed=n + 2) if n else np.zeros(0, np.uint32)
            print(f"encode codec={codec} stride={stride} n={n} kind={kind}", flush=True)
            got = gpu_encode(codec, x, stride)
            want = oracle_encode(codec, x, stride)
            assert got.size == want.size, (n, kind, got.size, want.size)
            assert_same(got, want, f"n={n} kind={kind}")


@pytest.mark.parametrize("codec", [wp.CODEC_BP, wp.CODEC_FP])
def test_encode_every_width(codec):
    rng = np.random.default_rng(8)
    blocks = []
    for b in list(range(33)) + list(range(32, -1, -1)):
        hi = (1 << b) - 1
        v = (rng.integers(0, 2**32, size=128, dtype=np.uint64) & hi).astype(np.uint32)
        v[int(rng.integers(0, 128))] = hi
        blocks.append(v)
    x = np.concatenate(blocks)
    for stride in (0, 1, 4):
        assert_same(gpu_encode(codec, x, stride), oracle_encode(codec, x, stride))


def test_encode_full_sizes():
    for codec, x in ((wp.CODEC_BP, datagen.cluster_sorted()), (wp.CODEC_BP, datagen.uniform_sorted()),
                     (wp.CODEC_FP, datagen.patched_gaps())):
        print("full-size encode", codec, x.size, flush=True)
        got = gpu_encode(codec, x, 1)
        want = oracle_encode(codec, x, 1)
        assert got.size == want.size
        assert np.array_equal(got, want)


def test_encode_capacity_and_argument_errors():
    x = to_dev(datagen.single_geometric(5000, seed=1))
    cap = wp.max_compressed_words(wp.CODEC_BP, 5000)
    out = torch.empty(cap, dtype=torch.int32, device="cuda")
    words = torch.zeros(1, dtype=torch.int64, device="cuda")
    L = wp.lib()
    s = wp._stream(None)
    assert L.bp_encode(wp._ptr(x), 5000, 1, wp._ptr(out), cap - 1, wp._ptr(words), s) == wp.ERR_CAPACITY
    assert L.bp_encode(wp._ptr(x), 5000, 3, wp._ptr(out), cap, wp._ptr(words), s) == wp.ERR_INVALID_ARG
    assert L.fastpfor_encode(wp._ptr(x), 5000, 1, None, cap, wp._ptr(words), s) == wp.ERR_INVALID_ARG
    assert L.bp_encode(wp._ptr(x), 5000, 1, wp._ptr(out), cap, wp._ptr(words), s) == wp.OK
    assert wp.check_code() == wp.OK


def test_gpu_roundtrip_of_gpu_streams():
    # GPU encode then GPU decode reproduces the input (both codecs, strides)
    x = datagen.patched_gaps(3 * 65536 + 1111, seed=3)
    xd = to_dev(x)
    for codec in (wp.CODEC_BP, wp.CODEC_FP):
        for stride in (0, 1, 4):
            comp = wp.encode_trimmed(xd, codec, stride)
            out = (wp.bp_decode if codec == wp.CODEC_BP else wp.fastpfor_decode)(comp, x.size)
            assert wp.check_code() == wp.OK
            assert torch.equal(out, xd)


@pytest.mark.parametrize("wide_frac", [0.05, 0.15, 0.4])
def test_fastpfor_encode_exception_heavy_pages(wide_frac):
    # pages whose metadata and exception arrays take from a few KB to more
    # than 32 KB (the encoder assembles them in LDS when they fit and in
    # place in HBM otherwise): both forms give the oracle's stream
    rng = np.random.default_rng(int(wide_frac * 100))
    n = 3 * 65536 + 128 * 7 + 5
    small = rng.integers(0, 16, size=n, dtype=np.uint64)
    wide = rng.integers(1 << 20, 1 << 24, size=n, dtype=np.uint64)
    x = np.where(rng.random(n) < wide_frac, wide, small).astype(np.uint32)
    got = gpu_encode(wp.CODEC_FP, x, 0)
    want = oracle_encode(wp.CODEC_FP, x, 0)
    assert got.size == want.size
    assert_same(got, want, f"wide_frac={wide_frac}")
    # the page tails: metadata + exception words after the packed words
    hdr_words = 8
    p0 = int(want[hdr_words])
    nb, packed, meta_bytes, bitset = (int(v) for v in want[p0:p0 + 4])
    assert nb == 512
    p1 = int(want[hdr_words + 1])
    hdr_w = (4 + bin(bitset).count("1") + 3) & ~3
    tail_words = (p1 - p0) - hdr_w - packed
    print(f"wide_frac={wide_frac}: first page tail {4 * tail_words} bytes", flush=True)


def test_binary_packing_encode_tiles_mixed_and_ragged():
    """Lists cut at and around the binary-packing encoder's tiles of 8
    meta-blocks (16384 integers), where every other tile holds 32-bit
    values (too long for the tile's LDS assembly, so it is assembled a
    meta-block at a time) and the others compress: both block layouts and
    every stride, word for word against the oracle."""
    rng = np.random.default_rng(77)
    tile = 8 * 2048
    for n in (tile - 1, tile, tile + 1, tile + 128, 3 * tile - 129, 3 * tile + 2047, 5 * tile + 3):
        x = datagen.single_geometric(n, mean=20.0, seed=n)
        for t in range(1, n // tile + 1, 2):
            hi = min(n, (t + 1) * tile)
            x[t * tile:hi] = rng.integers(0, 2**32, size=hi - t * tile, dtype=np.uint64).astype(np.uint32)
        for codec, enc in ((wp.CODEC_BP, oracle.bp_encode), (wp.CODEC_BPV, oracle.bpv_encode)):
            for stride in (0, 1, 4):
                print(f"tiles codec={codec} stride={stride} n={n}", flush=True)
                got = to_host(wp.encode_trimmed(to_dev(x), codec, stride))
                assert wp.check_code() == wp.OK
                want = enc(x, stride)
                assert got.size == want.size, (n, codec, stride)
                assert_same(got, want, f"n={n} codec={codec} stride={stride}")
