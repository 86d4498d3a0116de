"""Intersection of decoded posting lists on the GPU against the oracle's
two-pointer walk (exact comparison: integer work), over sizes that span
several 1024-element tiles with ragged ends, the full uint32 range, the
degenerate cases, and lists decoded from compressed streams."""
import numpy as np
import pytest
import torch

import oracle
import paper_1209_2137_amd as wp
from paper_1209_2137_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    wp.lib()


def dev(x):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    if x.size == 0:
        return torch.zeros(4, dtype=torch.int32, device="cuda")[:0]
    return torch.from_numpy(x.view(np.int32)).to("cuda")


def gpu_intersect(a, b):
    got = wp.intersect_trimmed(dev(a), dev(b))
    assert wp.check_code() == wp.OK
    return got.cpu().numpy().view(np.uint32)


def sorted_unique(rng, n, hi):
    return np.unique(rng.integers(0, hi, size=n, dtype=np.uint64)).astype(np.uint32)


@pytest.mark.parametrize("na,nb", [(1, 1), (5, 1000), (1023, 1024), (1024, 3000), (1025, 50), (4096 + 7, 4096 + 9),
                                   (100_003, 1_000_000), (1_000_000, 100_003)])
def test_intersect_matches_oracle(na, nb):
    rng = np.random.default_rng(na * 7 + nb)
    for hi in (2 * (na + nb), 2**32):
        a, b = sorted_unique(rng, na, hi), sorted_unique(rng, nb, hi)
        print(f"intersect na={a.size} nb={b.size} hi={hi}", flush=True)
        got = gpu_intersect(a, b)
        want = oracle.intersect(a, b)
        assert got.size == want.size and np.array_equal(got, want)


def test_intersect_degenerate_cases():
    e = np.zeros(0, np.uint32)
    x = np.arange(0, 3000, 3, dtype=np.uint32)
    assert gpu_intersect(e, x).size == 0
    assert gpu_intersect(x, e).size == 0
    assert np.array_equal(gpu_intersect(x, x), x)
    assert gpu_intersect(x, x + 1).size == 0
    sub = x[::7].copy()
    assert np.array_equal(gpu_intersect(sub, x), sub)
    assert np.array_equal(gpu_intersect(x, sub), sub)
    top = np.array([0, 2**31 - 1, 2**31, 2**32 - 2, 2**32 - 1], dtype=np.uint32)
    assert np.array_equal(gpu_intersect(top, top[1:]), top[1:])


def test_intersect_decoded_posting_lists():
    # two posting lists decoded from their compressed streams, intersected
    # on the device; against the oracle on the generator's arrays
    a = datagen.cluster_sorted(1 << 18, seed=11)
    b = datagen.cluster_sorted(1 << 21, seed=12)
    ca = wp.encode_trimmed(dev(a), wp.CODEC_BP, 1)
    cb = wp.encode_trimmed(dev(b), wp.CODEC_FP, 1)
    da = wp.bp_decode(ca, a.size)
    db = wp.fastpfor_decode(cb, b.size)
    got = wp.intersect_trimmed(da, db)
    assert wp.check_code() == wp.OK
    want = oracle.intersect(a, b)
    assert want.size > 0
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)


@pytest.mark.parametrize("codec", [wp.CODEC_BP, wp.CODEC_FP, wp.CODEC_BP32, wp.CODEC_FP32, wp.CODEC_BPV])
@pytest.mark.parametrize("stride", [0, 1, 4])
def test_intersect_compressed_matches_oracle(codec, stride):
    # the long list stays compressed: only the units the short list can
    # touch are decoded; ragged lengths (partial last unit and a tail)
    rng = np.random.default_rng(90 + 10 * codec + stride)
    for nb, na, hi in ((200_000 + 77, 300, 1 << 26), (70_000 + 5, 5000, 1 << 20), (128 * 17, 40, 1 << 16),
                       (100, 30, 1000), (300_000, 1, 1 << 30)):
        b = sorted_unique(rng, nb, hi)
        a = sorted_unique(rng, na, hi)
        if a.size > 4:  # make sure some values are common
            a = np.unique(np.concatenate([a, b[rng.integers(0, b.size, size=a.size // 4)]])).astype(np.uint32)
        comp = wp.encode_trimmed(dev(b), codec, stride)
        print(f"compressed intersect codec={codec} stride={stride} na={a.size} nb={b.size}", flush=True)
        out, count, work = wp.intersect_compressed(dev(a), comp, b.size, codec)
        assert wp.check_code() == wp.OK
        got = out[: int(count.item())].cpu().numpy().view(np.uint32)
        want = oracle.intersect(a, b)
        assert got.size == want.size and np.array_equal(got, want)


def test_intersect_compressed_decodes_only_touched_units():
    # one value of a in the middle of a long list: everything outside the
    # unit that holds it keeps the work buffer's fill pattern
    b = np.arange(1, 2 * 2048 * 40, 2, dtype=np.uint32)  # 81920 odd values, 40 meta-blocks
    comp = wp.encode_trimmed(dev(b), wp.CODEC_BP, 1)
    a = np.array([b[2048 * 7 + 100]], dtype=np.uint32)
    work = torch.full((b.size,), -1, dtype=torch.int32, device="cuda")
    out, count, work = wp.intersect_compressed(dev(a), comp, b.size, wp.CODEC_BP, work=work)
    assert wp.check_code() == wp.OK
    assert int(count.item()) == 1 and int(out[0].item()) == int(a[0])
    w = work.cpu().numpy().view(np.uint32)
    assert np.array_equal(w[2048 * 7:2048 * 8], b[2048 * 7:2048 * 8])
    untouched = np.ones(b.size, bool)
    untouched[2048 * 7:2048 * 8] = False
    assert np.all(w[untouched] == 0xFFFFFFFF)


@pytest.mark.parametrize("codec", [wp.CODEC_BP, wp.CODEC_FP, wp.CODEC_BP32, wp.CODEC_FP32, wp.CODEC_BPV])
def test_intersect_compressed_corrupt_and_empty(codec):
    b = np.arange(3, 3 * 5000, 3, dtype=np.uint32)
    comp = wp.encode_trimmed(dev(b), codec, 1)
    a = dev(b[::7])
    # a header that disagrees with nb is reported, nothing is read beyond it
    out, count, _ = wp.intersect_compressed(a, comp, b.size + 128, codec)
    assert wp.check_code() == wp.ERR_CORRUPT
    assert wp.check_code() == wp.OK
    # empty first list, or an empty second list
    out, count, _ = wp.intersect_compressed(dev(np.zeros(0, np.uint32)), comp, b.size, codec)
    assert int(count.item()) == 0
    empty = wp.encode_trimmed(dev(np.zeros(0, np.uint32)), codec, 1)
    out, count, _ = wp.intersect_compressed(a, empty, 0, codec)
    assert int(count.item()) == 0 and wp.check_code() == wp.OK
    # values beyond the largest of b, and below the smallest
    a2 = dev(np.array([0, 1, 2, 0xFFFFFFF0, 0xFFFFFFFF], np.uint32))
    out, count, _ = wp.intersect_compressed(a2, comp, b.size, codec)
    assert int(count.item()) == 0 and wp.check_code() == wp.OK
