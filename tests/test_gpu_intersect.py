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
