"""Random access by key on the GPU: wp_decode_range against the definition
of the range (the first index whose value is >= key_lo and the first whose
value is > key_hi, i.e. numpy's searchsorted on the input) and against the
input's values in that range. Exact comparisons (integer work). Lists that
are strictly increasing and lists with long runs of equal values straddling
unit boundaries; key ranges that are empty, hit one value, sit exactly on a
unit's stored base, lie before the first or after the last value, or span
the whole list; every codec and stride. The output sits between canary
fences, and a narrow range must leave most of it untouched."""
import numpy as np
import pytest
import torch

import oracle
import paper_1209_2137_amd as wp
from paper_1209_2137_amd import datagen

pytestmark = pytest.mark.gpu

CANARY = 0x5A5A5A5A
PAD = 64
ENC = {wp.CODEC_BP: oracle.bp_encode, wp.CODEC_FP: oracle.fp_encode, wp.CODEC_BP32: oracle.bp32_encode,
       wp.CODEC_FP32: oracle.fp32_encode, wp.CODEC_BPV: oracle.bpv_encode}
NAMES = {wp.CODEC_BP: "bp", wp.CODEC_FP: "fp", wp.CODEC_BP32: "bp32", wp.CODEC_FP32: "fp32", wp.CODEC_BPV: "bpv"}
UNIT = {wp.CODEC_BP: 2048, wp.CODEC_FP: 65536, wp.CODEC_BP32: 2048, wp.CODEC_FP32: 65536, wp.CODEC_BPV: 2048}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    wp.lib()


def dev(x):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    if x.size == 0:
        return torch.zeros(4, dtype=torch.int32, device="cuda")[:0]
    return torch.from_numpy(x.view(np.int32)).to("cuda")


def want_range(x, lo, hi):
    # the definition: values v with lo <= v <= hi of a non-decreasing list
    return int(np.searchsorted(x, lo, side="left")), int(np.searchsorted(x, hi, side="right"))


def gpu_range(comp_dev, n, codec, lo, hi):
    buf = torch.full((n + 2 * PAD,), CANARY, dtype=torch.int32, device="cuda")
    out, rng = wp.decode_range(comp_dev, n, codec, lo, hi, out=buf[PAD:PAD + n])
    rc = wp.check_code()
    h = buf.cpu().numpy().view(np.uint32)
    assert (h[:PAD] == CANARY).all() and (h[PAD + n:] == CANARY).all(), "write outside [out, out + n)"
    r = rng.cpu().numpy()
    return rc, (int(r[0]), int(r[1])), h[PAD:PAD + n]


def key_ranges(x, rng):
    """Key ranges over a non-decreasing list: empty, single values, a unit's
    stored base, before the first and after the last value, everything,
    and random spans of a few values to a few units."""
    n = x.size
    top = 0xFFFFFFFF
    ks = [(0, top), (0, 0), (top, top)]
    if n == 0:
        return ks
    first, last = int(x[0]), int(x[-1])
    ks += [(first, first), (last, last), (0, first), (last, top)]
    if first > 0:
        ks.append((0, first - 1))
    if last < top:
        ks.append((last + 1, top))
    for i in rng.integers(0, n, size=6):
        v = int(x[i])
        ks.append((v, v))
        if v > 0 and (i == 0 or int(x[i - 1]) < v - 1):
            ks.append((v - 1, v - 1))  # empty: between two values
        j = min(n - 1, int(i) + int(rng.integers(1, 5000)))
        ks.append((v, int(x[j])))
    for e in range(2048, n, 2048 * 7):  # values at unit edges (stored bases)
        ks.append((int(x[e - 1]), int(x[e - 1])))
        ks.append((int(x[e - 1]), int(x[e])))
        ks.append((int(x[e]), int(x[min(n - 1, e + 300)])))
    return ks


def check_list(x, codec, stride, rng, untouched_check=True):
    s = ENC[codec](x, stride)
    comp = dev(s)
    n = x.size
    for lo, hi in key_ranges(x, rng):
        print(f"range {NAMES[codec]} stride={stride} n={n} keys=[{lo}, {hi}]", flush=True)
        rc, r, got = gpu_range(comp, n, codec, lo, hi)
        assert rc == wp.OK
        w = want_range(x, lo, hi)
        assert r == w, (lo, hi)
        assert np.array_equal(got[w[0]:w[1]], x[w[0]:w[1]]), (lo, hi)
        if untouched_check and stride != 0 and n >= 40 * UNIT[codec] and w[1] - w[0] < 1000:
            # a narrow range decodes a few units only
            assert (got == CANARY).sum() > n // 2, (lo, hi)


@pytest.mark.parametrize("codec", sorted(NAMES))
@pytest.mark.parametrize("stride", [1, 4, 0])
def test_range_strictly_increasing(codec, stride):
    rng = np.random.default_rng(700 + 10 * codec + stride)
    for n in (0, 1, 127, 129, 2048 * 3 + 77, 65536 + 2048 * 2 + 300, 40 * 65536 + 1000):
        if n > 200_000 and codec not in (wp.CODEC_BP, wp.CODEC_FP):
            continue
        x = datagen.cluster_sorted(n, max_depth=14, seed=n + codec) if n else np.zeros(0, np.uint32)
        assert n == 0 or (np.diff(x.astype(np.int64)) > 0).all()
        check_list(x, codec, stride, rng)


@pytest.mark.parametrize("codec", sorted(NAMES))
@pytest.mark.parametrize("stride", [1, 4])
def test_range_runs_of_equal_values(codec, stride):
    # long runs of one value cross unit boundaries: a key range on such a
    # value starts in one unit and ends several units later
    rng = np.random.default_rng(800 + 10 * codec + stride)
    n = 6 * 65536 + 2048 * 5 + 91
    x = np.sort(rng.integers(0, 300, size=n, dtype=np.uint64)).astype(np.uint32)
    check_list(x, codec, stride, rng, untouched_check=False)
    y = np.repeat(np.arange(0, 4 * n, 40, dtype=np.uint32)[: n // 5000 + 1], 5000)[:n]
    check_list(y, codec, stride, rng, untouched_check=False)


def test_range_full_size_cluster_list():
    # the 2^26 recursive-cluster list, every codec's stream of it
    x = datagen.cluster_sorted()
    n = x.size
    rng = np.random.default_rng(901)
    xd = dev(x)
    for codec in sorted(NAMES):
        comp = wp.encode_trimmed(xd, codec, 1)
        for _ in range(4):
            i = int(rng.integers(0, n))
            j = min(n - 1, i + int(rng.integers(0, 1 << int(rng.integers(0, 22)))))
            lo, hi = int(x[i]), int(x[j])
            print(f"range full {NAMES[codec]} keys=[{lo}, {hi}]", flush=True)
            out = torch.empty(n, dtype=torch.int32, device="cuda")
            out, r = wp.decode_range(comp, n, codec, lo, hi, out=out)
            assert wp.check_code() == wp.OK
            i0, i1 = (int(v) for v in r.cpu().numpy())
            assert (i0, i1) == want_range(x, lo, hi)
            assert torch.equal(out[i0:i1], xd[i0:i1])


def test_range_errors():
    x = np.arange(0, 3 * 65536 + 500, 3, dtype=np.uint32)
    n = x.size
    s = oracle.bp_encode(x, 1)
    comp = dev(s)
    with pytest.raises(wp.WavepackError):
        wp.decode_range(comp, n, wp.CODEC_BP, 10, 9)
    with pytest.raises(wp.WavepackError):
        wp.decode_range(comp, n, 9, 0, 10)
    for what, at, val in (("magic", 0, int(s[0]) ^ 1), ("total", 7, int(s[7]) + 100)):
        bad = s.copy()
        bad[at] = val
        print("range corruption", what, flush=True)
        rc, r, _ = gpu_range(dev(bad), n, wp.CODEC_BP, 100, 200)
        assert rc == wp.ERR_CORRUPT and r == (0, 0), what
    rc, r, _ = gpu_range(comp, n - 1, wp.CODEC_BP, 100, 200)
    assert rc == wp.ERR_CORRUPT
    rc, r, got = gpu_range(comp, n, wp.CODEC_BP, 100, 200)
    assert rc == wp.OK and r == want_range(x, 100, 200)
