"""Batched decoding on the GPU: every list decoded in one launch
must equal its generator array (which the single-list path and the CPU
oracle decode to as well), for graph and plain launches and for every
workgroup shape. Integer work: exact comparison."""
import numpy as np
import pytest
import torch

import oracle
import paper_1209_2137_amd as wp
from paper_1209_2137_amd import datagen
from paper_1209_2137_amd.pool import ListPool

pytestmark = pytest.mark.gpu

TUNES = [
    dict(waves=4, vpl=4, depth=2, run_units=8, wg_per_cu=4, use_graph=1),
    dict(waves=4, vpl=4, depth=2, run_units=8, wg_per_cu=4, use_graph=0),
    dict(waves=2, vpl=4, depth=3, run_units=1, wg_per_cu=8, use_graph=1),
    dict(waves=2, vpl=4, depth=4, run_units=63, wg_per_cu=16, use_graph=1),
    dict(waves=8, vpl=4, depth=2, run_units=5, wg_per_cu=2, use_graph=0),
    dict(waves=8, vpl=4, depth=3, run_units=16, wg_per_cu=0, use_graph=1),
]


@pytest.fixture(scope="module")
def pool():
    assert torch.cuda.is_available()
    # posting-list shapes: Zipf lengths (scaled to 400 lists), 50/50 codecs,
    # geometric gaps of log-uniform mean
    lens, codec, means, list_array = datagen.posting_lists(n_lists=400, total=4e6, seed=15, lmax=1 << 18)
    return ListPool(list_array, codec, stride=1, count=400)


def test_pool_streams_match_oracle_encoder(pool):
    # the pool's GPU-encoded streams are the oracle's streams, word for word
    p = pool.pool.cpu().numpy().view(np.uint32)
    v = pool.values.cpu().numpy().view(np.uint32)
    for i in range(0, 400, 37):
        co, cw, oo, n, codec = pool.rows[i]
        x = v[oo:oo + n]
        want = (oracle.bp_encode if codec == wp.CODEC_BP else oracle.fp_encode)(x, 1)
        assert np.array_equal(p[co:co + cw], want), i


def test_pool_streams_round_trip(pool):
    # the packed streams make a pool again whose batched decode equals the inputs
    packed, rows = pool.streams()
    again = ListPool.from_streams(packed, rows)
    assert again.total_n == pool.total_n and again.comp_bytes == pool.comp_bytes
    assert again.total_out == pool.total_out
    out = torch.full((pool.total_out + 64,), -1, dtype=torch.int32, device="cuda")
    plan = again.plan(out)
    plan.decode()
    assert wp.check_code() == wp.OK
    for i, (co, cw, oo, n, codec) in enumerate(pool.rows):
        assert again.rows[i][1:] == (cw, oo, n, codec)
        if not torch.equal(out[oo:oo + n], pool.values[oo:oo + n]):
            raise AssertionError(f"list {i} (codec {codec}, n {n}) differs")
    plan.free()


@pytest.mark.parametrize("tune", TUNES, ids=lambda t: "w{waves}v{vpl}d{depth}r{run_units}c{wg_per_cu}g{use_graph}".format(**t))
def test_batch_decode_matches_inputs(pool, tune):
    out = torch.full((pool.total_out + 64,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    plan = pool.plan(out, tune=tune)
    assert plan.items > 0
    for rep in range(3):  # graph replays with eager work in between
        out[: pool.total_out].fill_(-1)
        plan.decode()
        assert wp.check_code() == wp.OK
        for i in range(len(pool.rows)):
            co, cw, oo, n, codec = pool.rows[i]
            if not torch.equal(out[oo:oo + n], pool.values[oo:oo + n]):
                raise AssertionError(f"list {i} (codec {codec}, n {n}) differs on replay {rep}")
        assert (out[pool.total_out:] == 0x5A5A5A5A).all()
    plan.free()


def test_batch_equals_single_list_decodes(pool):
    a = torch.zeros(pool.total_out + 4, dtype=torch.int32, device="cuda")
    b = torch.zeros_like(a)
    plan = pool.plan(a)
    plan.decode()
    for i in range(len(pool.rows)):
        pool.decode_one(i, b)
    assert wp.check_code() == wp.OK
    assert torch.equal(a, b)
    plan.free()


def test_batch_flags_a_corrupt_list_and_decodes_the_rest(pool):
    rows = list(pool.rows)
    bad = 3
    co, cw, oo, n, codec = rows[bad]
    saved = pool.pool[co].clone()
    pool.pool[co] = 0x12345678  # bad magic
    out = torch.zeros(pool.total_out + 4, dtype=torch.int32, device="cuda")
    plan = pool.plan(out)
    plan.decode()
    rc = wp.check_code()
    pool.pool[co] = saved
    assert rc == wp.ERR_CORRUPT
    for i in range(len(rows)):
        if i == bad:
            continue
        _, _, oo2, n2, _ = rows[i]
        assert torch.equal(out[oo2:oo2 + n2], pool.values[oo2:oo2 + n2]), i
    plan.free()


def test_batch_plan_rejects_bad_registry(pool):
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(wp.WavepackError):
        wp.BatchPlan(pool.pool, out, [(1, 100, 0, 10, 0)])  # misaligned stream offset
    with pytest.raises(wp.WavepackError):
        wp.BatchPlan(pool.pool, out, [(0, 100, 0, 10, 7)])  # unknown codec
    with pytest.raises(wp.WavepackError):
        wp.BatchPlan(pool.pool, out, pool.rows[:2], tune=dict(waves=3))


@pytest.mark.parametrize("stride", [0, 4])
def test_batch_strides_and_page_sizes(stride):
    # lists of every item shape at strides 0 and 4: patched lists of one
    # small page (<= 64 blocks, one wavefront), of one large page (a
    # workgroup), of several pages, binary-packing lists, and lists shorter
    # than one block (a tail item only); each decoded list equals its input
    rng = np.random.default_rng(40 + stride)
    lens = [5, 127, 128, 129, 64 * 128, 64 * 128 + 77, 65 * 128 + 3, 300 * 128 + 50, 512 * 128, 512 * 128 + 9000,
            3 * 512 * 128 + 4000, 2048 * 3 + 17, 33 * 2048 + 1]
    arrays, codecs = [], []
    for i, n in enumerate(lens):
        for codec in (wp.CODEC_BP, wp.CODEC_FP):
            arrays.append(datagen.patched_gaps(n, seed=1000 * stride + 10 * i + codec) if i % 2 else
                          datagen.single_geometric(n, mean=float(rng.integers(2, 3000)), seed=i + 7 * codec))
            codecs.append(codec)
    pool = ListPool(arrays, codecs, stride=stride)
    for tune in (dict(waves=4, vpl=4, depth=2, run_units=4, wg_per_cu=2, use_graph=1),
                 dict(waves=2, vpl=4, depth=3, run_units=16, wg_per_cu=0, use_graph=0)):
        out = torch.full((pool.total_out + 64,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        plan = pool.plan(out, tune=tune)
        for rep in range(2):
            out[: pool.total_out].fill_(-1)
            plan.decode()
            assert wp.check_code() == wp.OK
            for i in range(len(pool.rows)):
                co, cw, oo, n, codec = pool.rows[i]
                if not torch.equal(out[oo:oo + n], pool.values[oo:oo + n]):
                    raise AssertionError(f"list {i} (codec {codec}, n {n}, stride {stride}) differs on replay {rep}")
            assert (out[pool.total_out:] == 0x5A5A5A5A).all()
        plan.free()


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_batch_partial_pages(waves):
    # patched lists of one partial page of 65..511 blocks (decoded by whole
    # workgroups in the batch) plus a Variable Byte tail: every list exact
    rng = np.random.default_rng(40 + waves)
    lists = []
    for i in range(200):
        nb = int(rng.integers(65, 512))
        lists.append(datagen.single_geometric(nb * 128 + int(rng.integers(0, 128)),
                                              mean=float(rng.integers(2, 4000)), seed=500 + i))
    pool = ListPool(lists, [wp.CODEC_FP] * len(lists), stride=1)
    out = torch.zeros(pool.total_out + 4, dtype=torch.int32, device="cuda")
    plan = pool.plan(out, tune=dict(waves=waves, vpl=4, depth=2, run_units=4, use_graph=1))
    plan.decode()
    assert wp.check_code() == wp.OK
    bad = [i for i, (co, cw, oo, n, c) in enumerate(pool.rows) if not torch.equal(out[oo:oo + n], pool.values[oo:oo + n])]
    plan.free()
    assert not bad, f"{len(bad)} lists differ, first {bad[:5]}"
