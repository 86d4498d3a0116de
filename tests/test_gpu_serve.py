"""Continuous-batching server on the GPU: every request's output, decoded in
the mix with whatever else was in flight, straight into the caller's buffer,
equals the generator's arrays (every request checked; tolerance 0: integer
decoding), and the same requests decoded alone equal them too. Admission
respects the output budget."""
import numpy as np
import pytest
import torch

import paper_1209_2137_amd as wp
from paper_1209_2137_amd import datagen
from paper_1209_2137_amd.pool import ListPool
from paper_1209_2137_amd.serve import CheckingCaller, Server, summarize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    assert torch.cuda.is_available()
    lens, codec, means, list_array = datagen.posting_lists(n_lists=300, total=3e6, seed=25, lmax=1 << 17)
    return ListPool(list_array, codec, stride=1, count=300)


def decode_alone(pool, ids):
    """The request decoded by itself: one single-list decode per list."""
    n = sum((int(pool.lens[i]) + 3) & ~3 for i in ids)
    out = torch.zeros(max(n, 4), dtype=torch.int32, device="cuda")
    o = 0
    for i in ids:
        co, cw, _, n_i, codec = pool.rows[i]
        fn = wp.lib().bp_decode if codec == wp.CODEC_BP else wp.lib().fastpfor_decode
        assert fn(pool.pool.data_ptr() + 4 * co, cw, out.data_ptr() + 4 * o, n_i, wp._stream(None)) == wp.OK
        o += (n_i + 3) & ~3
    return out


@pytest.mark.parametrize("budget_elems,streams", [(1 << 22, 4), (1 << 20, 2)])
def test_mix_equals_alone_and_inputs(pool, budget_elems, streams):
    times, reqs = datagen.poisson_arrivals(rate=2000.0, duration=0.5, pool=300, seed=7)
    print(f"serve budget={budget_elems} streams={streams} requests={len(times)}", flush=True)
    srv = Server(pool, budget_bytes=4 * budget_elems, streams=streams)
    caller = CheckingCaller(pool, budget_elems)
    done = srv.run(times, reqs, caller.get, caller.done)
    stats = summarize(done, srv.wall)
    srv.close()
    bad = caller.finish()
    assert wp.check_code() == wp.OK
    assert len(done) == len(times) and caller.checked == len(done)
    assert bad == 0, f"{bad} wrong elements"
    assert srv.peak_bytes <= 4 * budget_elems
    assert stats["p99_ms"] is not None and stats["p50_ms"] <= stats["p99_ms"]
    # the same requests decoded alone, bit for bit
    for r in done[:: max(1, len(done) // 40)]:
        alone = decode_alone(pool, r.lists)
        for li, o in zip(r.lists, r.offsets):
            n = int(pool.lens[li])
            _, _, oo, _, _ = pool.rows[li]
            assert torch.equal(alone[o:o + n], pool.values[oo:oo + n])


def test_requests_larger_than_half_the_budget_still_complete(pool):
    # a budget that holds about one request at a time: admission queues the rest
    times = np.zeros(20)  # all at once
    rng = np.random.default_rng(3)
    reqs = [rng.integers(0, 300, size=int(rng.integers(1, 33))) for _ in times]
    need = max(sum((int(pool.lens[i]) + 3) & ~3 for i in r) for r in reqs)
    budget = max(need, 4096)
    srv = Server(pool, budget_bytes=4 * budget, streams=2)
    caller = CheckingCaller(pool, 2 * budget)
    done = srv.run(times, reqs, caller.get, caller.done)
    srv.close()
    assert caller.finish() == 0
    assert len(done) == 20 and wp.check_code() == wp.OK
    assert srv.peak_bytes <= 4 * budget and srv.waited_for_budget > 0
