"""delta_decode_inplace_noalloc (no allocation: status words in the
library's fixed per-device array) against delta_decode_inplace on the same
seeded inputs, bit for bit, through the C ABI: two calls in a row, the
second on a smaller input (the array keeps the first call's words, which
the second must clear), for both strides; the size limit is checked on the
host. Both are also compared with the oracle's in-place prefix sum."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1209_2137_amd as wp

pytestmark = pytest.mark.gpu

MAX_N = 1 << 28


def _run(fn, x, init, stride, stream):
    t = torch.from_numpy(x.view(np.int32)).to("cuda")
    rc = fn(ctypes.c_void_p(t.data_ptr()), x.size, init, stride, ctypes.c_void_p(stream))
    assert rc == wp.OK, wp.strerror(rc)
    assert wp.lib().wp_check(ctypes.c_void_p(stream)) == wp.OK
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("stride", [1, 4])
def test_noalloc_equals_allocating_entry_point_twice(stride):
    L = wp.lib()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(71 + stride)
    # first call large (many tiles and a ragged last tile), the second smaller
    for n, init in ((3_000_017, 0xFFFFFF00), (40_001, 7)):
        print(f"stride {stride} n {n}", flush=True)
        x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        got = _run(L.delta_decode_inplace_noalloc, x, init, stride, stream)
        want = _run(L.delta_decode_inplace, x, init, stride, stream)
        assert np.array_equal(got, want), f"n {n}: differs from delta_decode_inplace"
        ref = x.copy()
        oracle.delta_decode_inplace(ref, init, stride)
        assert np.array_equal(got, ref), f"n {n}: differs from the oracle"


def test_noalloc_at_its_size_limit():
    L = wp.lib()
    stream = torch.cuda.current_stream().cuda_stream
    n = MAX_N
    print(f"stride 1 n {n}", flush=True)
    t = torch.ones(n, dtype=torch.int32, device="cuda")
    rc = L.delta_decode_inplace_noalloc(ctypes.c_void_p(t.data_ptr()), n, 5, 1, ctypes.c_void_p(stream))
    assert rc == wp.OK
    assert L.wp_check(ctypes.c_void_p(stream)) == wp.OK
    want = torch.arange(6, 6 + n, dtype=torch.int64, device="cuda").to(torch.int32)
    assert torch.equal(t, want)
    del t, want
    torch.cuda.empty_cache()


def test_noalloc_rejects_sizes_beyond_its_array():
    L = wp.lib()
    # host-side checks: nothing is enqueued
    assert L.delta_decode_inplace_noalloc(ctypes.c_void_p(16), MAX_N + 1, 0, 1, None) == wp.ERR_CAPACITY
    assert L.delta_decode_inplace_noalloc(ctypes.c_void_p(16), 10, 0, 2, None) == wp.ERR_INVALID_ARG
    assert L.delta_decode_inplace_noalloc(None, 0, 0, 1, None) == wp.OK
