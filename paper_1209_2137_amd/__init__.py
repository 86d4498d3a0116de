"""wavepack: MI355X (gfx950) decoding of binary-packed and patched uint32
streams (Lemire & Boytsov, arXiv:1209.2137), behind a C ABI.

This module is argument marshalling only: every decode/encode step runs in
the HIP kernels of ``libwavepack.so``. PyTorch provides device memory and
streams. Tensors holding uint32 data may be ``torch.int32`` or
``torch.uint32`` (same bits); outputs are allocated as ``torch.int32``.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwavepack.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_CAPACITY = -2
ERR_CORRUPT = -3
ERR_HIP = -4
CODEC_BP = 0
CODEC_FP = 1
CODEC_BP32 = 2
CODEC_FP32 = 3
CODEC_BPV = 4
CODEC_SP = 5
CODEC_FPI = 6

EXPORTS = (
    "bp_encode", "bp_decode", "bp32_encode", "bp32_decode", "fastpfor_encode", "fastpfor_decode",
    "fastpfor32_encode", "fastpfor32_decode", "bp_vertical_encode", "bp_vertical_decode", "delta_decode_inplace",
    "wp_max_compressed_words", "wp_check", "wp_strerror", "wp_set_decode_tune", "wp_time_next_launch",
    "wp_batch_plan", "wp_batch_replan", "wp_batch_decode", "wp_batch_items", "wp_batch_free",
    "wp_intersect", "wp_intersect_compressed", "wp_decode_range",
    "simplepfor_decode", "simplepfor_encode", "delta_decode_inplace_noalloc", "fastpfor_inline_encode",
    "fastpfor_inline_decode",
)

_lib = None


class WavepackError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


class wp_list(ctypes.Structure):
    _fields_ = [("comp_off_words", ctypes.c_uint64), ("comp_words", ctypes.c_uint64),
                ("out_off", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("codec", ctypes.c_int32), ("reserved", ctypes.c_int32), ("out", ctypes.c_void_p)]


class wp_tune(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("vpl", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("run_units", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


def lib():
    """The loaded C library. Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(wavepack has no CPU fallback)")
    # let torch bring the HIP runtime up first (as every caller that hands
    # the library torch tensors has done): the library's own code objects
    # then load into the runtime torch uses
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32
    for name in ("bp_encode", "bp32_encode", "fastpfor_encode", "fastpfor32_encode", "bp_vertical_encode",
                 "simplepfor_encode", "fastpfor_inline_encode"):
        f = getattr(L, name)
        f.argtypes = [vp, u64, i32, vp, u64, vp, vp]
        f.restype = i32
    for name in ("bp_decode", "bp32_decode", "fastpfor_decode", "fastpfor32_decode", "bp_vertical_decode",
                 "simplepfor_decode", "fastpfor_inline_decode"):
        f = getattr(L, name)
        f.argtypes = [vp, u64, vp, u64, vp]
        f.restype = i32
    L.delta_decode_inplace.argtypes = [vp, u64, u32, i32, vp]
    L.delta_decode_inplace.restype = i32
    L.delta_decode_inplace_noalloc.argtypes = [vp, u64, u32, i32, vp]
    L.delta_decode_inplace_noalloc.restype = i32
    L.wp_max_compressed_words.argtypes = [i32, u64]
    L.wp_max_compressed_words.restype = u64
    L.wp_check.argtypes = [vp]
    L.wp_check.restype = i32
    L.wp_strerror.argtypes = [i32]
    L.wp_strerror.restype = ctypes.c_char_p
    L.wp_set_decode_tune.argtypes = [i32, i32, i32, i32, i32]
    L.wp_set_decode_tune.restype = i32
    L.wp_time_next_launch.argtypes = [vp, vp]
    L.wp_time_next_launch.restype = i32
    L.wp_batch_plan.argtypes = [vp, vp, ctypes.POINTER(wp_list), u64, ctypes.POINTER(wp_tune),
                                ctypes.POINTER(vp), vp]
    L.wp_batch_plan.restype = i32
    L.wp_batch_replan.argtypes = [vp, vp, vp, ctypes.POINTER(wp_list), u64, vp]
    L.wp_batch_replan.restype = i32
    L.wp_batch_decode.argtypes = [vp, vp]
    L.wp_batch_decode.restype = i32
    L.wp_batch_items.argtypes = [vp]
    L.wp_batch_items.restype = u64
    L.wp_batch_free.argtypes = [vp]
    L.wp_batch_free.restype = i32
    L.wp_intersect.argtypes = [vp, u64, vp, u64, vp, vp, vp]
    L.wp_intersect.restype = i32
    L.wp_intersect_compressed.argtypes = [vp, u64, vp, u64, u64, i32, vp, vp, vp, vp]
    L.wp_intersect_compressed.restype = i32
    L.wp_decode_range.argtypes = [vp, u64, u64, i32, u32, u32, vp, vp, vp]
    L.wp_decode_range.restype = i32
    _lib = L
    # workgroup shapes chosen by the autotuner for this architecture, if any
    try:
        from .autotune import apply
        apply()
    except Exception:  # a missing or stale table leaves the built-in shapes
        pass
    return L


def strerror(code: int) -> str:
    try:
        return lib().wp_strerror(code).decode()
    except RuntimeError:
        return f"code {code}"


def _check(rc: int, what: str):
    if rc != OK:
        raise WavepackError(rc, what)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _ptr_or_null(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


def _need_u32(t, what):
    import torch
    if t.dtype not in (torch.int32, torch.uint32) or not t.is_contiguous() or not t.is_cuda:
        raise TypeError(f"{what} must be a contiguous int32/uint32 CUDA tensor")


def max_compressed_words(codec: int, n: int) -> int:
    return int(lib().wp_max_compressed_words(codec, n))


def set_decode_tune(codec: int, waves: int, vpl: int, wg_per_cu: int = 0, depth: int = 0):
    """Workgroup shape of the single-list decoders: `waves` wavefronts per
    workgroup, `vpl` integers per lane and pass; for binary packing about
    `wg_per_cu` runs of meta-blocks per compute unit and `depth` loads in
    flight per thread (0 = defaults)."""
    _check(lib().wp_set_decode_tune(codec, waves, vpl, depth, wg_per_cu), "set_decode_tune")


def time_next_launch(start, stop):
    """The calling thread's next bp_decode / fastpfor_decode /
    delta_decode_inplace records the torch.cuda.Event `start` when its main
    kernel starts and `stop` when it ends (both must already exist on the
    device: record them once before first use)."""
    _check(lib().wp_time_next_launch(ctypes.c_void_p(start.cuda_event), ctypes.c_void_p(stop.cuda_event)),
           "time_next_launch")


def _decode(fn, comp, n, out, stream, name):
    import torch
    _need_u32(comp, "comp")
    if out is None:
        out = torch.empty(max(int(n), 0), dtype=torch.int32, device=comp.device)
    _need_u32(out, "out")
    if out.numel() < n:
        raise ValueError("out is smaller than n")
    _check(fn(_ptr(comp), comp.numel(), _ptr(out), int(n), _stream(stream)), name)
    return out


def bp_decode(comp, n: int, out=None, stream=None):
    """Decodes a binary-packing stream (device tensor) into out[0:n]."""
    return _decode(lib().bp_decode, comp, n, out, stream, "bp_decode")


def bp32_decode(comp, n: int, out=None, stream=None):
    """Decodes a BP32 stream (32-integer blocks) into out[0:n]."""
    return _decode(lib().bp32_decode, comp, n, out, stream, "bp32_decode")


def fastpfor_decode(comp, n: int, out=None, stream=None):
    """Decodes a patched (FastPFOR page) stream (device tensor) into out[0:n]."""
    return _decode(lib().fastpfor_decode, comp, n, out, stream, "fastpfor_decode")


def bp_vertical_decode(comp, n: int, out=None, stream=None):
    """Decodes a SIMD-BP128 stream in the four-lane block layout into out[0:n]."""
    return _decode(lib().bp_vertical_decode, comp, n, out, stream, "bp_vertical_decode")


def fastpfor32_decode(comp, n: int, out=None, stream=None):
    """Decodes a FastPFOR stream (exception arrays padded to 32) into out[0:n]."""
    return _decode(lib().fastpfor32_decode, comp, n, out, stream, "fastpfor32_decode")


def simplepfor_decode(comp, n: int, out=None, stream=None):
    """Decodes a SimplePFOR stream (exception high parts in Simple-8b) into out[0:n]."""
    return _decode(lib().simplepfor_decode, comp, n, out, stream, "simplepfor_decode")


def _encode(fn, codec, x, stride, out, out_words, stream, name):
    import torch
    _need_u32(x, "x")
    n = x.numel()
    cap = max_compressed_words(codec, n)
    if cap == 0:
        raise ValueError("n beyond the stream format")
    if out is None:
        out = torch.empty(cap, dtype=torch.int32, device=x.device)
    _need_u32(out, "out")
    if out_words is None:
        out_words = torch.zeros(1, dtype=torch.int64, device=x.device)
    _check(fn(_ptr(x), n, int(stride), _ptr(out), out.numel(), _ptr(out_words), _stream(stream)), name)
    return out, out_words


def bp_encode(x, stride: int = 1, out=None, out_words=None, stream=None):
    """Encodes x (device uint32) as a binary-packing stream. Returns
    (buffer, words) where words is a one-element device int64 tensor."""
    return _encode(lib().bp_encode, CODEC_BP, x, stride, out, out_words, stream, "bp_encode")


def bp32_encode(x, stride: int = 1, out=None, out_words=None, stream=None):
    """Encodes x (device uint32) as a BP32 stream."""
    return _encode(lib().bp32_encode, CODEC_BP32, x, stride, out, out_words, stream, "bp32_encode")


def fastpfor_encode(x, stride: int = 1, out=None, out_words=None, stream=None):
    """Encodes x (device uint32) as a patched-page stream."""
    return _encode(lib().fastpfor_encode, CODEC_FP, x, stride, out, out_words, stream, "fastpfor_encode")


def fastpfor32_encode(x, stride: int = 1, out=None, out_words=None, stream=None):
    """Encodes x (device uint32) as FastPFOR pages (exception arrays padded to 32)."""
    return _encode(lib().fastpfor32_encode, CODEC_FP32, x, stride, out, out_words, stream, "fastpfor32_encode")


def bp_vertical_encode(x, stride: int = 1, out=None, out_words=None, stream=None):
    """Encodes x (device uint32) as SIMD-BP128 with the four-lane block layout."""
    return _encode(lib().bp_vertical_encode, CODEC_BPV, x, stride, out, out_words, stream, "bp_vertical_encode")


def fastpfor_inline_encode(x, stride: int = 1, out=None, out_words=None, stream=None):
    """Encodes x (device uint32) as FastPFOR pages in the paper's own layout."""
    return _encode(lib().fastpfor_inline_encode, CODEC_FPI, x, stride, out, out_words, stream,
                   "fastpfor_inline_encode")


def fastpfor_inline_decode(comp, n: int, out=None, stream=None):
    """Decodes a stream of FastPFOR pages in the paper's own layout into out[0:n]."""
    return _decode(lib().fastpfor_inline_decode, comp, n, out, stream, "fastpfor_inline_decode")


def simplepfor_encode(x, stride: int = 1, out=None, out_words=None, stream=None):
    """Encodes x (device uint32) as SimplePFOR pages (exception high parts in Simple-8b)."""
    return _encode(lib().simplepfor_encode, CODEC_SP, x, stride, out, out_words, stream, "simplepfor_encode")


def encode_trimmed(x, codec: int = CODEC_BP, stride: int = 1, stream=None):
    """Encodes and returns a tensor of exactly the stream's length
    (synchronises the stream to read the length)."""
    enc = {CODEC_BP: bp_encode, CODEC_FP: fastpfor_encode, CODEC_BP32: bp32_encode, CODEC_FP32: fastpfor32_encode,
           CODEC_BPV: bp_vertical_encode, CODEC_SP: simplepfor_encode, CODEC_FPI: fastpfor_inline_encode}[codec]
    buf, words = enc(x, stride, stream=stream)
    check(stream)
    return buf[: int(words.item())].clone()


def intersect(a, b, out=None, count=None, stream=None):
    """Values present in both strictly increasing device arrays a and b,
    ascending, written to out[0:count] (out holds a.numel() values; count is
    a one-element device int64 tensor). Returns (out, count); asynchronous."""
    import torch
    _need_u32(a, "a")
    _need_u32(b, "b")
    if out is None:
        out = torch.empty(max(a.numel(), 1), dtype=torch.int32, device=a.device)
    _need_u32(out, "out")
    if out.numel() < a.numel():
        raise ValueError("out is smaller than a")
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device=a.device)
    _check(lib().wp_intersect(_ptr(a), a.numel(), _ptr(b), b.numel(), _ptr(out), _ptr(count), _stream(stream)),
           "wp_intersect")
    return out, count


def intersect_compressed(a, b_comp, nb: int, codec: int, work=None, out=None, count=None, stream=None):
    """intersect() with the second list given as a compressed stream of nb
    integers: only the units that a's values fall in are decoded (into
    `work`, nb integers). Returns (out, count, work); asynchronous."""
    import torch
    _need_u32(a, "a")
    _need_u32(b_comp, "b_comp")
    if work is None:
        work = torch.empty(max(nb, 4), dtype=torch.int32, device=a.device)
    _need_u32(work, "work")
    if work.numel() < nb:
        raise ValueError("work is smaller than nb")
    if out is None:
        out = torch.empty(max(a.numel(), 1), dtype=torch.int32, device=a.device)
    _need_u32(out, "out")
    if out.numel() < a.numel():
        raise ValueError("out is smaller than a")
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device=a.device)
    _check(lib().wp_intersect_compressed(_ptr(a), a.numel(), _ptr(b_comp), b_comp.numel(), int(nb), int(codec),
                                         _ptr(work), _ptr(out), _ptr(count), _stream(stream)),
           "wp_intersect_compressed")
    return out, count, work


def decode_range(comp, n: int, codec: int, key_lo: int, key_hi: int, out=None, rng=None, stream=None):
    """Random access by key: decodes only the units of the compressed
    non-decreasing list (n integers) whose values can lie in
    [key_lo, key_hi], each at its place in `out` (n integers), and writes
    the index range [i0, i1) of those values to `rng` (two-element device
    int64 tensor). Returns (out, rng); asynchronous."""
    import torch
    _need_u32(comp, "comp")
    if out is None:
        out = torch.empty(max(n, 4), dtype=torch.int32, device=comp.device)
    _need_u32(out, "out")
    if out.numel() < n:
        raise ValueError("out is smaller than n")
    if rng is None:
        rng = torch.zeros(2, dtype=torch.int64, device=comp.device)
    _check(lib().wp_decode_range(_ptr(comp), comp.numel(), int(n), int(codec), int(key_lo) & 0xFFFFFFFF,
                                 int(key_hi) & 0xFFFFFFFF, _ptr(out), _ptr(rng), _stream(stream)),
           "wp_decode_range")
    return out, rng


def intersect_trimmed(a, b, stream=None):
    """intersect() returning exactly the common values (synchronises the
    stream to read the count)."""
    out, count = intersect(a, b, stream=stream)
    check(stream)
    return out[: int(count.item())].clone()


def delta_decode_inplace(data, init: int = 0, stride: int = 1, stream=None):
    """In-place prefix sum (differential decoding, Section 3) of a device tensor."""
    _need_u32(data, "data")
    _check(lib().delta_decode_inplace(_ptr(data), data.numel(), int(init) & 0xFFFFFFFF, int(stride),
                                      _stream(stream)), "delta_decode_inplace")
    return data


def check(stream=None):
    """Synchronises the stream and raises WavepackError if a kernel flagged
    a corrupt stream since the last check."""
    rc = lib().wp_check(_stream(stream))
    _check(rc, "device check")


def check_code(stream=None) -> int:
    return int(lib().wp_check(_stream(stream)))


def _registry(lists):
    """wp_list array of rows (comp_off_words, comp_words, out_off, n, codec)
    or (..., codec, out_ptr): a non-zero out_ptr is the list's own device
    destination (out_off is then ignored)."""
    n = len(lists)
    arr = (wp_list * max(n, 1))()
    for i, row in enumerate(lists):
        co, cw, oo, nn, codec = row[:5]
        dst = int(row[5]) if len(row) > 5 else 0
        arr[i] = wp_list(int(co), int(cw), int(oo), int(nn), int(codec), 0, dst or None)
    return arr, n


class BatchPlan:
    """A batched decode of many lists (see wp_batch_plan).

    pool: device tensor holding all compressed streams; out: device tensor
    receiving the outputs at the rows' offsets (None when every row names
    its own destination); lists: rows (comp_off_words, comp_words, out_off,
    n, codec[, out_ptr]). tune: dict with waves, vpl, depth, run_units,
    wg_per_cu, use_graph (missing keys take the library defaults)."""

    def __init__(self, pool, out, lists, tune=None, stream=None):
        _need_u32(pool, "pool")
        if out is not None:
            _need_u32(out, "out")
        arr, n = _registry(lists)
        t = None
        if tune is not None:
            t = wp_tune(int(tune.get("waves", 0)), int(tune.get("vpl", 0)), int(tune.get("depth", 0)),
                        int(tune.get("run_units", 0)), int(tune.get("wg_per_cu", 0)),
                        int(tune.get("use_graph", 1)))
        self._h = ctypes.c_void_p()
        self.pool, self.out = pool, out  # keep the buffers alive
        _check(lib().wp_batch_plan(_ptr(pool), _ptr_or_null(out), arr, n,
                                   ctypes.byref(t) if t is not None else None, ctypes.byref(self._h),
                                   _stream(stream)), "wp_batch_plan")

    def replan(self, pool, out, lists, stream=None):
        """Points the plan at a new registry without allocating (async copy)."""
        _need_u32(pool, "pool")
        if out is not None:
            _need_u32(out, "out")
        arr, n = _registry(lists)
        self.pool, self.out = pool, out
        _check(lib().wp_batch_replan(self._h, _ptr(pool), _ptr_or_null(out), arr, n, _stream(stream)),
               "wp_batch_replan")

    @property
    def items(self) -> int:
        return int(lib().wp_batch_items(self._h))

    def decode(self, stream=None):
        _check(lib().wp_batch_decode(self._h, _stream(stream)), "wp_batch_decode")

    def free(self):
        if self._h:
            rc = lib().wp_batch_free(self._h)
            self._h = ctypes.c_void_p()
            _check(rc, "wp_batch_free")

    def __del__(self):
        try:
            if self._h:
                lib().wp_batch_free(self._h)
        except Exception:
            pass
