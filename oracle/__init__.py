"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``wp_oracle.c``: a plain scalar encoder/decoder written
from the paper (Lemire & Boytsov, arXiv:1209.2137). Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package;
the GPU library never does, and shares no code with it.

Functions take and return numpy ``uint32`` arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_ARG, ERR_CAP, ERR_CORRUPT = 0, -1, -2, -3
CODEC_BP, CODEC_FP, CODEC_BP32, CODEC_FP32, CODEC_BPV, CODEC_SP, CODEC_FPI = 0, 1, 2, 3, 4, 5, 6


def build() -> str:
    """Compile the oracle with gcc (plain C99, -O2, no vector intrinsics)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
                    _SRC, "-o", tmp], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64 = ctypes.c_uint64
    lib.oracle_bits.argtypes = [ctypes.c_uint32]
    lib.oracle_bits.restype = ctypes.c_uint32
    lib.oracle_pack.argtypes = [u32p, u64, ctypes.c_uint32, u32p]
    lib.oracle_unpack.argtypes = [u32p, u64, ctypes.c_uint32, u32p]
    lib.oracle_pack_vertical.argtypes = [u32p, u64, ctypes.c_uint32, u32p]
    lib.oracle_unpack_vertical.argtypes = [u32p, u64, ctypes.c_uint32, u32p]
    for f in (lib.oracle_delta_encode_inplace, lib.oracle_delta_decode_inplace):
        f.argtypes = [u32p, u64, ctypes.c_uint32, ctypes.c_int]
        f.restype = ctypes.c_int
    lib.oracle_vbyte_encode.argtypes = [u32p, ctypes.c_uint32, u8p]
    lib.oracle_vbyte_encode.restype = ctypes.c_uint32
    lib.oracle_vbyte_decode.argtypes = [u8p, u64, ctypes.c_uint32, u32p]
    lib.oracle_vbyte_decode.restype = ctypes.c_int64
    lib.oracle_fp_choose.argtypes = [u32p, ctypes.c_uint32, u32p, u32p, u32p]
    lib.oracle_intersect.argtypes = [u32p, u64, u32p, u64, u32p]
    lib.oracle_intersect.restype = u64
    lib.oracle_max_words.argtypes = [ctypes.c_int, u64]
    lib.oracle_max_words.restype = u64
    for f in (lib.oracle_bp_encode, lib.oracle_fp_encode, lib.oracle_bp32_encode, lib.oracle_fp32_encode,
              lib.oracle_bpv_encode, lib.oracle_sp_encode, lib.oracle_fpi_encode):
        f.argtypes = [u32p, u64, ctypes.c_int, u32p, u64]
        f.restype = ctypes.c_int64
    for f in (lib.oracle_bp_decode, lib.oracle_fp_decode, lib.oracle_bp32_decode, lib.oracle_fp32_decode,
              lib.oracle_bpv_decode, lib.oracle_sp_decode, lib.oracle_fpi_decode):
        f.argtypes = [u32p, u64, u32p, u64]
        f.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_s8_mode.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
    lib.oracle_s8_mode.restype = None
    lib.oracle_s8_encode.argtypes = [u32p, u64, u64p]
    lib.oracle_s8_encode.restype = u64
    lib.oracle_s8_decode.argtypes = [u64p, u64, u32p, u64]
    lib.oracle_s8_decode.restype = ctypes.c_int64
    _lib = lib
    return lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def bits(x: int) -> int:
    return int(_load().oracle_bits(int(x) & 0xFFFFFFFF))


def pack(vals, b: int) -> np.ndarray:
    v = _u32(vals)
    out = np.zeros((v.size * b + 31) // 32, dtype=np.uint32)
    _load().oracle_pack(_p32(v), v.size, b, _p32(out))
    return out


def unpack(words, count: int, b: int) -> np.ndarray:
    w = _u32(words)
    if w.size * 32 < count * b:
        raise ValueError("not enough words")
    out = np.zeros(count, dtype=np.uint32)
    _load().oracle_unpack(_p32(w if w.size else np.zeros(1, np.uint32)), count, b, _p32(out))
    return out


def pack_vertical(vals, b: int) -> np.ndarray:
    """Four interleaved 32-bit lanes, value i in lane i % 4 (Section 4's
    vectorized layout); len(vals) a multiple of 4."""
    v = _u32(vals)
    out = np.zeros(4 * ((v.size // 4 * b + 31) // 32) or 1, dtype=np.uint32)
    _load().oracle_pack_vertical(_p32(v), v.size, b, _p32(out))
    return out[:4 * ((v.size // 4 * b + 31) // 32)]


def unpack_vertical(words, count: int, b: int) -> np.ndarray:
    w = _u32(words)
    out = np.zeros(max(count, 1), dtype=np.uint32)
    _load().oracle_unpack_vertical(_p32(w if w.size else np.zeros(1, np.uint32)), count, b, _p32(out))
    return out[:count]


def delta_encode_inplace(data: np.ndarray, init: int = 0, stride: int = 1) -> int:
    assert data.dtype == np.uint32 and data.flags.c_contiguous
    return _load().oracle_delta_encode_inplace(_p32(data), data.size, init, stride)


def delta_decode_inplace(data: np.ndarray, init: int = 0, stride: int = 1) -> int:
    assert data.dtype == np.uint32 and data.flags.c_contiguous
    return _load().oracle_delta_decode_inplace(_p32(data), data.size, init, stride)


def vbyte_encode(vals) -> bytes:
    v = _u32(vals)
    buf = np.zeros(v.size * 5 + 1, dtype=np.uint8)
    nb = _load().oracle_vbyte_encode(_p32(v), v.size, _p8(buf))
    return buf[:nb].tobytes()


def vbyte_decode(data: bytes, count: int):
    """Returns (values, bytes consumed) or raises ValueError on a bad stream."""
    buf = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8).copy()
    out = np.zeros(max(count, 1), dtype=np.uint32)
    used = _load().oracle_vbyte_decode(_p8(buf), len(data), count, _p32(out))
    if used < 0:
        raise ValueError("corrupt Variable Byte data")
    return out[:count], int(used)


def fp_choose(vals):
    """Width choice of the patched codec for one block: (b, maxb, c)."""
    v = _u32(vals)
    b = np.zeros(1, np.uint32)
    m = np.zeros(1, np.uint32)
    c = np.zeros(1, np.uint32)
    _load().oracle_fp_choose(_p32(v), v.size, _p32(b), _p32(m), _p32(c))
    return int(b[0]), int(m[0]), int(c[0])


def max_words(codec: int, n: int) -> int:
    return int(_load().oracle_max_words(codec, n))


def _encode(fn, codec, x, stride):
    x = _u32(x)
    cap = max_words(codec, x.size)
    out = np.zeros(cap, dtype=np.uint32)
    src = x if x.size else np.zeros(1, np.uint32)
    w = fn(_p32(src), x.size, stride, _p32(out), cap)
    if w < 0:
        raise ValueError(f"oracle encode failed: {w}")
    return out[:w].copy()


def bp_encode(x, stride: int = 1) -> np.ndarray:
    """Binary-packing (SIMD-BP128 layout) stream of x."""
    return _encode(_load().oracle_bp_encode, CODEC_BP, x, stride)


def fp_encode(x, stride: int = 1) -> np.ndarray:
    """Patched (SIMD-FastPFOR layout) stream of x."""
    return _encode(_load().oracle_fp_encode, CODEC_FP, x, stride)


def bp32_encode(x, stride: int = 1) -> np.ndarray:
    """BP32 stream of x: 32-integer blocks, four per meta-block behind a
    word of widths."""
    return _encode(_load().oracle_bp32_encode, CODEC_BP32, x, stride)


def fp32_encode(x, stride: int = 1) -> np.ndarray:
    """Patched (FastPFOR) stream of x: exception arrays padded to 32 values."""
    return _encode(_load().oracle_fp32_encode, CODEC_FP32, x, stride)


def bpv_encode(x, stride: int = 1) -> np.ndarray:
    """SIMD-BP128 stream of x with the paper's four-lane (vertical) block layout."""
    return _encode(_load().oracle_bpv_encode, CODEC_BPV, x, stride)


def _decode(fn, stream, n):
    s = _u32(stream)
    out = np.zeros(max(n, 1), dtype=np.uint32)
    rc = fn(_p32(s if s.size else np.zeros(1, np.uint32)), s.size, _p32(out), n)
    return rc, out[:n]


def bp_decode(stream, n: int) -> np.ndarray:
    rc, out = _decode(_load().oracle_bp_decode, stream, n)
    if rc != OK:
        raise ValueError(f"oracle decode failed: {rc}")
    return out


def fp_decode(stream, n: int) -> np.ndarray:
    rc, out = _decode(_load().oracle_fp_decode, stream, n)
    if rc != OK:
        raise ValueError(f"oracle decode failed: {rc}")
    return out


def bp32_decode(stream, n: int) -> np.ndarray:
    rc, out = _decode(_load().oracle_bp32_decode, stream, n)
    if rc != OK:
        raise ValueError(f"oracle decode failed: {rc}")
    return out


def fp32_decode(stream, n: int) -> np.ndarray:
    rc, out = _decode(_load().oracle_fp32_decode, stream, n)
    if rc != OK:
        raise ValueError(f"oracle decode failed: {rc}")
    return out


def fp32_decode_rc(stream, n: int) -> int:
    return _decode(_load().oracle_fp32_decode, stream, n)[0]


def bpv_decode(stream, n: int) -> np.ndarray:
    rc, out = _decode(_load().oracle_bpv_decode, stream, n)
    if rc != OK:
        raise ValueError(f"oracle decode failed: {rc}")
    return out


def bpv_decode_rc(stream, n: int) -> int:
    return _decode(_load().oracle_bpv_decode, stream, n)[0]


def bp32_decode_rc(stream, n: int) -> int:
    return _decode(_load().oracle_bp32_decode, stream, n)[0]


def bp_decode_rc(stream, n: int) -> int:
    return _decode(_load().oracle_bp_decode, stream, n)[0]


def fp_decode_rc(stream, n: int) -> int:
    return _decode(_load().oracle_fp_decode, stream, n)[0]


def intersect(a, b) -> np.ndarray:
    """Values present in both strictly increasing arrays a and b, ascending."""
    a, b = _u32(a), _u32(b)
    out = np.zeros(max(1, min(a.size, b.size)), dtype=np.uint32)
    k = _load().oracle_intersect(_p32(a), a.size, _p32(b), b.size, _p32(out))
    return out[:k].copy()


def sp_encode(x, stride: int = 1) -> np.ndarray:
    """SimplePFOR stream of x: FastPFOR pages whose exceptions' high parts
    are one Simple-8b array per page."""
    return _encode(_load().oracle_sp_encode, CODEC_SP, x, stride)


def sp_decode(stream, n: int) -> np.ndarray:
    rc, out = _decode(_load().oracle_sp_decode, stream, n)
    if rc != OK:
        raise ValueError(f"oracle decode failed: {rc}")
    return out


def sp_decode_rc(stream, n: int) -> int:
    return _decode(_load().oracle_sp_decode, stream, n)[0]


def fpi_encode(x, stride: int = 1) -> np.ndarray:
    """FastPFOR stream of x whose pages keep the paper's own layout (offset
    word, truncated values, counted byte array, bitset and counted arrays)."""
    return _encode(_load().oracle_fpi_encode, CODEC_FPI, x, stride)


def fpi_decode(stream, n: int) -> np.ndarray:
    rc, out = _decode(_load().oracle_fpi_decode, stream, n)
    if rc != OK:
        raise ValueError(f"oracle decode failed: {rc}")
    return out


def fpi_decode_rc(stream, n: int) -> int:
    return _decode(_load().oracle_fpi_decode, stream, n)[0]


def s8_mode(selector: int):
    """(integers per word, bits per integer) of a Simple-8b selector."""
    c, b = ctypes.c_uint32(), ctypes.c_uint32()
    _load().oracle_s8_mode(selector, ctypes.byref(c), ctypes.byref(b))
    return int(c.value), int(b.value)


def s8_encode(v) -> np.ndarray:
    """Simple-8b words (uint64) of the uint32 values v, greedy."""
    v = _u32(v)
    out = np.zeros(max(v.size, 1), dtype=np.uint64)
    src = v if v.size else np.zeros(1, np.uint32)
    w = _load().oracle_s8_encode(_p32(src), v.size, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out[:w].copy()


def s8_decode(words, n: int):
    """(count or negative error, values) of Simple-8b words holding at most n values."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    out = np.zeros(max(n, 1), dtype=np.uint32)
    src = w if w.size else np.zeros(1, np.uint64)
    k = _load().oracle_s8_decode(src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), w.size, _p32(out), n)
    return int(k), out[:max(k, 0)]
