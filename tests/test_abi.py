"""The C-ABI library loads and exports every entry point its header
declares (no GPU calls). Also checks host-only logic: the capacity bound
agrees with what the oracle can produce."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1209_2137_amd as wp
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "wavepack.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\([^;{]*\)\s*;", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("bp_encode", "bp_decode", "fastpfor_encode", "fastpfor_decode", "delta_decode_inplace",
                 "wp_max_compressed_words", "wp_check", "wp_strerror", "wp_batch_plan",
                 "wp_batch_decode", "wp_batch_free", "wp_batch_items"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(wp.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    for name in wp.EXPORTS:
        assert hasattr(lib, name), name


def test_strerror_and_capacity_bound():
    L = wp.lib()
    assert wp.strerror(wp.ERR_CORRUPT) == "corrupt compressed stream"
    assert L.wp_max_compressed_words(7, 10) == 0
    rng = np.random.default_rng(0)
    for n in (0, 1, 127, 128, 2049, 65536 + 5, 200000):
        x = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        for codec, enc in ((wp.CODEC_BP, oracle.bp_encode), (wp.CODEC_FP, oracle.fp_encode)):
            for stride in (0, 1, 4):
                assert enc(x, stride).size <= wp.max_compressed_words(codec, n)


def test_host_argument_errors_need_no_gpu():
    L = wp.lib()
    # bad stride is rejected before any device call
    assert L.delta_decode_inplace(None, 10, 0, 2, None) == wp.ERR_INVALID_ARG
    assert L.delta_decode_inplace(None, 0, 0, 1, None) == wp.OK
    # null stream pointer / too-short stream
    assert L.bp_decode(None, 8, None, 0, None) == wp.ERR_INVALID_ARG
    assert L.fastpfor_decode(ctypes.c_void_p(16), 4, None, 0, None) == wp.ERR_INVALID_ARG
    # misaligned pointers
    assert L.bp_decode(ctypes.c_void_p(4), 8, ctypes.c_void_p(16), 1, None) == wp.ERR_INVALID_ARG


def test_range_and_intersection_argument_errors_need_no_gpu():
    L = wp.lib()
    p16, r8 = ctypes.c_void_p(16), ctypes.c_void_p(64)
    # key_lo > key_hi, unknown codec, null or misaligned pointers: rejected on the host
    assert L.wp_decode_range(p16, 64, 10, wp.CODEC_BP, 5, 4, p16, r8, None) == wp.ERR_INVALID_ARG
    assert L.wp_decode_range(p16, 64, 10, 9, 0, 4, p16, r8, None) == wp.ERR_INVALID_ARG
    assert L.wp_decode_range(None, 64, 10, wp.CODEC_BP, 0, 4, p16, r8, None) == wp.ERR_INVALID_ARG
    assert L.wp_decode_range(p16, 64, 10, wp.CODEC_BP, 0, 4, p16, None, None) == wp.ERR_INVALID_ARG
    assert L.wp_decode_range(p16, 64, 10, wp.CODEC_BP, 0, 4, ctypes.c_void_p(20), r8, None) == wp.ERR_INVALID_ARG
    assert L.wp_decode_range(p16, 64, 10, wp.CODEC_BP, 0, 4, p16, ctypes.c_void_p(68), None) == wp.ERR_INVALID_ARG
    assert L.wp_decode_range(p16, 4, 10, wp.CODEC_BP, 0, 4, p16, r8, None) == wp.ERR_INVALID_ARG
