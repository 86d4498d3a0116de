"""A resident pool of compressed lists on the GPU.

Lists are encoded by the GPU encoders straight into slots of one device
buffer (each slot sized for its list's worst case, so no synchronisation is
needed between lists), their lengths land in a device array and are read
back once. The registry rows (comp_off_words, comp_words, out_off, n, codec)
feed BatchPlan. Argument marshalling only: all encoding runs in the HIP
kernels.
"""
from __future__ import annotations

import numpy as np

from . import CODEC_BP, CODEC_FP, BatchPlan, _check, _need_u32, _ptr, _stream, lib, max_compressed_words


def _round4(v: int) -> int:
    return (int(v) + 3) & ~3


class ListPool:
    """Compressed lists resident in device memory.

    arrays: sequence of 1-D uint32 numpy arrays (or a callable i -> array
    with `count` lists); codecs: per-list CODEC_BP / CODEC_FP; stride: delta
    stride used for every list.
    Attributes: pool (device int32), values (device int32, all inputs
    concatenated with 4-aligned starts, kept only if keep_values), rows
    (registry), out_offsets, total_n, comp_bytes.
    """

    def __init__(self, arrays, codecs, stride: int = 1, count: int | None = None, keep_values: bool = True,
                 stream=None, device="cuda"):
        import torch
        get = arrays if callable(arrays) else (lambda i: arrays[i])
        count = len(codecs) if count is None else count
        lens = np.zeros(count, dtype=np.int64)
        host = []
        for i in range(count):
            a = np.ascontiguousarray(get(i), dtype=np.uint32)
            host.append(a)
            lens[i] = a.size
        out_off = np.zeros(count, dtype=np.int64)
        comp_off = np.zeros(count, dtype=np.int64)
        o = c = 0
        for i in range(count):
            out_off[i] = o
            comp_off[i] = c
            o += _round4(lens[i])
            c += _round4(max_compressed_words(int(codecs[i]), int(lens[i])))
        self.total_out = int(o)
        vals = np.zeros(max(self.total_out, 4), dtype=np.uint32)
        for i in range(count):
            vals[out_off[i]:out_off[i] + lens[i]] = host[i]
        del host
        self.values = torch.from_numpy(vals.view(np.int32)).to(device)
        del vals
        self.pool = torch.empty(max(int(c), 4), dtype=torch.int32, device=device)
        words = torch.zeros(max(count, 1), dtype=torch.int64, device=device)
        L = lib()
        s = _stream(stream)
        wptr = words.data_ptr()
        vptr, pptr = self.values.data_ptr(), self.pool.data_ptr()
        for i in range(count):
            fn = L.bp_encode if int(codecs[i]) == CODEC_BP else L.fastpfor_encode
            cap = max_compressed_words(int(codecs[i]), int(lens[i]))
            _check(fn(vptr + 4 * int(out_off[i]), int(lens[i]), int(stride), pptr + 4 * int(comp_off[i]), cap,
                      wptr + 8 * i, s), "encode into pool")
        torch.cuda.synchronize()
        _check(L.wp_check(s), "encode into pool")
        w = words.cpu().numpy()[:count]
        self.rows = [(int(comp_off[i]), int(w[i]), int(out_off[i]), int(lens[i]), int(codecs[i]))
                     for i in range(count)]
        self.lens = lens
        self.codecs = np.asarray(codecs[:count], dtype=np.int32)
        self.out_offsets = out_off
        self.total_n = int(lens.sum())
        self.comp_bytes = int(4 * w.sum())
        if not keep_values:
            self.values = None

    def streams(self):
        """The compressed lists back to back in one host uint32 array (each
        stream on a 4-word boundary) and their registry rows, with offsets
        into that array; from_streams() makes a pool of them again."""
        words = self.pool.cpu().numpy().view(np.uint32)
        offs, o = [], 0
        for co, cw, _, _, _ in self.rows:
            offs.append(o)
            o += _round4(cw)
        packed = np.zeros(max(o, 4), dtype=np.uint32)
        for (co, cw, _, _, _), po in zip(self.rows, offs):
            packed[po:po + cw] = words[co:co + cw]
        rows = np.array([(po, cw, oo, n, codec) for (_, cw, oo, n, codec), po in zip(self.rows, offs)],
                        dtype=np.int64).reshape(-1, 5)
        return packed, rows

    @classmethod
    def from_streams(cls, packed, rows, device="cuda"):
        """A resident pool of already compressed lists (the arrays returned
        by streams()); no input values are kept."""
        import torch
        self = cls.__new__(cls)
        packed = np.ascontiguousarray(packed, dtype=np.uint32)
        self.pool = torch.from_numpy(packed.view(np.int32)).to(device)
        rows = np.asarray(rows, dtype=np.int64).reshape(-1, 5)
        self.rows = [tuple(int(v) for v in r) for r in rows]
        self.lens = rows[:, 3].copy()
        self.codecs = rows[:, 4].astype(np.int32)
        self.out_offsets = rows[:, 2].copy()
        self.total_out = int(max((r[2] + _round4(r[3]) for r in self.rows), default=0))
        self.total_n = int(self.lens.sum())
        self.comp_bytes = int(4 * rows[:, 1].sum())
        self.values = None
        return self

    def rows_for(self, ids, out_offsets):
        """Registry rows of lists `ids` writing to the given output offsets."""
        return [(self.rows[i][0], self.rows[i][1], int(oo), self.rows[i][3], self.rows[i][4])
                for i, oo in zip(ids, out_offsets)]

    def plan(self, out, tune=None, stream=None) -> BatchPlan:
        """A plan decoding every list of the pool into `out` at the pool's offsets."""
        _need_u32(out, "out")
        return BatchPlan(self.pool, out, self.rows, tune=tune, stream=stream)

    def decode_one(self, i: int, out, stream=None):
        """Single-list decode of list i into out (at its pool offset)."""
        co, cw, oo, n, codec = self.rows[i]
        fn = lib().bp_decode if codec == CODEC_BP else lib().fastpfor_decode
        _check(fn(self.pool.data_ptr() + 4 * co, cw, out.data_ptr() + 4 * oo, n, _stream(stream)),
               "single-list decode")


__all__ = ["ListPool", "CODEC_BP", "CODEC_FP"]
