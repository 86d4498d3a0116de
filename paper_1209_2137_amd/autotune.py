"""Autotuner for the decoders' workgroup shapes.

Knobs:
  waves      wavefronts per workgroup (1, 2, 4, 8; batched 2, 4, 8)
  vpl        integers per lane and pass (4)
  depth      binary packing: 16-byte loads in flight per lane, which also
             sizes each wavefront's LDS ring (2 or 3: 4 KB, 4: 8 KB)
  wg_per_cu  single list, binary packing (SIMD-BP128 and BP32, each its
             own shape): runs (one per wavefront) per compute unit;
             batched decoding: 0 = one-shot grid, > 0 = persistent
             workgroups per compute unit pulling items from a work queue
  run_units  batched decoding: meta-blocks per work item

Each candidate is timed with HIP events (median of `steps` launches after
warm-up, inputs rotated so the 256 MB Infinity Cache cannot serve them);
the fastest goes into a JSON table keyed by architecture, codec and
workload class. `apply()` installs a table's single-list shapes in the C
library; the package applies `tuning.json` when it loads the library.
"""
from __future__ import annotations

import json
import os
import time

TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

BP_SINGLE = [dict(waves=w, vpl=4, depth=d, wg_per_cu=c)
             for w in (1, 2, 4, 8) for d in (2, 3) for c in (28, 56, 128, 256)] + \
            [dict(waves=w, vpl=4, depth=4, wg_per_cu=c) for w in (1, 4) for c in (64, 128)]
FP_SINGLE = [dict(waves=w, vpl=4) for w in (1, 2, 4, 8)]
BP32_SINGLE = [dict(waves=w, vpl=4, depth=d, wg_per_cu=c) for w in (2, 4, 8) for d in (2, 3) for c in (56, 128, 256)]
BATCH = [dict(waves=w, vpl=4, depth=d, run_units=r, wg_per_cu=0, use_graph=1)
         for w in (2, 4, 8) for d in (2, 3) for r in (1, 2, 4, 8)] + \
        [dict(waves=4, vpl=4, depth=2, run_units=r, wg_per_cu=c, use_graph=1) for r in (4, 8) for c in (4, 8)]


def load(path: str = TUNING_PATH) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(table: dict, path: str = TUNING_PATH):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "gfx950"


def apply(table: dict | None = None, arch_name: str = "gfx950"):
    """Installs the table's single-list shapes (binary packing, patched,
    BP32; BP32 takes its default shape when the table has none)."""
    from . import CODEC_BP, CODEC_BP32, CODEC_FP, lib
    table = load() if table is None else table
    ent = table.get(arch_name, {})
    bp = ent.get("bp_single")
    if bp:
        lib().wp_set_decode_tune(CODEC_BP, bp["waves"], bp["vpl"], bp.get("depth", 0), bp.get("wg_per_cu", 0))
    fp = ent.get("fp_single")
    if fp:
        lib().wp_set_decode_tune(CODEC_FP, fp["waves"], fp["vpl"], fp.get("depth", 0), 0)
    b32 = ent.get("bp32_single") or dict(waves=4, vpl=4, depth=2, wg_per_cu=0)
    lib().wp_set_decode_tune(CODEC_BP32, b32["waves"], b32["vpl"], b32.get("depth", 0), b32.get("wg_per_cu", 0))


def batch_tune(table: dict | None = None, arch_name: str = "gfx950") -> dict | None:
    table = load() if table is None else table
    return table.get(arch_name, {}).get("batch")


def _median_ms(fn, steps, warmup):
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    ts = []
    for i in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn(warmup + i)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune_single(codec: int, x_np, candidates=None, steps: int = 9, warmup: int = 3, log=print):
    """Times every candidate shape decoding x (numpy uint32) with `codec`."""
    import torch
    from . import CODEC_BP, CODEC_BP32, CODEC_FP, bp32_decode, bp_decode, check, encode_trimmed, fastpfor_decode, \
        set_decode_tune
    xd = torch.from_numpy(x_np.view("int32")).to("cuda")
    comp = encode_trimmed(xd, codec, 1)
    reps = max(2, min(16, (512 << 20) // max(comp.numel() * 4, 1)))
    comps = [comp] + [comp.clone() for _ in range(reps - 1)]
    outs = [torch.empty_like(xd) for _ in range(2)]
    dec = {CODEC_BP: bp_decode, CODEC_FP: fastpfor_decode, CODEC_BP32: bp32_decode}[codec]
    cands = candidates or {CODEC_BP: BP_SINGLE, CODEC_FP: FP_SINGLE, CODEC_BP32: BP32_SINGLE}[codec]
    results = []
    for c in cands:
        set_decode_tune(codec, c["waves"], c["vpl"], c.get("wg_per_cu", 0), c.get("depth", 0))
        dec(comps[0], xd.numel(), outs[0])
        check()
        if not torch.equal(outs[0], xd):
            raise RuntimeError(f"shape {c} decoded wrongly")
        ms = _median_ms(lambda i: dec(comps[i % reps], xd.numel(), outs[i % 2]), steps, warmup)
        results.append((ms, c))
        log(f"  {c}: {ms * 1e3:.1f} us, {xd.numel() / ms / 1e6:.0f} G ints/s")
    results.sort(key=lambda t: t[0])
    best = dict(results[0][1])
    set_decode_tune(codec, best["waves"], best["vpl"], best.get("wg_per_cu", 0), best.get("depth", 0))
    return best, results


def tune_batch(pool, candidates=None, steps: int = 7, warmup: int = 2, log=print):
    """Times batched decoding of a ListPool for every candidate shape."""
    import torch
    from . import check
    out = torch.empty(pool.total_out + 4, dtype=torch.int32, device="cuda")
    results = []
    for c in (candidates or BATCH):
        plan = pool.plan(out, tune=c)
        plan.decode()
        check()
        ms = _median_ms(lambda i: plan.decode(), steps, warmup)
        plan.free()
        results.append((ms, c))
        log(f"  {c}: {ms:.3f} ms, {pool.total_n / ms / 1e6:.0f} G ints/s")
    results.sort(key=lambda t: t[0])
    return dict(results[0][1]), results


def main():
    """Tunes single-list and batched shapes on the standard synthetic
    workloads and writes tuning.json."""
    import argparse
    from . import CODEC_BP, CODEC_BP32, CODEC_FP, datagen
    from .pool import ListPool
    ap = argparse.ArgumentParser()
    ap.add_argument("--lists", type=int, default=20000, help="lists in the batched-decoding pool")
    ap.add_argument("--total", type=float, default=2.4e8, help="integers in the batched-decoding pool")
    ap.add_argument("--out", default=TUNING_PATH, help="where to write the table")
    args = ap.parse_args()
    t0 = time.time()
    table = load(args.out) if os.path.exists(args.out) else load()
    a = arch()
    ent = table.setdefault(a, {})
    print("binary packing, 2^26 recursive-cluster list", flush=True)
    best_bp, _ = tune_single(CODEC_BP, datagen.cluster_sorted(1 << 26, seed=2))
    ent["bp_single"] = best_bp
    print("BP32, 2^26 recursive-cluster list", flush=True)
    best_b32, _ = tune_single(CODEC_BP32, datagen.cluster_sorted(1 << 26, seed=2))
    ent["bp32_single"] = best_b32
    print("patched, 2^28 list", flush=True)
    best_fp, _ = tune_single(CODEC_FP, datagen.patched_gaps(1 << 28, seed=4))
    ent["fp_single"] = best_fp
    print(f"batched, {args.lists} posting lists", flush=True)
    lens, codec, means, list_array = datagen.posting_lists(n_lists=args.lists, total=args.total, seed=5)
    pool = ListPool(list_array, codec, stride=1, count=args.lists, keep_values=False)
    best_batch, _ = tune_batch(pool)
    ent["batch"] = best_batch
    ent["tuned_at"] = time.strftime("%Y-%m-%d %H:%M:%S")
    save(table, args.out)
    print(json.dumps(ent), f"({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
