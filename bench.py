#!/usr/bin/env python3
"""Decode throughput of wavepack on one MI355X.

A step is one decode of the whole headline list: 2^26 sorted distinct
uint32 from the recursive-cluster generator in [0, 2^30), compressed with
binary packing (128-integer blocks, 16 per meta-block) and standard
differential coding, decoded back to the sorted array (unpack + prefix sum
in one kernel). Inputs are resident in HBM before the timed region; the
compressed stream is produced by the GPU encoder.

Prints ONE JSON line. Extra workloads (the 2^26 uniform list, the 2^28
patched list, the in-place delta scan, batched decoding) are reported under
"extra"; `--quick` skips them.

  python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--quick]
  python bench.py --rocprof-summary DIR   # summarise rocprofv3 CSV output
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded uint32/s (G ints/s) + % HBM peak; batched vs per-list; p99 latency"
HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256 << 20
KERNEL_SOURCES = ("paper_1209_2137_amd/csrc/wp_device.hpp", "paper_1209_2137_amd/csrc/wp_decode.hip",
                  "paper_1209_2137_amd/tuning.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "bp_decode_cluster_2e26_counters.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_alg_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel sources."""
    try:
        with open(COUNTERS_FILE) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_hash") != kernel_hash():
        return None
    return c.get("traffic_bytes_per_launch")


def to_dev(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to("cuda")


def time_launches(fn, steps, warmup, stream, kernel_events=None):
    """Runs fn(i) warmup times, then `steps` times back to back with nothing
    between the launches (the host clock around them gives the wall time
    per step), then `steps` more times with timing events. Returns (wall ms
    per step, mean event ms). With kernel_events (the package), each
    launch's own main kernel records a pair of HIP events when it starts and
    ends (wp_time_next_launch), so the event time is the kernel's duration;
    otherwise the events bracket each launch on `stream`. (Events between
    launches add a few microseconds of gap each, so they stay out of the
    wall-time loop; with kernel events, `warmup` untimed launches queued just
    before the timed ones keep the GPU busy between them.)"""
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn(warmup + i)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    if kernel_events is not None:
        for e in starts + ends:  # create the events on the device before handing them over
            e.record(stream)
        torch.cuda.synchronize()
        # a backlog of untimed launches first, so that the timed kernels run
        # back to back as in the wall-time loop instead of each starting on
        # an idle GPU after the host's per-launch work
        for i in range(warmup):
            fn(warmup + i)
    for i in range(steps):
        if kernel_events is not None:
            kernel_events.time_next_launch(starts[i], ends[i])
        else:
            starts[i].record(stream)
        fn(warmup + steps + i)
        if kernel_events is None:
            ends[i].record(stream)
    torch.cuda.synchronize()
    ev = sum(s.elapsed_time(e) for s, e in zip(starts, ends)) / steps
    return wall, ev


def replicas(t, nbytes_each):
    """Copies of t so that the rotation's working set is well above the
    256 MB Infinity Cache."""
    r = max(2, min(16, math.ceil(2 * MALL_BYTES / max(nbytes_each, 1))))
    return [t] + [t.clone() for _ in range(r - 1)]


def bench_single(wp, x_np, codec, stride, steps, warmup, name, comp=None, n=None):
    """Decoder timing on x_np, encoded here; or on a given stream `comp`
    (device) of n integers, with no comparison against the input."""
    import torch
    if comp is None:
        xd = to_dev(x_np)
        n = x_np.size
        comp = wp.encode_trimmed(xd, codec, stride)
    else:
        xd = None
    comps = replicas(comp, comp.numel() * 4)
    outs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(2)]
    dec = {wp.CODEC_BP: wp.bp_decode, wp.CODEC_FP: wp.fastpfor_decode, wp.CODEC_BP32: wp.bp32_decode,
           wp.CODEC_FP32: wp.fastpfor32_decode, wp.CODEC_BPV: wp.bp_vertical_decode,
           wp.CODEC_SP: wp.simplepfor_decode, wp.CODEC_FPI: wp.fastpfor_inline_decode}[codec]
    stream = torch.cuda.current_stream()
    dec(comps[0], n, outs[0])
    wp.check()
    if xd is not None and not torch.equal(outs[0], xd):
        raise RuntimeError(f"{name}: decoded output differs from the input")
    del xd
    wall, ev = time_launches(lambda i: dec(comps[i % len(comps)], n, outs[i % 2]), steps, warmup, stream,
                            kernel_events=wp)
    wp.check()
    comp_bytes = comp.numel() * 4
    alg = comp_bytes + 4 * n
    return {
        "name": name, "n": n,
        "codec": {wp.CODEC_BP: "bp", wp.CODEC_FP: "fp", wp.CODEC_BP32: "bp32", wp.CODEC_FP32: "fp32",
                  wp.CODEC_BPV: "bpv", wp.CODEC_SP: "sp", wp.CODEC_FPI: "fpi"}[codec],
        "stride": stride,
        "bits_per_int": comp_bytes * 8 / n, "ms_per_step": wall, "kernel_ms": ev,
        "gints_per_s": n / (wall * 1e-3) / 1e9, "kernel_gints_per_s": n / (ev * 1e-3) / 1e9,
        "alg_bytes": alg, "achieved_gbs": alg / (ev * 1e-3) / 1e9,
        "hbm_frac": alg / (ev * 1e-3) / 1e9 / HBM_PEAK_GBS, "replicas": len(comps),
    }


def bench_encode(wp, x_np, codec, stride, steps, warmup, name):
    """Encoder throughput (all its kernels, timed as one call): algorithmic
    bytes = the input read once plus the stream written."""
    import torch
    xd = to_dev(x_np)
    n = x_np.size
    xs = replicas(xd, n * 4)
    enc = {wp.CODEC_BP: wp.bp_encode, wp.CODEC_FP: wp.fastpfor_encode, wp.CODEC_BP32: wp.bp32_encode,
           wp.CODEC_FP32: wp.fastpfor32_encode, wp.CODEC_BPV: wp.bp_vertical_encode,
           wp.CODEC_SP: wp.simplepfor_encode, wp.CODEC_FPI: wp.fastpfor_inline_encode}[codec]
    buf, words = enc(xd, stride)
    wp.check()
    comp_words = int(words.item())
    bufs = [buf, torch.empty_like(buf)]
    stream = torch.cuda.current_stream()
    wall, ev = time_launches(lambda i: enc(xs[i % len(xs)], stride, out=bufs[i % 2], out_words=words), steps,
                             warmup, stream)
    wp.check()
    if int(words.item()) != comp_words:
        raise RuntimeError(f"{name}: the stream length changed between calls")
    alg = 4 * n + 4 * comp_words
    return {"name": name, "n": n, "ms_per_step": wall, "event_ms": ev, "gints_per_s": n / (ev * 1e-3) / 1e9,
            "bits_per_int": comp_words * 32 / n, "alg_bytes": alg, "achieved_gbs": alg / (ev * 1e-3) / 1e9,
            "hbm_frac": alg / (ev * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_intersect(wp, steps, warmup, na=1 << 20, nb=1 << 24):
    """Intersection of two decoded posting lists (recursive-cluster lists of
    2^20 and 2^24 values in [0, 2^30)); checked against numpy once. Bytes:
    both lists read once and the result written (what a merge would move)."""
    import numpy as np
    import torch
    from paper_1209_2137_amd import datagen
    a_np, b_np = datagen.cluster_sorted(na, seed=21), datagen.cluster_sorted(nb, seed=22)
    a, b = to_dev(a_np), to_dev(b_np)
    out = torch.empty(na, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    wp.intersect(a, b, out=out, count=count)
    wp.check()
    k = int(count.item())
    want = np.intersect1d(a_np, b_np, assume_unique=True)
    if k != want.size or not np.array_equal(out[:k].cpu().numpy().view(np.uint32), want):
        raise RuntimeError("intersection differs from numpy's")
    wall, ev = time_launches(lambda i: wp.intersect(a, b, out=out, count=count), steps, warmup,
                             torch.cuda.current_stream())
    alg = 4 * (na + nb + k)
    return {"name": "intersect 2^20 x 2^24 cluster lists", "na": na, "nb": nb, "common": k, "ms_per_step": wall,
            "event_ms": ev, "lookups_per_s": na / (ev * 1e-3) / 1e9, "achieved_gbs": alg / (ev * 1e-3) / 1e9,
            "hbm_frac": alg / (ev * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_intersect_compressed(wp, steps, warmup, nb=1 << 24, nas=(1 << 10, 1 << 14, 1 << 18)):
    """A short list against a 2^24-value list that stays compressed (binary
    packing, differential coding): only the units the short list falls in
    are decoded. Timed beside decoding the whole list and intersecting the
    decoded lists; each result checked against numpy once."""
    import numpy as np
    import torch
    from paper_1209_2137_amd import datagen
    b_np = datagen.cluster_sorted(nb, seed=22)
    b = to_dev(b_np)
    comp = wp.encode_trimmed(b, wp.CODEC_BP, 1)
    work = torch.empty(nb, dtype=torch.int32, device="cuda")
    full = torch.empty(nb, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for na in nas:
        a_np = datagen.cluster_sorted(na, seed=23)
        a = to_dev(a_np)
        out = torch.empty(na, dtype=torch.int32, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        wp.intersect_compressed(a, comp, nb, wp.CODEC_BP, work=work, out=out, count=count)
        wp.check()
        k = int(count.item())
        want = np.intersect1d(a_np, b_np, assume_unique=True)
        if k != want.size or not np.array_equal(out[:k].cpu().numpy().view(np.uint32), want):
            raise RuntimeError("compressed intersection differs from numpy's")
        wall, ev = time_launches(lambda i: wp.intersect_compressed(a, comp, nb, wp.CODEC_BP, work=work, out=out,
                                                                   count=count), steps, warmup, stream)

        def decode_then_intersect(i):
            wp.bp_decode(comp, nb, full)
            wp.intersect(a, full, out=out, count=count)

        wall_full, ev_full = time_launches(decode_then_intersect, steps, warmup, stream)
        rows.append({"na": na, "common": k, "ms_per_step": wall, "event_ms": ev, "decode_all_ms": wall_full,
                     "decode_all_event_ms": ev_full, "speedup": wall_full / wall})
    return {"name": "intersect short lists x compressed 2^24 cluster list", "nb": nb, "comp_words": comp.numel(),
            "rows": rows}


def bench_decode_range(wp, x, steps, warmup, spans=(1 << 10, 1 << 16, 1 << 22)):
    """Random access by key on the 2^26 recursive-cluster list (binary
    packing, differential coding): key ranges covering about 2^10, 2^16 and
    2^22 values, only the units they touch decoded; timed beside decoding
    the whole list. Each range checked against numpy's searchsorted once."""
    import numpy as np
    import torch
    n = x.size
    xd = to_dev(x)
    comp = wp.encode_trimmed(xd, wp.CODEC_BP, 1)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    rng_t = torch.zeros(2, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    wall_full, ev_full = time_launches(lambda i: wp.bp_decode(comp, n, out), steps, warmup, stream)
    rows = []
    for span in spans:
        i = n // 3
        lo, hi = int(x[i]), int(x[i + span - 1])
        wp.decode_range(comp, n, wp.CODEC_BP, lo, hi, out=out, rng=rng_t)
        wp.check()
        i0, i1 = (int(v) for v in rng_t.cpu().numpy())
        if (i0, i1) != (int(np.searchsorted(x, lo)), int(np.searchsorted(x, hi, side="right"))) or \
                not np.array_equal(out[i0:i1].cpu().numpy().view(np.uint32), x[i0:i1]):
            raise RuntimeError("decode_range differs from numpy's searchsorted")
        wall, ev = time_launches(lambda k: wp.decode_range(comp, n, wp.CODEC_BP, lo, hi, out=out, rng=rng_t),
                                 steps, warmup, stream)
        rows.append({"values": i1 - i0, "ms_per_step": wall, "event_ms": ev, "speedup_vs_full": wall_full / wall})
    return {"name": "decode_range on the 2^26 cluster list", "n": n, "full_decode_ms": wall_full, "rows": rows}


def bench_delta(wp, n, steps, warmup):
    import torch
    rng_t = torch.randint(0, 1 << 8, (n,), dtype=torch.int32, device="cuda")
    bufs = replicas(rng_t, n * 4)
    stream = torch.cuda.current_stream()
    wall, ev = time_launches(lambda i: wp.delta_decode_inplace(bufs[i % len(bufs)], 0, 1), steps, warmup, stream,
                             kernel_events=wp)
    alg = 8 * n
    return {"name": "delta_decode_inplace 2^28 stride 1", "n": n, "ms_per_step": wall, "kernel_ms": ev,
            "gints_per_s": n / (wall * 1e-3) / 1e9, "achieved_gbs": alg / (ev * 1e-3) / 1e9,
            "hbm_frac": alg / (ev * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_copy(n_bytes, steps, warmup):
    """A plain device copy of known size: the bandwidth reference."""
    import torch
    src = torch.empty(n_bytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    dsts = [torch.empty_like(src) for _ in range(2)]
    stream = torch.cuda.current_stream()
    wall, ev = time_launches(lambda i: dsts[i % 2].copy_(src), steps, warmup, stream)
    return {"bytes": 2 * n_bytes, "kernel_ms": ev, "gbs": 2 * n_bytes / (ev * 1e-3) / 1e9}


def bench_batch(wp, steps, warmup, per_list_passes=2):
    """Posting-list pool: one batched decode launch (hipGraph) vs one
    single-list launch per list on the same stream."""
    import torch
    from paper_1209_2137_amd.autotune import batch_tune
    t0 = time.perf_counter()
    pool = posting_pool(True)
    t_setup = time.perf_counter() - t0
    out = torch.zeros(pool.total_out + 4, dtype=torch.int32, device="cuda")
    tune = batch_tune() or dict(waves=4, vpl=4, depth=3, run_units=4, wg_per_cu=0, use_graph=1)
    tune = dict(tune, use_graph=1)
    plan = pool.plan(out, tune=tune)
    plan.decode()
    wp.check()
    if not torch.equal(out[:pool.total_out], pool.values[:pool.total_out]):
        raise RuntimeError("batched decode differs from the inputs")
    stream = torch.cuda.current_stream()
    wall_b, ev_b = time_launches(lambda i: plan.decode(), steps, warmup, stream)
    out.zero_()
    n = len(pool.rows)

    def per_list(_i):
        for j in range(n):
            pool.decode_one(j, out)

    wall_p, ev_p = time_launches(per_list, per_list_passes, 1, stream)
    wp.check()
    if not torch.equal(out[:pool.total_out], pool.values[:pool.total_out]):
        raise RuntimeError("per-list decode differs from the inputs")
    alg = pool.comp_bytes + 4 * pool.total_n
    res = {
        "name": "batched posting lists", "lists": n, "n": pool.total_n, "items": plan.items,
        "bits_per_int": pool.comp_bytes * 8 / pool.total_n, "tune": tune,
        "batched_ms": wall_b, "batched_kernel_ms": ev_b, "batched_gints_per_s": pool.total_n / (wall_b * 1e-3) / 1e9,
        "batched_achieved_gbs": alg / (ev_b * 1e-3) / 1e9, "batched_hbm_frac": alg / (ev_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "per_list_ms": wall_p, "per_list_gpu_ms": ev_p, "per_list_gints_per_s": pool.total_n / (wall_p * 1e-3) / 1e9,
        "speedup_batched_vs_per_list": wall_p / wall_b, "setup_s": t_setup,
    }
    plan.free()
    del out
    return res, pool


def bench_serve(wp, pool, seconds=60.0, rate=2000.0, budget_bytes=64 << 30):
    """Poisson arrivals of requests for 1..32 lists of the resident pool,
    continuous batching under an HBM output budget, each request decoded
    into a buffer its caller owns (carved from the caller's arena, as large
    as the budget). Every request's output is checked against the pool's
    inputs on a stream of the caller's own."""
    from paper_1209_2137_amd import datagen
    from paper_1209_2137_amd.serve import CheckingCaller, Server, summarize
    times, reqs = datagen.poisson_arrivals(rate=rate, duration=seconds, pool=len(pool.rows), seed=6)
    arena = budget_bytes // 4
    srv = Server(pool, budget_bytes=budget_bytes, streams=4)
    caller = CheckingCaller(pool, arena)
    done = srv.run(times, reqs, caller.get, caller.done)
    srv.close()
    bad = caller.finish()
    wp.check()
    if bad or caller.checked != len(done):
        raise RuntimeError(f"served outputs: {bad} wrong elements, {caller.checked} of {len(done)} checked")
    st = summarize(done, srv.wall)
    st.update({"rate_req_s": rate, "seconds": seconds, "budget_bytes": budget_bytes,
               "arena_bytes": 4 * arena, "streams": 4, "checked_requests": caller.checked,
               "peak_in_flight_bytes": srv.peak_bytes, "waited_for_budget": srv.waited_for_budget,
               "waited_for_buffer": srv.waited_for_buffer})
    del caller
    return st


BOX_CPU_SHARE = 16  # host cores a one-GPU machine grants a run when nothing narrower is visible


def host_cpus():
    """The host's CPUs: os.cpu_count(), the CPUs this process may run on
    (affinity), the cgroup CPU quota if one is set, the CPU model, and the
    number of threads to use: the narrowest of these limits (with neither
    affinity nor quota narrower, the machine's CPU share)."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
        if q != "max":
            quota = int(q) / int(per)
    except (OSError, ValueError):
        pass
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    use = aff if quota is None else max(1, min(aff, int(math.ceil(quota))))
    share_capped = quota is None and use > BOX_CPU_SHARE
    if share_capped:
        use = BOX_CPU_SHARE
    return {"cpu_count": os.cpu_count(), "affinity_cpus": aff, "cgroup_quota_cpus": quota, "model": model,
            "threads": use, "capped_at_box_share": share_capped}


def cpu_baseline(x_np, min_seconds=10.0, par_seconds=8.0):
    """The CPU oracle (plain scalar C, as it stands) decoding the same list:
    first on one thread, then as independent decodes of the same stream on
    every usable host core at once (ctypes releases the interpreter lock for
    each call); `value` and `cores` are the all-cores run's."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    stream = oracle.bp_encode(x_np, 1)
    n = x_np.size
    reps, t0 = 0, time.perf_counter()
    while True:
        out = oracle.bp_decode(stream, n)
        reps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    if not np.array_equal(out, x_np):
        raise RuntimeError("oracle decode mismatch")
    single = reps * n / dt / 1e9
    cpus = host_cpus()
    threads = cpus["threads"]

    def worker(deadline):
        k = 0
        while time.perf_counter() < deadline:
            oracle.bp_decode(stream, n)
            k += 1
        return k

    t1 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        counts = list(ex.map(worker, [t1 + par_seconds] * threads))
    dt1 = time.perf_counter() - t1
    preps = sum(counts)
    return {"value": preps * n / dt1 / 1e9, "unit": "G ints/s", "cores": threads, "kind": "oracle",
            "single_thread_value": single, "model": cpus["model"], "cpu_count": cpus["cpu_count"],
            "affinity_cpus": cpus["affinity_cpus"], "cgroup_quota_cpus": cpus["cgroup_quota_cpus"],
            "sample": f"oracle bp_decode of the whole {n}-integer list: {preps} decodes on {threads} threads "
                      f"({'the box CPU share; ' if cpus['capped_at_box_share'] else ''}"
                      f"{cpus['affinity_cpus']} CPUs in the affinity mask, quota "
                      f"{cpus['cgroup_quota_cpus']}, os.cpu_count() {cpus['cpu_count']}) in {dt1:.1f} s; "
                      f"on one thread {reps} runs in {dt:.1f} s ({single:.3f} G ints/s)"}


def rocprof_summary(d):
    """Markdown summary of rocprofv3 kernel statistics / counter CSVs in d."""
    import csv
    lines = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        lines.append(f"### {os.path.relpath(path, d)}")
        with open(path) as f:
            rows = list(csv.DictReader(f))
        lines.append("| kernel | calls | total ns | avg ns | min ns | max ns |")
        lines.append("|---|---|---|---|---|---|")
        for r in rows:
            lines.append(f"| {r.get('Name', '')[:90]} | {r.get('Calls')} | {r.get('TotalDurationNs')} | "
                         f"{float(r.get('AverageNs', 0)):.0f} | {r.get('MinNs')} | {r.get('MaxNs')} |")
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        lines.append(f"### {os.path.relpath(path, d)}")
        agg = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (r.get("Kernel_Name", "")[:90], r.get("Counter_Name"))
                agg.setdefault(key, []).append(float(r.get("Counter_Value", 0)))
        lines.append("| kernel | counter | dispatches | mean value |")
        lines.append("|---|---|---|---|")
        for (k, c), v in sorted(agg.items()):
            lines.append(f"| {k} | {c} | {len(v)} | {sum(v) / len(v):.1f} |")
    print("\n".join(lines))


def posting_pool(keep_values):
    from paper_1209_2137_amd import datagen
    from paper_1209_2137_amd.pool import ListPool
    lens, codec, means, list_array = datagen.posting_lists(n_lists=100_000, total=1.2e9, seed=5)
    return ListPool(list_array, codec, stride=1, count=len(lens), keep_values=keep_values)


def prepare_inputs(d):
    """Encodes the profiled workloads on the GPU and saves the streams in d,
    so that a profiled run (--profile-run --inputs d) launches decoders
    only."""
    import numpy as np
    import torch
    import paper_1209_2137_amd as wp
    from paper_1209_2137_amd import datagen
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wp.lib()
    os.makedirs(d, exist_ok=True)
    cluster = datagen.cluster_sorted(1 << 26, seed=2)
    patched = datagen.patched_gaps(1 << 28, seed=4)
    for name, x, codec in (("bp_cluster_2e26", cluster, wp.CODEC_BP), ("fp_patched_2e28", patched, wp.CODEC_FP),
                           ("bp32_cluster_2e26", cluster, wp.CODEC_BP32),
                           ("bpv_cluster_2e26", cluster, wp.CODEC_BPV),
                           ("fp32_patched_2e28", patched, wp.CODEC_FP32),
                           ("sp_patched_2e28", patched, wp.CODEC_SP),
                           ("fpi_patched_2e28", patched, wp.CODEC_FPI)):
        comp = wp.encode_trimmed(to_dev(x), codec, 1)
        np.save(os.path.join(d, name + ".npy"), comp.cpu().numpy())
        np.save(os.path.join(d, name + ".n.npy"), np.array([x.size], dtype=np.int64))
        del comp
    packed, rows = posting_pool(False).streams()
    np.save(os.path.join(d, "pool_words.npy"), packed)
    np.save(os.path.join(d, "pool_rows.npy"), rows)
    print(json.dumps({"prepared": d}))
    return 0


def profile_batch(wp, steps, pool):
    """The posting-list pool decoded `steps` times by one batched launch
    each (no per-list leg, no value check: the tests cover it)."""
    import torch
    from paper_1209_2137_amd.autotune import batch_tune
    out = torch.empty(pool.total_out + 4, dtype=torch.int32, device="cuda")
    plan = pool.plan(out, tune=dict(batch_tune() or {}, use_graph=1))
    _, ev = time_launches(lambda i: plan.decode(), steps, 2, torch.cuda.current_stream())
    wp.check()
    plan.free()
    return {"ms": ev, "alg_bytes": pool.comp_bytes + 4 * pool.total_n, "n": pool.total_n}


def profile_variants(steps, inputs):
    """For rocprofv3: the variant codecs' decoders (BP32 and the four-lane
    SIMD-BP128 layout on the 2^26 cluster list; FastPFOR with 32-value
    padding, SimplePFOR and FastPFOR pages in the paper's own layout on the
    2^28 patched list) `steps` times each, from the streams that
    --prepare-inputs saved."""
    import numpy as np
    import torch
    import paper_1209_2137_amd as wp
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wp.lib()
    res = {}
    for name, codec in (("bp32_cluster_2e26", wp.CODEC_BP32), ("bpv_cluster_2e26", wp.CODEC_BPV),
                        ("fp32_patched_2e28", wp.CODEC_FP32), ("sp_patched_2e28", wp.CODEC_SP),
                        ("fpi_patched_2e28", wp.CODEC_FPI)):
        comp = torch.from_numpy(np.load(os.path.join(inputs, name + ".npy"))).to("cuda")
        n = int(np.load(os.path.join(inputs, name + ".n.npy"))[0])
        r = bench_single(wp, None, codec, 1, steps, 2, name, comp=comp, n=n)
        res[name] = {"kernel_ms": r["kernel_ms"], "alg_bytes": r["alg_bytes"], "bits_per_int": r["bits_per_int"]}
        del comp
        torch.cuda.synchronize()
    print(json.dumps(res))
    return 0


def profile_encoders(steps):
    """For rocprofv3 kernel traces (never under counter collection): the
    encoders on their bench workloads, `steps` timed calls each after one
    warm-up: binary packing (both block layouts) and BP32 on the 2^26
    cluster list, FastPFOR (both paddings), SimplePFOR and FastPFOR pages in
    the paper's own layout on the 2^28 patched list."""
    import torch
    import paper_1209_2137_amd as wp
    from paper_1209_2137_amd import datagen
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wp.lib()
    res = {}
    cluster = datagen.cluster_sorted(1 << 26, seed=2)
    for name, codec in (("bp_encode_cluster_2e26", wp.CODEC_BP), ("bpv_encode_cluster_2e26", wp.CODEC_BPV),
                        ("bp32_encode_cluster_2e26", wp.CODEC_BP32)):
        r = bench_encode(wp, cluster, codec, 1, steps, 1, name)
        res[name] = {"event_ms": r["event_ms"], "alg_bytes": r["alg_bytes"], "bits_per_int": r["bits_per_int"]}
    del cluster
    patched = datagen.patched_gaps(1 << 28, seed=4)
    for name, codec in (("fp_encode_patched_2e28", wp.CODEC_FP), ("fp32_encode_patched_2e28", wp.CODEC_FP32),
                        ("sp_encode_patched_2e28", wp.CODEC_SP), ("fpi_encode_patched_2e28", wp.CODEC_FPI)):
        r = bench_encode(wp, patched, codec, 1, steps, 1, name)
        res[name] = {"event_ms": r["event_ms"], "alg_bytes": r["alg_bytes"], "bits_per_int": r["bits_per_int"]}
        torch.cuda.synchronize()
    print(json.dumps(res))
    return 0


def profile_run(steps, inputs=None):
    """For rocprofv3: the headline decode, the 2^28 patched decode, the
    2^28 in-place delta decode and the batched posting-list decode `steps`
    times each (after their warm-ups), then a 1 GiB device copy `steps`
    times (the counter calibration). With `inputs` (a directory written by
    --prepare-inputs) the streams are loaded instead of encoded here."""
    import numpy as np
    import torch
    import paper_1209_2137_amd as wp
    from paper_1209_2137_amd import datagen
    from paper_1209_2137_amd.pool import ListPool
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wp.lib()

    def single(name, make, codec, label):
        if inputs is None:
            return bench_single(wp, make(), codec, 1, steps, 2, label)
        comp = torch.from_numpy(np.load(os.path.join(inputs, name + ".npy"))).to("cuda")
        n = int(np.load(os.path.join(inputs, name + ".n.npy"))[0])
        return bench_single(wp, None, codec, 1, steps, 2, label, comp=comp, n=n)

    r = single("bp_cluster_2e26", lambda: datagen.cluster_sorted(1 << 26, seed=2), wp.CODEC_BP, "bp cluster 2^26")
    f = single("fp_patched_2e28", lambda: datagen.patched_gaps(1 << 28, seed=4), wp.CODEC_FP,
               "fastpfor patched 2^28")
    d = bench_delta(wp, 1 << 28, steps, 2)
    if inputs is None:
        pool = posting_pool(False)
    else:
        pool = ListPool.from_streams(np.load(os.path.join(inputs, "pool_words.npy")),
                                     np.load(os.path.join(inputs, "pool_rows.npy")))
    b = profile_batch(wp, steps, pool)
    del pool
    c = bench_copy(1 << 30, steps, 0)
    torch.cuda.synchronize()
    print(json.dumps({"decode_kernel_ms": r["kernel_ms"], "decode_alg_bytes": r["alg_bytes"],
                      "fp_kernel_ms": f["kernel_ms"], "fp_alg_bytes": f["alg_bytes"],
                      "delta_kernel_ms": d["kernel_ms"], "delta_alg_bytes": 8 * (1 << 28),
                      "batch_ms": b["ms"], "batch_alg_bytes": b["alg_bytes"], "batch_n": b["n"],
                      "copy_bytes_each_way": 1 << 30, "copy_kernel_ms": c["kernel_ms"],
                      "kernel_hash": kernel_hash()}))
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and serving legs")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving run (the stated workload: 60 s)")
    ap.add_argument("--rocprof-summary", metavar="DIR")
    ap.add_argument("--profile-run", action="store_true",
                    help="for rocprofv3: the headline decode, the 2^28 patched decode, the 2^28 "
                         "in-place delta decode and the batched posting-list decode `--steps` times each, "
                         "then a 1 GiB device copy (the counter calibration kernel) `--steps` times")
    ap.add_argument("--profile-variants", action="store_true",
                    help="for rocprofv3: the BP32, four-lane SIMD-BP128 and FastPFOR-32 decoders (needs --inputs)")
    ap.add_argument("--profile-encoders", action="store_true",
                    help="for rocprofv3 kernel traces: every encoder on its bench workload `--steps` times")
    ap.add_argument("--inputs", metavar="DIR",
                    help="with --profile-run / --profile-variants: load the streams saved by --prepare-inputs")
    ap.add_argument("--prepare-inputs", metavar="DIR",
                    help="encode the profiled workloads and save their streams in DIR (run it without the profiler)")
    args = ap.parse_args()
    if args.rocprof_summary:
        rocprof_summary(args.rocprof_summary)
        return 0
    if args.prepare_inputs:
        return prepare_inputs(args.prepare_inputs)
    if args.profile_run:
        return profile_run(args.steps, args.inputs)
    if args.profile_encoders:
        return profile_encoders(args.steps)
    if args.profile_variants:
        if not args.inputs:
            print("--profile-variants needs --inputs DIR (from --prepare-inputs)", file=sys.stderr)
            return 2
        return profile_variants(args.steps, args.inputs)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the library decodes on a "
              "single MI355X; lists and units would shard across GPUs without any exchange)",
              file=sys.stderr)
        return 2
    import torch
    import paper_1209_2137_amd as wp
    from paper_1209_2137_amd import datagen
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wp.lib()
    t_start = time.perf_counter()
    x = datagen.cluster_sorted(1 << 26, seed=2)
    head = bench_single(wp, x, wp.CODEC_BP, 1, args.steps, args.warmup, "bp cluster 2^26")
    print(f"# headline done: {head['gints_per_s']:.1f} G ints/s ({time.perf_counter() - t_start:.0f} s)",
          file=sys.stderr, flush=True)
    extra = {}
    if not args.quick:
        copy = bench_copy(1 << 30, 10, 3)
        extra["copy_1GiB_gbs"] = copy["gbs"]
        u = bench_single(wp, datagen.uniform_sorted(1 << 26, seed=3), wp.CODEC_BP, 1, args.steps, args.warmup,
                         "bp uniform 2^26")
        extra["bp_uniform_2e26"] = u
        print("# uniform done", file=sys.stderr, flush=True)
        p = bench_single(wp, datagen.patched_gaps(1 << 28, seed=4), wp.CODEC_FP, 1, args.steps, args.warmup,
                         "fastpfor patched 2^28")
        extra["fp_patched_2e28"] = p
        extra["fp32_patched_2e28"] = bench_single(wp, datagen.patched_gaps(1 << 28, seed=4), wp.CODEC_FP32, 1,
                                                  args.steps, args.warmup, "fastpfor (arrays padded to 32) 2^28")
        extra["sp_patched_2e28"] = bench_single(wp, datagen.patched_gaps(1 << 28, seed=4), wp.CODEC_SP, 1,
                                                args.steps, args.warmup, "simplepfor (Simple-8b high parts) 2^28")
        extra["fpi_patched_2e28"] = bench_single(wp, datagen.patched_gaps(1 << 28, seed=4), wp.CODEC_FPI, 1,
                                                 max(3, args.steps // 4), 2,
                                                 "fastpfor pages in the paper's own layout 2^28")
        print("# patched done", file=sys.stderr, flush=True)
        extra["delta_inplace_2e28"] = bench_delta(wp, 1 << 28, args.steps, args.warmup)
        print("# delta done", file=sys.stderr, flush=True)
        extra["bp_encode_cluster_2e26"] = bench_encode(wp, x, wp.CODEC_BP, 1, args.steps, args.warmup,
                                                       "bp_encode cluster 2^26")
        extra["fp_encode_patched_2e28"] = bench_encode(wp, datagen.patched_gaps(1 << 28, seed=4), wp.CODEC_FP, 1,
                                                       args.steps, args.warmup, "fastpfor_encode patched 2^28")
        extra["bp32_cluster_2e26"] = bench_single(wp, x, wp.CODEC_BP32, 1, args.steps, args.warmup,
                                                  "bp32 cluster 2^26")
        extra["bpv_cluster_2e26"] = bench_single(wp, x, wp.CODEC_BPV, 1, args.steps, args.warmup,
                                                 "simd-bp128 four-lane layout cluster 2^26")
        extra["bpv_cluster_2e26_stride4"] = bench_single(wp, x, wp.CODEC_BPV, 4, args.steps, args.warmup,
                                                         "simd-bp128 four-lane layout, stride-4 deltas, cluster 2^26")
        extra["bp32_encode_cluster_2e26"] = bench_encode(wp, x, wp.CODEC_BP32, 1, args.steps, args.warmup,
                                                         "bp32_encode cluster 2^26")
        extra["sp_encode_patched_2e28"] = bench_encode(wp, datagen.patched_gaps(1 << 28, seed=4), wp.CODEC_SP, 1,
                                                       max(3, args.steps // 4), 1, "simplepfor_encode patched 2^28")
        print("# encoders done", file=sys.stderr, flush=True)
        extra["intersect_2e20_2e24"] = bench_intersect(wp, args.steps, args.warmup)
        print("# intersection done", file=sys.stderr, flush=True)
        extra["intersect_compressed_2e24"] = bench_intersect_compressed(wp, args.steps, args.warmup)
        print("# compressed intersection done", file=sys.stderr, flush=True)
        extra["decode_range_cluster_2e26"] = bench_decode_range(wp, x, args.steps, args.warmup)
        print("# key-range decoding done", file=sys.stderr, flush=True)
        head["pct_of_copy"] = head["achieved_gbs"] / copy["gbs"]
        if not args.no_batch:
            extra["batched_posting_lists"], pool = bench_batch(wp, max(3, args.steps // 2), 2)
            print("# batched done", file=sys.stderr, flush=True)
            if args.serve_seconds > 0:
                extra["serving"] = bench_serve(wp, pool, seconds=args.serve_seconds)
                print("# serving done", file=sys.stderr, flush=True)
            del pool
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(x)
        print("# cpu baseline done", file=sys.stderr, flush=True)
    traffic = measured_traffic(head["alg_bytes"])
    line = {
        "metric": METRIC,
        "value": head["gints_per_s"],
        "unit": "G ints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "SIMD-BP128 single list: 2^26 sorted distinct uint32, recursive-cluster generator in "
                        "[0,2^30) (depth 20, leaves <= 64), binary packing 16x128 per meta-block, stride-1 "
                        "differential decode",
            "n": head["n"], "bits_per_int": round(head["bits_per_int"], 4),
            "decode_tune": wp_tune_of(),
            "input_replicas": head["replicas"],
        },
        "roofline": {
            "bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": head["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": head["alg_bytes"], "kernel_ms": head["kernel_ms"],
        },
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))
    return 0


def wp_tune_of():
    from paper_1209_2137_amd.autotune import arch, load
    return load().get(arch(), {}).get("bp_single")


if __name__ == "__main__":
    sys.exit(main())
