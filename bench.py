#!/usr/bin/env python
"""Benchmark of the hsort hot path on one MI355X.

Workload (the headline metric): n = 2^28 int32 keys uniform in [0, 2^31-1),
keys only, sorted by the full method (one-step decimal MSD partition -- ten
buckets, or the finer one hundred or one thousand the tuning table picks --,
LDS tile sort of each bucket's partitions, merge-path merge rounds).
A step is one complete sort of one resident copy of that array; every step
sorts its own pristine copy, all copies in HBM before the timed region.

Prints ONE JSON line on stdout:
  value      Gkeys/s over the K timed steps (n * K / elapsed)
  roofline   the dominant kernel's algorithmic bytes per launch / its average
             launch time (HIP events on the sorting stream, recorded in a
             separate run of up to five sorts so that the timed steps carry no
             per-kernel events) vs 8 TB/s HBM peak
  cpu_baseline  the CPU oracle (single-threaded) on the metric's own input,
             once; extra.cpu_openmp_hybrid is the paper's method with OpenMP
             on all host cores, same input
  extra      per-kernel table and the other workloads (2^20 keys eager and
             graph-replayed, stable pairs with heavy duplicates, skewed keys,
             int64 keys, batched segmented vs a per-array loop of the plain
             method, eager and graph-captured, and the serving loop)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

import workloads as W

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_RECORD = os.path.join(HERE, "profiles", "sort_i32_2e28_hbm_bytes.md")
KERNEL_SOURCES = ["hs_kernels.hip", "hs_device.h", "hs_io.h", "hs_work.h", "hs_launch.h"]


def kernel_sources_sha256():
    """Hash of the device sources the kernels are compiled from."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_2003_01216_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per dispatch of the dominant kernel from the committed FETCH_SIZE/WRITE_SIZE record,
    or None when the kernel source changed since the counters were taken."""
    import re

    try:
        text = open(TRAFFIC_RECORD).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        sha = kernel_sources_sha256()
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("kernels_source_sha256") != sha:
        return None
    return rec["fetch_bytes_per_dispatch"] + rec["write_bytes_per_dispatch"]


def kernel_table(rec, steps):
    """{name: {launches, ms_per_launch, GB/s, frac}} from hsort_timing_read()."""
    out = {}
    for name, (launches, ms, by) in rec.items():
        d = {"launches_per_step": launches / steps, "ms_per_step": ms / steps,
             "avg_ms_per_launch": ms / max(launches, 1)}
        if by > 0 and ms > 0:
            gbs = by / (ms * 1e-3) / 1e9
            d["GBps"] = round(gbs, 1)
            d["frac_hbm_peak"] = round(gbs / HBM_PEAK_GBS, 4)
            d["bytes_per_launch"] = by / launches
        out[name] = d
    return out


def timed_sorts(hs, torch, make_copies, run_one, steps, warmup, timing=True):
    """Run `warmup` untimed then `steps` timed calls, each on its own copy."""
    copies = make_copies(steps + warmup)
    for i in range(warmup):
        run_one(copies[i])
    torch.cuda.synchronize()
    hs.hsort_timing_read()  # drop warm-up records
    hs.hsort_timing_enable(timing)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for i in range(steps):
        run_one(copies[warmup + i])
    b.record()
    torch.cuda.synchronize()
    hs.hsort_timing_enable(False)
    rec = hs.hsort_timing_read()
    return a.elapsed_time(b), rec, copies


def rate_then_records(hs, torch, make_copies, run_one, steps, warmup, rec_steps=3):
    """Time `steps` calls with the per-kernel event records off (they add
    about twenty event records per call to the timed window), then take the
    records from a short second run on fresh copies: (ms, records, their
    number of calls)."""
    ms, _, copies = timed_sorts(hs, torch, make_copies, run_one, steps, warmup, timing=False)
    del copies
    rec_steps = min(rec_steps, steps)
    _, rec, copies = timed_sorts(hs, torch, make_copies, run_one, rec_steps, 1)
    del copies
    torch.cuda.empty_cache()
    return ms, rec, rec_steps


def bench_metric(hs, torch, n, steps, warmup):
    k = W.uniform_i32(n, 0)
    base = torch.from_numpy(k).cuda()
    scratch = torch.empty(hs.scratch_bytes(hs.KEYS_I32, n), dtype=torch.uint8, device="cuda")

    def make(m):
        return [base.clone() for _ in range(m)]

    # the timed steps run with the per-kernel event records off (they would
    # add ~20 event records per sort to the timed region); the records come
    # from a second, shorter run on fresh copies
    ms, _, copies = timed_sorts(hs, torch, make, lambda t: hs.hsort_keys(t, scratch), steps, warmup, timing=False)
    last = copies[-1]
    ok = bool(torch.all(last[1:] >= last[:-1]).item()) and int(last.to(torch.int64).sum()) == int(k.astype(np.int64).sum())
    out = last.cpu().numpy()
    del copies, last
    torch.cuda.empty_cache()
    rec_steps = min(steps, 5)
    _, rec, copies = timed_sorts(hs, torch, make, lambda t: hs.hsort_keys(t, scratch), rec_steps, 1)
    del copies
    torch.cuda.empty_cache()
    return ms, rec, rec_steps, ok, k, out


def bench_pairs(hs, torch, n, steps, warmup):
    k, v = W.dup_pairs_i32(n, 0)
    bk, bv = torch.from_numpy(k).cuda(), torch.from_numpy(v.view(np.int32)).cuda()
    scratch = torch.empty(hs.scratch_bytes(hs.PAIRS_I32_U32, n), dtype=torch.uint8, device="cuda")

    def make(m):
        return [(bk.clone(), bv.clone()) for _ in range(m)]

    ms, rec, rs = rate_then_records(hs, torch, make, lambda kv: hs.hsort_pairs(kv[0], kv[1], scratch), steps, warmup)
    return n * steps / (ms * 1e-3) / 1e9, kernel_table(rec, rs)


def bench_keys(hs, torch, k, steps, warmup):
    base = torch.from_numpy(k).cuda()
    kind = hs.KEYS_I32 if k.dtype == np.int32 else hs.KEYS_I64
    scratch = torch.empty(hs.scratch_bytes(kind, k.size), dtype=torch.uint8, device="cuda")
    ms, rec, rs = rate_then_records(hs, torch, lambda m: [base.clone() for _ in range(m)],
                                    lambda t: hs.hsort_keys(t, scratch), steps, warmup)
    return k.size * steps / (ms * 1e-3) / 1e9, kernel_table(rec, rs)


def bench_typed(hs, torch, k, vals, desc, steps, warmup):
    """hsort_sort on keys of any supported dtype (bits moved as a signed tensor of the same width)."""
    kt = {np.dtype(np.int32): hs.I32, np.dtype(np.uint32): hs.U32, np.dtype(np.float32): hs.F32,
          np.dtype(np.int64): hs.I64, np.dtype(np.uint64): hs.U64, np.dtype(np.float64): hs.F64}[k.dtype]
    base = torch.from_numpy(k.view(np.int32 if k.dtype.itemsize == 4 else np.int64)).cuda()
    bv = None if vals is None else torch.from_numpy(vals.view(np.int32)).cuda()
    scratch = torch.empty(hs.sort_scratch_bytes(kt, vals is not None, k.size), dtype=torch.uint8, device="cuda")

    def make(m):
        return [(base.clone(), None if bv is None else bv.clone()) for _ in range(m)]

    ms, rec, rs = rate_then_records(
        hs, torch, make, lambda kv: hs.hsort_sort(kv[0], kv[1], descending=desc, key_type=kt, scratch=scratch),
        steps, warmup)
    return round(k.size * steps / (ms * 1e-3) / 1e9, 3), kernel_table(rec, rs)


def bench_small_keys(hs, torch, n, steps=50, warmup=5):
    """n uniform int32 keys (seed 0): per-call time of the plain sort, eager and replayed from a hipGraph,
    refilling the same buffer from a resident copy outside the timed window before every call."""
    base = torch.from_numpy(W.uniform_i32(n, 0)).cuda()
    scratch = torch.empty(hs.scratch_bytes(hs.KEYS_I32, n), dtype=torch.uint8, device="cuda")
    out = {"workload": f"sort 2^{int(np.log2(n))} int32 keys uniform in [0, 2^31-1), keys only, seed 0"}
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ms_eager, _ = timed_refill(torch, base, lambda t: hs.hsort_keys(t, scratch), steps, warmup)
        hs.hsort_graph_mode(True)
        try:
            ms_graph, _ = timed_refill(torch, base, lambda t: hs.hsort_keys(t, scratch), steps, warmup)
        finally:
            hs.hsort_graph_mode(False)
            hs.hsort_graph_clear()
    out.update({"eager_ms": round(ms_eager, 4), "eager_Gkeys_s": round(n / ms_eager / 1e6, 3),
                "graph_ms": round(ms_graph, 4), "graph_Gkeys_s": round(n / ms_graph / 1e6, 3)})
    return out


def timed_refill(torch, base, run_one, steps, warmup):
    """Per-call event times of `run_one(work)`, refilling `work` from `base`
    outside the timed window each time (same buffers on every call)."""
    work = base.clone()
    total = 0.0
    for i in range(warmup + steps):
        work.copy_(base)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        run_one(work)
        b.record()
        torch.cuda.synchronize()
        if i >= warmup:
            total += a.elapsed_time(b)
    return total / steps, work


def bench_segmented(hs, torch, steps, warmup, loop=True):
    """16384 arrays, log-uniform sizes in [1, 2^16]: one batched call vs a loop of plain calls
    (the loop is skipped when `loop` is false)."""
    keys, off = W.segments_i32(16384, 2**16, 0)
    n = keys.size
    max_len = int(np.diff(off).max())
    side = torch.cuda.Stream()
    out = {"workload": "16384 int32 arrays, sizes log-uniform [1, 2^16], keys uniform [0, 2^31-1)", "keys": int(n)}
    with torch.cuda.stream(side):
        base = torch.from_numpy(keys).cuda()
        doff = torch.from_numpy(off).cuda()
        scratch = torch.empty(hs.scratch_bytes(hs.SEG_I32, n, 16384), dtype=torch.uint8, device="cuda")

        def batched(t):
            hs.hsort_segmented(t, doff, max_seg_len=max_len, scratch=scratch)

        ms_eager, _ = timed_refill(torch, base, batched, steps, warmup)
        hs.hsort_graph_mode(True)
        try:
            hs.hsort_timing_read()
            ms_graph, work = timed_refill(torch, base, batched, steps, warmup)
        finally:
            hs.hsort_graph_mode(False)
        # the kernels of one batched call, timed separately (eager, per-kernel events)
        hs.hsort_timing_enable(True)
        w2 = base.clone()
        batched(w2)
        torch.cuda.synchronize()
        hs.hsort_timing_enable(False)
        kernels = kernel_table(hs.hsort_timing_read(), 1)
        out.update({"batched_graph_Gkeys_s": round(n / ms_graph / 1e6, 3),
                    "batched_eager_Gkeys_s": round(n / ms_eager / 1e6, 3), "batched_graph_ms": round(ms_graph, 4),
                    "batched_kernels": kernels})
        if not loop:
            torch.cuda.empty_cache()
            return out
        # per-array loop of the plain method on sub-views, same stream, one scratch
        loop_scratch = torch.empty(hs.scratch_bytes(hs.KEYS_I32, max_len), dtype=torch.uint8, device="cuda")
        offs = off.tolist()

        def loop(t):
            for i in range(16384):
                a, b = offs[i], offs[i + 1]
                if b > a:
                    hs.hsort_keys(t[a:b], loop_scratch)

        loop(base.clone())  # warm-up
        torch.cuda.synchronize()
        lw = base.clone()
        t0 = time.perf_counter()
        loop(lw)
        torch.cuda.synchronize()
        loop_s = time.perf_counter() - t0
        same = bool(torch.equal(lw, work))  # loop and batched agree
        # the same loop captured once into one graph on the side stream and
        # replayed: no host launch cost per call, the fair comparison
        lw.copy_(base)
        side.synchronize()
        g = torch.cuda.CUDAGraph()
        t0 = time.perf_counter()
        with torch.cuda.graph(g, stream=side):
            loop(lw)
        capture_s = time.perf_counter() - t0
        loop_graph = []
        for i in range(4):
            lw.copy_(base)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            g.replay()
            b.record()
            torch.cuda.synchronize()
            if i:
                loop_graph.append(a.elapsed_time(b))
        same_graph = bool(torch.equal(lw, work))
        del g
    torch.cuda.empty_cache()
    loop_graph_ms = float(np.median(loop_graph))
    out.update({"per_array_loop_Gkeys_s": round(n / loop_s / 1e9, 4), "per_array_loop_ms": round(loop_s * 1e3, 2),
                "speedup_graph_vs_loop": round(loop_s * 1e3 / ms_graph, 1), "loop_equals_batched": same,
                "per_array_loop_graph_Gkeys_s": round(n / loop_graph_ms / 1e6, 4),
                "per_array_loop_graph_ms": round(loop_graph_ms, 3),
                "per_array_loop_graph_capture_s": round(capture_s, 2),
                "speedup_graph_vs_loop_graph": round(loop_graph_ms / ms_graph, 1),
                "loop_graph_equals_batched": same_graph})
    return out


def bench_serving(count=1000, budget=64 << 30, small_budget=384 << 20, streams=3, load=0.7):
    """Poisson stream of int64 sort requests (sizes log-uniform in [2^10, 2^24], keys over the full int64
    range) through the continuous-batching server with a 64 GiB HBM budget.  The arrival rate is `load` times
    the saturation rate measured first with every request submitted at once.  The same arrivals are then
    replayed against a 384 MiB budget (the largest request needs 270 MiB with its scratch), under which two
    large requests cannot be in flight together and admission has to wait for memory."""
    import threading

    import paper_2003_01216_amd.serve as serve

    sizes = W.request_sizes(count, 2**10, 2**24, seed=0)
    info = np.iinfo(np.int64)
    reqs = [np.random.default_rng((0, i)).integers(info.min, info.max, int(s), dtype=np.int64, endpoint=True)
            for i, s in enumerate(sizes)]
    with serve.SortServer(hbm_budget=budget, streams=streams) as srv:  # warm-up
        for f in [srv.submit(r) for r in reqs[:8]]:
            f.result()
    with serve.SortServer(hbm_budget=budget, streams=streams) as srv:
        futs = [srv.submit(r) for r in reqs]
        for f in futs:
            f.result()
        sat = srv.stats()
    rate = load * count / sat["wall_s"]
    gaps = np.random.default_rng(1).exponential(1.0 / rate, count)

    def poisson_run(bud):
        with serve.SortServer(hbm_budget=bud, streams=streams) as srv:
            futs = []

            def client():
                for r, g in zip(reqs, gaps):
                    time.sleep(g)
                    futs.append(srv.submit(r))

            th = threading.Thread(target=client)
            th.start()
            th.join()
            outs = [f.result() for f in futs]
            st = srv.stats()
        ok = all(bool(np.all(o[1:] >= o[:-1])) for o in outs[:: max(1, count // 20)])
        return {"budget_bytes": bud, "Gkeys_s": round(st["Gkeys_s"], 3), "p50_ms": round(st["p50_ms"], 3),
                "p99_ms": round(st["p99_ms"], 3), "mean_batch_requests": round(st["mean_batch_requests"], 2),
                "batches": st["batches"], "overlap_s": round(st["overlap_s"], 3),
                "peak_in_flight_bytes": st["peak_in_flight_bytes"], "budget_waits": st["budget_waits"],
                "sorted_check": ok}

    full = poisson_run(budget)
    small = poisson_run(small_budget)
    out = {"workload": f"{count} int64 requests, sizes log-uniform [2^10, 2^24], keys full int64 range, "
                       "Poisson arrivals", "streams": streams, "saturation_Gkeys_s": round(sat["Gkeys_s"], 3),
           "saturation_requests_s": round(count / sat["wall_s"], 1), "rate_requests_s": round(rate, 1)}
    out.update(full)
    out["reduced_budget"] = small
    out["note"] = "end to end: host arrays in, host arrays out (PCIe copies included)"
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baselines(k, gpu_out):
    """The oracle (single-threaded C) on the metric's own input, once, and the paper's method on all host
    cores (OpenMP: one-step ten-bucket partition, per-thread quicksort, merge rounds) on the same input."""
    import oracle

    n = k.size
    host_cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref = oracle.sort_keys(k)
    dt = time.perf_counter() - t0
    base = {"value": round(n / dt / 1e9, 5), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": f"the metric's input itself (2^{int(np.log2(n))} int32 keys uniform in [0, 2^31-1), seed 0), "
                      f"sorted once in {dt:.1f} s",
            "cpu_model": cpu_model(), "host_cores": host_cores,
            "equals_gpu_output": bool(np.array_equal(ref, gpu_out)) if gpu_out is not None else None}
    del ref
    t0 = time.perf_counter()
    out, used = oracle.omp_hybrid_sort(k, host_cores)
    dt = time.perf_counter() - t0
    omp = {"value": round(n / dt / 1e9, 5), "unit": "Gkeys/s", "cores": used,
           "kind": "the paper's method on the host (OpenMP, Sections 3.2-3.4)",
           "sample": f"the metric's input, sorted once in {dt:.2f} s", "cpu_model": base["cpu_model"],
           "equals_gpu_output": bool(np.array_equal(out, gpu_out)) if gpu_out is not None else None}
    return base, omp


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28, help="keys in the metric workload (2^log2n)")
    ap.add_argument("--no-extras", action="store_true", help="only the metric workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--extras", default="small,pairs,keys,typed,segmented,serving",
                    help="comma list of the extra workloads to run: small, pairs, keys, typed, segmented, serving")
    ap.add_argument("--no-loop", action="store_true", help="segmented: skip the per-array loop of plain calls")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the sort runs on one GPU (no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    extras = set() if args.no_extras else {e.strip() for e in args.extras.split(",") if e.strip()}
    unknown = extras - {"small", "pairs", "keys", "typed", "segmented", "serving"}
    if unknown:
        print(f"bench.py: unknown extra workloads {sorted(unknown)} "
              "(choose from small, pairs, keys, typed, segmented, serving)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2003_01216_amd as hs

    hs.load_library()
    n = 1 << args.log2n
    log(f"[bench] metric workload: 2^{args.log2n} int32 uniform keys, {args.steps} steps, {args.warmup} warm-up")
    ms, rec, rec_steps, ok, metric_in, metric_out = bench_metric(hs, torch, n, args.steps, args.warmup)
    if not ok:
        log("[bench] ERROR: output of the last step is not sorted")
        sys.exit(1)
    # plain copy through the library's copy kernel: the practical streaming ceiling, and the
    # reference a byte-counter profile of this same command is scaled by
    cb = 1 << 30
    src = torch.empty(cb, dtype=torch.uint8, device="cuda")
    dst = torch.empty(cb, dtype=torch.uint8, device="cuda")
    hs.hsort_copy(src, dst)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        hs.hsort_copy(src, dst)
    b.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * cb / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    ms_step = ms / args.steps
    value = n / (ms_step * 1e-3) / 1e9
    table = kernel_table(rec, rec_steps)
    log(f"[bench] {value:.2f} Gkeys/s, {ms_step:.3f} ms/step")
    for name, d in table.items():
        log(f"[bench]   {name:10s} {d['ms_per_step']:.3f} ms/step  {d.get('GBps', '-')} GB/s")
    dom = max((kv for kv in table.items() if "GBps" in kv[1]), key=lambda kv: kv[1]["ms_per_step"])
    traffic = measured_traffic() if dom[0] == "merge" else None
    roof = {"bound": "hbm", "kernel": dom[0], "achieved": dom[1]["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dom[1]["GBps"] / HBM_PEAK_GBS, 4),
            "traffic": round(traffic / 1e9, 4) if traffic else None,
            "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_GB_per_launch": round(dom[1]["bytes_per_launch"] / 1e9, 4)}
    total_bytes = sum(d.get("bytes_per_launch", 0) * d["launches_per_step"] for d in table.values())
    extra = {"kernels": table, "copy_kernel_GBps": round(copy_gbps, 1),
             "algorithmic_bytes_per_key": round(total_bytes / n, 2),
             "whole_sort_frac_hbm_peak": round(total_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    if "small" in extras:
        log("[bench] 2^20 uniform int32 (eager and graph replay)")
        extra["uniform_2e20"] = bench_small_keys(hs, torch, 2**20)
    if "pairs" in extras:
        log("[bench] stable pairs 2^28, keys in [0,1000), payload = index")
        extra["pairs_dup_2e28_Gkeys_s"], extra["pairs_kernels"] = bench_pairs(hs, torch, 2**28, 5, 1)
    if "keys" in extras:
        log("[bench] 2^26 uniform / log-uniform / int64 full range")
        extra["uniform_2e26_Gkeys_s"] = round(bench_keys(hs, torch, W.uniform_i32(2**26, 0), 10, 2)[0], 3)
        extra["loguniform_2e26_Gkeys_s"] = round(bench_keys(hs, torch, W.loguniform_i32(2**26, 0), 10, 2)[0], 3)
        extra["int64_full_range_2e26_Gkeys_s"] = round(bench_keys(hs, torch, W.uniform_i64(2**26, 0), 10, 2)[0], 3)
    if "typed" in extras:
        log("[bench] other key types: float32 2^28, int32 descending 2^28, int64 + payload 2^26")
        r = np.random.default_rng(0)
        f32 = (r.standard_normal(2**28, dtype=np.float32) * np.float32(1e3))
        extra["float32_2e28_Gkeys_s"], _ = bench_typed(hs, torch, f32, None, False, 5, 1)
        del f32
        extra["int32_descending_2e28_Gkeys_s"], _ = bench_typed(hs, torch, W.uniform_i32(2**28, 0), None, True, 5, 1)
        k64 = W.uniform_i64(2**26, 0)
        extra["int64_pairs_2e26_Gkeys_s"], extra["int64_pairs_kernels"] = bench_typed(
            hs, torch, k64, np.arange(2**26, dtype=np.uint32), False, 5, 1)
    if "segmented" in extras:
        log("[bench] batched segmented" + ("" if args.no_loop else " vs per-array loop"))
        extra["segmented"] = bench_segmented(hs, torch, 10, 2, loop=not args.no_loop)
    if "serving" in extras:
        log("[bench] serving loop")
        extra["serving"] = bench_serving()

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU baselines: the oracle on one core, the OpenMP hybrid on all cores")
        cpu, extra["cpu_openmp_hybrid"] = cpu_baselines(metric_in, metric_out)

    line = {
        "metric": "Gkeys/s + % HBM peak, int32 n=2^28; batched segmented vs per-array plain",
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"sort 2^{args.log2n} int32 keys uniform in [0, 2^31-1), keys only, seed 0",
                   "n": n, "parallelism": "one GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
