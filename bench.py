#!/usr/bin/env python3
"""Benchmark of the set-intersection hot path on one MI355X.

A step is one full counting pass over the resident trie of the workload:
one launch of the counting kernel (eh_count_add_async), which reads every
neighbour-set intersection of Generic-Join once.  The trie is built and
uploaded before timing (index creation is excluded from the paper's timings,
section 5.1), so inputs are resident in HBM when the timed region starts.

Prints one JSON line.  Workloads (--workload):
  rmat20_triangles  (default) R-MAT scale 20, edge factor 16, a,b,c,d =
                    .57/.19/.19/.05, hybrid layout: edges/s of triangle counting
  rmat18_4cliques   R-MAT scale 18, 4-clique counting
  er4096_triangles  G(n=4096, M=32768), uint-only layout
  batch_triangles   20,000 Chung-Lu graphs counted in one launch, beside one
                    launch per graph
  orderings         node orderings of appendix A on Chung-Lu graphs (n = 2^20,
                    degree exponents 1.75 .. 3): triangle counting per ordering
  build             trie construction on the host and on the GPU, R-MAT scales
                    20 and 22, with the first (planning) and a repeated count
  ablation          R-MAT scale 20 with layout / algorithm choices switched off
  unpruned          R-MAT scale 20 with both directions of every edge: ordered
                    triangles and the Lollipop query, beside pruned triangles
  composite         set layouts at relation, set and block level: pairs of sets
                    with a shared dense region, and R-MAT s20 triangles as
                    pairwise intersections per layout
  served            resident R-MAT scale 22, Poisson stream of rooted
                    triangle / 4-clique requests: p50/p99 latency
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "edges/s triangle count (plain vs batched); HBM GB/s; p50/p99 query latency"
HBM_PEAK_GBS = 8000.0
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4  # vector lane operations per ns: CUs x SIMDs x lanes x GHz
TUNING_FILE = os.path.join(ROOT, "paper_1503_02368_amd", "tuning.json")

from paper_1503_02368_amd.profile_summary import measured_traffic, valu_issue  # noqa: E402
from paper_1503_02368_amd.workloads import WORKLOADS, make_graph  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_tuning(name: str) -> dict:
    """The autotuner's choice for this workload: {layout, tau, tuning}, or {}."""
    if os.path.exists(TUNING_FILE):
        with open(TUNING_FILE) as f:
            return json.load(f).get(name, {})
    return {}


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def one_thread_rate(fn, n: int, budget_s: float) -> dict:
    """The oracle on one thread: the whole workload if it fits the budget,
    else the prefix of outer vertices that does (rate = edges visited / s)."""
    t0 = time.perf_counter()
    fn(threads=1, x_begin=0, x_end=max(1, n // 256))
    est = (time.perf_counter() - t0) * 256
    x_end = n if est <= budget_s else max(1, int(n * budget_s / est))
    t0 = time.perf_counter()
    res = fn(threads=1, x_begin=0, x_end=x_end)
    t = time.perf_counter() - t0
    return {"value": res["edges"] / t, "unit": "edges/s", "cores": 1,
            "sample": "whole workload" if x_end == n else
                      f"outer vertices of rank < {x_end} ({res['edges']} oriented edges)",
            "seconds": t}


def cpu_baseline(el, pattern: int, budget_s: float = 20.0) -> dict:
    """The oracle, as it stands, on this host's cores; full workload if it fits
    the time budget, else a prefix of outer vertices scaled by edges visited."""
    import oracle
    g = oracle.Graph.from_edgelist(el)
    threads = oracle.max_threads()
    fn = g.triangles if pattern == 3 else g.cliques4
    # probe on a small prefix of outer vertices to size the sample
    t0 = time.perf_counter()
    probe = fn(threads=threads, x_begin=0, x_end=max(1, g.n // 64))
    dt = time.perf_counter() - t0
    est_full = dt * 64
    if est_full <= budget_s / 3:
        times = []
        res = None
        for _ in range(3):
            t0 = time.perf_counter()
            res = fn(threads=threads)
            times.append(time.perf_counter() - t0)
        t = statistics.median(times)
        return {"value": res["edges"] / t, "unit": "edges/s", "cores": threads, "kind": "oracle",
                "sample": f"whole workload, median of 3 runs ({t:.3f} s each)", "count": res["count"],
                "bytes": res["bytes"], "held_bytes": res.get("held_bytes"),
                "held_tests": res.get("held_tests"),
                "one_thread": one_thread_rate(fn, g.n, budget_s / 2),
                **cpu_info()}
    frac = max(1.0 / 64, min(1.0, (budget_s / 2) / max(est_full, 1e-9)))
    x_end = max(1, int(g.n * frac))
    t0 = time.perf_counter()
    res = fn(threads=threads, x_begin=0, x_end=x_end)
    t = time.perf_counter() - t0
    del probe
    return {"value": res["edges"] / t, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"outer vertices of rank < {x_end} ({res['edges']} of {g.m} oriented edges), "
                      f"{t:.2f} s", "count": None, "bytes": None,
            "one_thread": one_thread_rate(fn, g.n, budget_s / 2), **cpu_info()}


def bench_graph(name, w, args, ctx, eh, torch):
    el = make_graph(w)
    log(f"[bench] {name}: generated n={el.n} raw pairs={el.m_raw}")
    tune = load_tuning(name)
    layout = tune.get("layout", w["layout"])
    tau = tune.get("tau", w["tau"])
    if tune.get("tuning"):
        ctx.set_tuning(**tune["tuning"])
    t0 = time.perf_counter()
    s_min = tune.get("s_min", 1)
    trie = ctx.build_edgelist(el, layout=layout, tau=tau, s_min=s_min)
    t_build = time.perf_counter() - t0
    info = trie.info
    log(f"[bench] trie built in {t_build:.2f} s: {info}")
    pattern = w["pattern"]
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = ctx.stream
    s.wait_stream(torch.cuda.current_stream())
    # the process's first count also loads the planner's and kernels' code:
    # a count of a small graph with the same settings does that beforehand
    cold_ms = None
    if not args.no_code_warmup:
        from paper_1503_02368_amd import inputs
        small = ctx.build_edgelist(inputs.rmat(10, 16, seed=1), layout=layout, tau=tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.count_add_async(small, pattern, out)
        torch.cuda.synchronize()
        cold_ms = (time.perf_counter() - t0) * 1e3
        small.free()
    # the first count builds and caches the work-item plan (not timed below)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.count_add_async(trie, pattern, out)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    if cold_ms is None:
        log(f"[bench] first count (code loading, plan + count) {first_ms:.2f} ms")
    else:
        log(f"[bench] first count (plan + count) {first_ms:.2f} ms; the process's first count, of "
            f"a small graph, {cold_ms:.1f} ms (code loading)")
    for _ in range(args.warmup):
        ctx.count_add_async(trie, pattern, out)
    torch.cuda.synchronize()
    out.zero_()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s)
    for _ in range(args.steps):
        ctx.count_add_async(trie, pattern, out)
    ev1.record(s)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    total = int(out.cpu().numpy().view(np.uint64)[0])
    count, rem = divmod(total, args.steps)
    log(f"[bench] {args.steps} steps, {ms:.4f} ms/step, count {count}")
    if rem:
        raise RuntimeError("accumulated count is not a multiple of the step count")
    m_plus = info["m_plus"]
    result = {
        "metric": METRIC, "value": m_plus / (ms / 1e3), "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": name, **{k: v for k, v in w.items() if k not in ("kind",)},
                   "layout": ["uint", "hybrid", "bitset_all"][layout], "tau": tau, "s_min": s_min,
                   "n": info["n"], "m_plus": m_plus, "max_out_degree": info["max_out_degree"],
                   "bitset_sets": info["n_bitset_sets"], "tuning": ctx.get_tuning()},
        "count": count,
        "untimed": {"first_count_ms": first_ms, "process_first_count_ms": cold_ms,
                    "note": "first count = work-item planning (cached per trie, pattern and "
                            "tuning) plus one count, wall clock, "
                            + ("including the process's code loading (--no-code-warmup); "
                               if cold_ms is None else
                               "after a count of a small graph has loaded the code "
                               "(process_first_count_ms, that small count); ")
                            + f"trie build {t_build * 1e3:.0f} ms (host build and upload) also "
                            "untimed"},
    }
    cb = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle")
        cb = cpu_baseline(el, pattern, args.cpu_budget)
        if cb.get("count") is not None:
            result["parity_vs_oracle"] = cb["count"] == count
    tuning = ctx.get_tuning()
    target = (pattern == 3 and tuning["kernel"] != eh.KERNEL_PAIRWISE
              and tuning["staging"] != eh.STAGE_SOURCE and info["b_target"] > 0)
    # Algorithmic bytes per launch: what this design must read.  Triangles
    # with target staging: B_target from the trie (N+(v) once per held set,
    # the part of N+(u) above v once per in-edge, their descriptors).
    # 4-cliques: B_K4_held from the oracle's pass (N+(u) and S_uv held).
    # The list-merge figures (B_merge, B_K4: both sets of every intersection
    # read) are reported beside them as merge-equivalent rates.
    if pattern == 3:
        model, model_bytes = ("B_target", info["b_target"]) if target else ("B_merge", info["b_merge"])
        merge_bytes = info["b_merge"]
    else:
        model, model_bytes = "B_K4_held", (cb or {}).get("held_bytes")
        merge_bytes = (cb or {}).get("bytes")
        tests = (cb or {}).get("held_tests")
        if tests:
            # 4-cliques are not bound by HBM (the sets a launch reads stay in
            # L2 and the last-level cache), so the bound is the vector ALU:
            # the join's member tests against 256 CUs x 4 SIMDs x 16 lanes x
            # 2.4 GHz = 39.3 T lane operations per second.  The induced-
            # neighbourhood kernel makes the third level's tests as 32-bit
            # word ANDs, so this is an algorithmic rate, not an issue rate
            achieved = tests / (ms / 1e3) / 1e9
            result["roofline"] = {
                "bound": "alu", "achieved": achieved, "peak": ALU_PEAK_GOPS, "unit": "G tests/s",
                "frac": achieved / ALU_PEAK_GOPS, "traffic": measured_traffic(name),
                "traffic_kind": "L2-to-fabric bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                "copy-calibrated), summed over the launch's kernels",
                "model": "member tests of the join's intersections with N+(u) and S_uv held "
                         "(N+(v) against N+(u), N+(w) against S_uv)",
                "algorithmic_tests_per_launch": tests, "kernel_ms_per_launch": ms,
                "held_design_bytes_per_launch": model_bytes,
                "held_design_gbs": model_bytes / (ms / 1e3) / 1e9,
                "note": "the kernel tests the third level 32 members per lane operation (bitset "
                        "words over each root's local ids); per-kernel issue and residency "
                        "figures are in profiles/"}
            if merge_bytes:
                result["roofline"]["merge_equivalent"] = {
                    "model": "B_K4", "bytes_per_launch": merge_bytes,
                    "gbs": merge_bytes / (ms / 1e3) / 1e9}
            model_bytes = None
    if model_bytes:
        from paper_1503_02368_amd.calib import probe_gbs
        achieved = model_bytes / (ms / 1e3) / 1e9
        traffic = measured_traffic(name)
        probe = {"read": None, "kernel": None} if args.no_probe else probe_gbs(ctx)
        result["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_kind": "L2-to-fabric bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated); reads served by the 256 MB last-level cache are "
                            "included, so DRAM bytes are at most this",
            "model": model, "algorithmic_bytes_per_launch": model_bytes,
            "kernel_ms_per_launch": ms,
            "achievable_read_gbs": probe["read"], "achievable_read_kernel": probe["kernel"],
            "frac_of_achievable_read": achieved / probe["read"] if probe["read"] else None}
        if merge_bytes:
            result["roofline"]["merge_equivalent"] = {
                "model": "B_merge" if pattern == 3 else "B_K4", "bytes_per_launch": merge_bytes,
                "gbs": merge_bytes / (ms / 1e3) / 1e9,
                "note": "both sets of every intersection read once (a list merge); this design "
                        "reads less, so the rate may exceed the peak"}
        if traffic:
            tg = traffic / (ms / 1e3) / 1e9
            result["roofline"]["traffic_gbs"] = tg
            result["roofline"]["traffic_frac_of_peak"] = tg / HBM_PEAK_GBS
    if "roofline" in result:
        # the issue side of the same launch, from its committed counters
        result["roofline"].update(valu_issue(name, ms))
    if cb is not None:
        cb.pop("count", None)
        cb.pop("bytes", None)
        cb.pop("held_bytes", None)
        cb.pop("held_tests", None)
        result["cpu_baseline"] = cb
    trie.free()
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat20_triangles", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the streaming-read probe (for profiling runs)")
    ap.add_argument("--rates", default="100,200,500,1000,2000,5000",
                    help="served: arrival rates (QPS)")
    ap.add_argument("--policy", type=int, default=1, choices=(0, 1),
                    help="served: 0 oldest request first, 1 fewest items left first")
    ap.add_argument("--duration", type=float, default=10.0, help="served: measured seconds per rate")
    ap.add_argument("--warmup-s", type=float, default=1.0, help="served: warm-up seconds per rate")
    ap.add_argument("--max-requests", type=int, default=0,
                    help="served: cap on requests per rate (0: none)")
    ap.add_argument("--no-code-warmup", action="store_true",
                    help="skip the small-graph count that loads the code before the first count "
                         "(profiles: then every dispatch of the kernel is the workload's)")
    ap.add_argument("--no-per-instance", action="store_true",
                    help="batch: skip the one-launch-per-graph comparison (for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("this engine runs on one GPU; no multi-GPU path exists (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1503_02368_amd import eh
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    ctx = eh.Context(0)
    name = args.workload
    w = WORKLOADS[name]
    if w["kind"] == "graph":
        res = bench_graph(name, w, args, ctx, eh, torch)
    elif w["kind"] == "batch":
        import bench_legs as bench_extra
        res = bench_extra.bench_batch(name, w, args, ctx, eh, torch, METRIC)
    elif w["kind"] == "ablation":
        import bench_legs as bench_extra
        res = bench_extra.bench_ablation(name, w, args, ctx, eh, torch, METRIC)
    elif w["kind"] == "unpruned":
        import bench_legs as bench_extra
        res = bench_extra.bench_unpruned(name, w, args, ctx, eh, torch, METRIC)
    elif w["kind"] == "build":
        import bench_legs as bench_extra
        res = bench_extra.bench_build(name, w, args, ctx, eh, torch, METRIC)
    elif w["kind"] == "composite":
        import bench_legs as bench_extra
        res = bench_extra.bench_composite(name, w, args, ctx, eh, torch, METRIC)
    elif w["kind"] == "orderings":
        import bench_legs as bench_extra
        res = bench_extra.bench_orderings(name, w, args, ctx, eh, torch, METRIC)
    else:
        import bench_legs as bench_extra
        res = bench_extra.bench_served(name, w, args, ctx, eh, torch, METRIC)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
