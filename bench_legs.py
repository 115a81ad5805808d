"""Batched and served benchmark legs, called from the repository's bench.py.

Batched: many independent graphs counted by one launch over their
concatenated trie, beside one launch per graph (eager, and replayed from a
captured HIP graph) on the same GPU and data; the per-graph count vectors
must be identical.

Orderings: the node-ordering study of appendix A on Chung-Lu power-law
graphs of several exponents: triangle counting under each ordering, with
the trie statistics that explain the differences.

Build: the trie built on the host from host arrays (then uploaded) beside
the same trie built on the GPU from pairs already in device memory, and the
first count on each (which adds work-item planning) against a repeat.

Unpruned: the triangle and Lollipop queries on the full symmetric adjacency
of R-MAT s20 (section 5.3 runs Lollipop on undirected data), beside triangle
counting on the pruned trie.

Ablation: R-MAT s20 triangle counting with the layout choices switched off
one at a time (the paper's -R and -RA columns, section 5.4): uint-only and
all-bitset layouts, no bitset reads, and the pairwise kernel with merges only.

Served: a resident graph answers rooted count requests that arrive as an
open-loop Poisson stream; latency is completion time (taken on the device
step's completion) minus the request's scheduled arrival, so a backlog shows
up as latency (no coordinated omission).  A serial server that answers one
request per blocking call on the same schedule runs beside it.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
import sys
import threading
import time

import numpy as np

from paper_1503_02368_amd.profile_summary import SETS_SRC, kernel_sha, measured_traffic, valu_issue  # noqa: E402,F401

_PKG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1503_02368_amd")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_tuning(name: str) -> dict:
    import json
    import os
    path = os.path.join(_PKG, "tuning.json")
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f).get(name, {})
    return {}


def _pct(xs, q):
    if not xs:
        return None
    s = sorted(xs)
    k = min(len(s) - 1, max(0, int(round(q / 100.0 * (len(s) - 1)))))
    return s[k]


def bench_batch(name, w, args, ctx, eh, torch, metric):
    from paper_1503_02368_amd import inputs
    t0 = time.perf_counter()
    b = inputs.batch_chung_lu(w["graphs"], seed=w["seed"])
    log(f"[bench] batch generated in {time.perf_counter() - t0:.1f} s: {b.n_graphs} graphs, "
        f"{b.src.size} raw pairs")
    tune = load_tuning(name)
    layout = tune.get("layout", w["layout"])
    tau = tune.get("tau", w["tau"])
    if tune.get("tuning"):
        ctx.set_tuning(**tune["tuning"])
    t0 = time.perf_counter()
    trie = ctx.build_batch(b, layout=layout, tau=tau, s_min=tune.get("s_min", 1))
    info = trie.info
    log(f"[bench] batch trie built in {time.perf_counter() - t0:.1f} s: {info}")
    G = info["n_graphs"]
    pattern = w["pattern"]
    s = ctx.stream
    out = torch.zeros(G, dtype=torch.int64, device="cuda")
    s.wait_stream(torch.cuda.current_stream())
    for _ in range(max(1, args.warmup)):
        ctx.count_batch_async(trie, pattern, 0, G, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.steps):
        ctx.count_batch_async(trie, pattern, 0, G, out)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    one = out.cpu().numpy().view(np.uint64).copy()
    log(f"[bench] one launch: {ms:.3f} ms per pass")
    # the same launch captured once into a HIP graph and replayed
    ms_one_graph = None
    try:
        g1 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g1, stream=s):
            ctx.count_batch_async(trie, pattern, 0, G, out)
        # replays run on the context's stream, the one the events time
        with torch.cuda.stream(s):
            g1.replay()
        torch.cuda.synchronize()
        e0.record(s)
        with torch.cuda.stream(s):
            for _ in range(args.steps):
                g1.replay()
        e1.record(s)
        torch.cuda.synchronize()
        ms_one_graph = e0.elapsed_time(e1) / args.steps
        out.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g1.replay()
        torch.cuda.synchronize()
        if not np.array_equal(out.cpu().numpy().view(np.uint64), one):
            raise RuntimeError("graph-replayed batch counts differ from the eager launch")
        log(f"[bench] one launch, graph replay: {ms_one_graph:.3f} ms per pass")
        del g1
    except RuntimeError as e:
        if "differ" in str(e):
            raise
        log(f"[bench] graph capture unavailable: {e}")
    roofline = _batch_roofline(ctx, eh, info, ms, name)
    if getattr(args, "no_per_instance", False):
        trie.free()
        return {"metric": metric, "value": info["m_plus"] / (ms / 1e3), "unit": "edges/s",
                "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
                "data": "synthetic (seeded generator)",
                "config": {"workload": name, "graphs": G, "m_plus": info["m_plus"]},
                "count_total": int(one.sum(dtype=np.uint64)), "roofline": roofline}
    # one launch per graph, eager, on the static schedule: a per-graph launch
    # is too small for the cursor schedules to pay for their reset
    tuned = ctx.get_tuning()
    ctx.set_tuning(dynamic=0)
    per = torch.zeros(G, dtype=torch.int64, device="cuda")
    for i in range(min(G, 64)):
        ctx.count_batch_async(trie, pattern, i, 1, per[i:i + 1])
    torch.cuda.synchronize()
    e0.record(s)
    for i in range(G):
        ctx.count_batch_async(trie, pattern, i, 1, per[i:i + 1])
    e1.record(s)
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1)
    per_np = per.cpu().numpy().view(np.uint64).copy()
    log(f"[bench] one launch per graph: {ms_loop:.3f} ms per pass")
    # one launch per graph, captured once into a HIP graph and replayed
    ms_graph = None
    try:
        per_g = torch.zeros(G, dtype=torch.int64, device="cuda")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for i in range(G):
                ctx.count_batch_async(trie, pattern, i, 1, per_g[i:i + 1])
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        e0.record(s)
        reps = 3
        with torch.cuda.stream(s):
            for _ in range(reps):
                g.replay()
        e1.record(s)
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / reps
        per_g.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        if not np.array_equal(per_g.cpu().numpy().view(np.uint64), one):
            raise RuntimeError("graph-replayed per-graph counts differ from the one-launch counts")
        log(f"[bench] one launch per graph, graph replay: {ms_graph:.3f} ms per pass")
        del g
    except RuntimeError as e:
        if "differ" in str(e):
            raise
        log(f"[bench] graph capture unavailable: {e}")
    ctx.set_tuning(**tuned)
    if not np.array_equal(per_np, one):
        raise RuntimeError("per-graph launches and the single launch disagree")
    m_plus = info["m_plus"]
    res = {
        "metric": metric, "value": m_plus / (ms / 1e3), "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded generator)",
        "config": {"workload": name, "graphs": G, "n_total": info["n"], "m_plus": m_plus,
                   "generator": "Chung-Lu gamma 2.1, n log-U[64,16384], mean degree log-U[8,64]",
                   "seed": w["seed"], "layout": ["uint", "hybrid", "bitset_all"][layout], "tau": tau,
                   "tuning": ctx.get_tuning()},
        "count_total": int(one.sum(dtype=np.uint64)),
        "one_launch_graph_replay_ms": ms_one_graph,
        "per_instance": {"ms_per_pass": ms_loop, "edges_per_s": m_plus / (ms_loop / 1e3),
                         "graph_replay_ms_per_pass": ms_graph,
                         "speedup_of_one_launch": ms_loop / ms,
                         "identical_counts": True},
    }
    res["roofline"] = roofline
    if not args.no_cpu:
        # every graph's count against the oracle's, graphs counted in parallel
        import oracle
        threads = oracle.max_threads()
        t0 = time.perf_counter()
        want, _, _ = oracle.batch_triangles(b.n_vertices, b.edge_off, b.src, b.dst, threads=threads)
        t = time.perf_counter() - t0
        bad = np.flatnonzero(want != one)
        res["parity_vs_oracle"] = bool(bad.size == 0)
        res["graphs_compared_with_oracle"] = int(G)
        if bad.size:
            log(f"[bench] {bad.size} graphs differ from the oracle, first {int(bad[0])}")
        if pattern == 3:
            res["cpu_baseline"] = {"value": info["m_plus"] / t, "unit": "edges/s", "cores": threads,
                                   "kind": "oracle",
                                   "sample": f"all {G} graphs, in parallel over graphs (each graph's "
                                             f"clean, rank and orient included), {t:.1f} s"}
    trie.free()
    return res


def _batch_roofline(ctx, eh, info, ms, name):
    """Roofline of the batch's one launch: B_target (what target staging must
    read, summed over the graphs) when the tuning stages targets, else
    B_merge; the merge-equivalent rate beside it."""
    tun = ctx.get_tuning()
    target = (tun["kernel"] != eh.KERNEL_PAIRWISE and tun["staging"] != eh.STAGE_SOURCE
              and info["b_target"] > 0)
    model, mb = ("B_target", info["b_target"]) if target else ("B_merge", info["b_merge"])
    achieved = mb / (ms / 1e3) / 1e9
    r = {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
         "frac": achieved / 8000.0, "traffic": measured_traffic(name),
         "traffic_kind": "L2-to-fabric bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                         "copy-calibrated)",
         "algorithmic_bytes_per_launch": mb, "model": model, "kernel_ms_per_launch": ms,
         "merge_equivalent": {"model": "B_merge", "bytes_per_launch": info["b_merge"],
                              "gbs": info["b_merge"] / (ms / 1e3) / 1e9}}
    if r["traffic"]:
        r["traffic_gbs"] = r["traffic"] / (ms / 1e3) / 1e9
    r.update(valu_issue(name, ms))
    return r


def bench_served(name, w, args, ctx, eh, torch, metric):
    from paper_1503_02368_amd import inputs
    t0 = time.perf_counter()
    el = inputs.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
    log(f"[bench] served graph generated in {time.perf_counter() - t0:.1f} s")
    tune = load_tuning(name)
    if tune.get("tuning"):
        ctx.set_tuning(**tune["tuning"])  # servers copy the tuning when created
    trie = ctx.build_edgelist(el, layout=tune.get("layout", w["layout"]), tau=tune.get("tau", w["tau"]),
                              s_min=tune.get("s_min", 1))
    info = trie.info
    log(f"[bench] resident trie: {info}")
    rates = [float(x) for x in args.rates.split(",")]
    # out-degree of each original id: a request's root out-edges are its work
    ha = trie.host_arrays()
    dplus_by_id = np.diff(ha["row"].astype(np.int64))[ha["rank"].astype(np.int64)]
    del ha
    root_t = root_k = None
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = oracle.max_threads()
        og = oracle.Graph.from_edgelist(el)
        tt = time.perf_counter()
        rt = og.triangles(threads=threads, rooted=True)
        t_tri = time.perf_counter() - tt
        root_t = rt["root"]
        tt = time.perf_counter()
        # the rooted 4-clique table in 16 ranges of outer vertices (a progress
        # line each: the whole table takes minutes at scale 22)
        root_k = np.zeros(og.n, np.uint64)
        cuts = np.linspace(0, og.n, 17).astype(np.int64)
        for a, b in zip(cuts[:-1], cuts[1:]):
            root_k += og.cliques4(threads=threads, rooted=True, x_begin=int(a), x_end=int(b))["root"]
            log(f"[bench] oracle 4-clique table: outer ranks < {b} done, "
                f"{time.perf_counter() - tt:.0f} s")
        t_k4 = time.perf_counter() - tt
        cpu = {"value": og.m / t_tri, "unit": "edges/s", "cores": threads, "kind": "oracle",
               "sample": f"whole graph: rooted triangle table {t_tri:.2f} s, rooted 4-clique table "
                         f"{t_k4:.2f} s; every served answer is checked against these tables"}
        log(f"[bench] oracle tables: triangles {t_tri:.1f} s, 4-cliques {t_k4:.1f} s")

    def want(r):
        tab = root_t if r.pattern == 3 else root_k
        return None if tab is None else int(tab[np.unique(r.roots.astype(np.int64))].sum(dtype=np.uint64))

    table = []
    all_ok = True
    checked = 0
    warm = args.warmup_s
    for rate in rates:
        span_s = warm + args.duration
        if args.max_requests:
            span_s = min(span_s, args.max_requests / rate)
        reqs = inputs.request_stream(el.n, rate_qps=rate, duration_s=span_s, seed=w["seed"] + int(rate))
        meas = [i for i, r in enumerate(reqs) if r.t_arrival >= warm]
        log(f"[bench] rate {rate:g} QPS: {len(reqs)} requests over {span_s:.1f} s, "
            f"{len(meas)} after the {warm:g} s warm-up")
        row = {"rate_qps": rate, "requests": len(reqs), "measured_requests": len(meas),
               "warmup_s": warm, "measured_s": span_s - warm}
        wall = (span_s - warm) if span_s > warm else span_s
        req_edges = sum(int(dplus_by_id[np.unique(reqs[i].roots.astype(np.int64))].sum()) for i in meas)
        wants = [want(r) for r in reqs] if root_t is not None else None
        for mode in ("batched", "serial"):
            # the serial server stops taking requests 5 s after the last arrival:
            # requests it never started count with the latency they had reached then
            lat, counts, done = serve_run(ctx, eh, trie, reqs, mode, policy=args.policy,
                                          deadline_s=span_s + 5.0 if mode == "serial" else None)
            ok = None
            if wants is not None:
                ok = all(counts[i] == wants[i] for i in range(len(reqs)) if done[i])
                checked += sum(done)
            all_ok = all_ok and (ok is not False)
            ml = [lat[i] for i in meas]
            finished = sum(1 for i in meas if done[i])
            row[mode] = {"p50_ms": 1e3 * _pct(ml, 50), "p99_ms": 1e3 * _pct(ml, 99),
                         "mean_ms": 1e3 * statistics.fmean(ml) if ml else None,
                         "completed_in_window": finished,
                         "completed_qps": finished / wall,
                         "root_out_edges_per_s": req_edges / wall if finished == len(meas) else None,
                         "exact": ok}
            if finished < len(meas):
                row[mode]["unserved"] = len(meas) - finished
                row[mode]["note"] = ("saturated: unserved requests enter the percentiles with the "
                                     "latency they had reached when the run stopped (lower bounds)")
            log(f"[bench]   {mode}: p50 {row[mode]['p50_ms']:.2f} ms, p99 {row[mode]['p99_ms']:.2f} ms, "
                f"{finished}/{len(meas)} served, exact {ok}")
        table.append(row)
    top = table[-1]
    res = {
        "metric": metric, "value": top["batched"]["p99_ms"], "unit": "ms (p99 latency at the highest rate)",
        "n_gpus": 1, "steps": len(rates), "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded generator)",
        "config": {"workload": name, "scale": w["scale"], "edge_factor": w["edge_factor"], "seed": w["seed"],
                   "n": info["n"], "m_plus": info["m_plus"], "pattern_mix": "80% triangle / 20% 4-clique",
                   "roots": "log-uniform 2^8..2^16 distinct ids", "tuning": ctx.get_tuning(),
                   "policy": ["oldest first", "fewest items left first"][args.policy]},
        "rates": table,
        "parity_vs_oracle": all_ok if root_t is not None else None,
        "answers_checked_vs_oracle": checked,
        "protocol": f"per rate: open-loop Poisson arrivals for {args.warmup_s:g} s of warm-up and "
                    f"{args.duration:g} s measured; latency from scheduled arrival to completion",
    }
    if cpu:
        res["cpu_baseline"] = cpu
    trie.free()
    return res


def _time_counts(ctx, torch, trie, pattern, steps, warmup):
    """Average ms of one counting launch over `steps` back-to-back launches
    on the context's stream, and the count."""
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = ctx.stream
    s.wait_stream(torch.cuda.current_stream())
    for _ in range(warmup):
        ctx.count_add_async(trie, pattern, out)
    torch.cuda.synchronize()
    out.zero_()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s)
    for _ in range(steps):
        ctx.count_add_async(trie, pattern, out)
    ev1.record(s)
    torch.cuda.synchronize()
    total = int(out.cpu().numpy().view(np.uint64)[0])
    count, rem = divmod(total, steps)
    if rem:
        raise RuntimeError("accumulated count is not a multiple of the step count")
    return ev0.elapsed_time(ev1) / steps, count


# Candidate kernel settings per cell, on top of the R-MAT s20 tuning: orderings
# that leave long out-sets favour other staging sides or the pairwise kernel.
ORDER_VARIANTS = {
    "tuned": {},
    "source": dict(staging=1),
    "full_words": dict(stage_words=0),
    "pairwise": dict(kernel=2, algo=0, group_lanes=0),
}


def bench_orderings(name, w, args, ctx, eh, torch, metric):
    from paper_1503_02368_amd import inputs
    base = dict(ctx.get_tuning())
    base.update(load_tuning("rmat20_triangles").get("tuning", {}))
    table = []
    parity = True
    tot_edges = tot_ms = 0.0
    for gamma in w["gammas"]:
        el0 = inputs.chung_lu(w["n"], w["avg_degree"], gamma, seed=w["seed"])
        ref = None
        if not args.no_cpu:
            import oracle
            t0 = time.perf_counter()
            ref = oracle.Graph.from_edgelist(el0).triangles(threads=oracle.max_threads())["count"]
            log(f"[bench] gamma {gamma}: oracle count {ref} in {time.perf_counter() - t0:.1f} s")
        for order in w["orders"]:
            # the paper's Random ordering: a seeded relabelling, ids then kept as given
            el = inputs.relabel(el0, w["seed"]) if order == "random" else el0
            code = eh.ORDER_INPUT if order == "random" else eh.ORDERS[order]
            t0 = time.perf_counter()
            trie = ctx.build_edgelist(el, layout=w["layout"], tau=w["tau"], order=code)
            t_build = time.perf_counter() - t0
            info = trie.info
            best = None
            counts = set()
            try:
                for vname, v in ORDER_VARIANTS.items():
                    t = dict(base)
                    t.update(v)
                    ctx.set_tuning(**t)
                    ms, cnt = _time_counts(ctx, torch, trie, 3, args.steps, args.warmup)
                    counts.add(cnt)
                    if best is None or ms < best[0]:
                        best = (ms, vname)
            finally:
                trie.free()
            ok = len(counts) == 1 and (ref is None or counts == {ref})
            parity = parity and ok
            row = {"gamma": gamma, "order": order, "ms": best[0], "kernel_setting": best[1],
                   "edges_per_s": info["m_plus"] / (best[0] / 1e3), "m_plus": info["m_plus"],
                   "b_merge": info["b_merge"], "max_out_degree": info["max_out_degree"],
                   "bitset_sets": info["n_bitset_sets"], "bitset_words": info["bitset_words"],
                   "host_build_s": t_build, "count": counts.pop() if len(counts) == 1 else None,
                   "exact": ok}
            if order == "degree":
                tot_edges += info["m_plus"]
                tot_ms += best[0]
            log(f"[bench] gamma {gamma} {order:>11}: {best[0]:.3f} ms ({best[1]}), d+max "
                f"{info['max_out_degree']}, bitset sets {info['n_bitset_sets']}, "
                f"B_merge {info['b_merge'] / 1e9:.2f} GB, build {t_build:.2f} s, exact {ok}")
            table.append(row)
    ctx.set_tuning(**base)
    return {
        "metric": metric, "value": tot_edges / (tot_ms / 1e3), "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": tot_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": name, "n": w["n"], "avg_degree": w["avg_degree"],
                   "gammas": w["gammas"], "orders": w["orders"], "layout": "hybrid", "tau": w["tau"],
                   "value_is": "sum of m_plus over the exponents / sum of ms, degree ordering",
                   "kernel_settings": "best of " + ", ".join(ORDER_VARIANTS) +
                                      " on the R-MAT s20 tuning, per cell"},
        "table": table,
        "parity_vs_oracle": parity,
    }


def bench_build(name, w, args, ctx, eh, torch, metric):
    from paper_1503_02368_amd import inputs
    rows = []
    for scale in w["scales"]:
        el = inputs.rmat(scale, w["edge_factor"], seed=scale)
        hs = torch.from_numpy(np.ascontiguousarray(el.src).view(np.int32)).pin_memory()
        hd = torch.from_numpy(np.ascontiguousarray(el.dst).view(np.int32)).pin_memory()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        src = hs.cuda(non_blocking=True)
        dst = hd.cuda(non_blocking=True)
        torch.cuda.synchronize()
        t_copy = time.perf_counter() - t0
        del hs, hd
        ctx.set_tuning(**dict(ctx.get_tuning(), **load_tuning("rmat20_triangles").get("tuning", {})))
        row = {"scale": scale, "raw_pairs": int(el.m_raw), "pairs_h2d_ms": 1e3 * t_copy,
               "pairs_h2d_gbs": 8 * el.m_raw / t_copy / 1e9}
        log(f"[bench] rmat{scale}: pairs to HBM (pinned) {1e3 * t_copy:.1f} ms")
        for how in ("host", "device"):
            times = []
            for rep in range(args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if how == "host":
                    trie = ctx.build_edgelist(el, layout=w["layout"], tau=w["tau"])
                else:
                    trie = ctx.build_trie_device(el.n, src, dst, layout=w["layout"], tau=w["tau"])
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                if rep < args.steps - 1:
                    trie.free()
            t_build = statistics.median(times)
            t0 = time.perf_counter()
            first = ctx.count_triangles(trie)
            t_first = time.perf_counter() - t0
            t0 = time.perf_counter()
            again = ctx.count_triangles(trie)
            t_again = time.perf_counter() - t0
            row[how] = {"build_ms": 1e3 * t_build, "build_ms_all": [1e3 * t for t in times],
                        "first_count_ms": 1e3 * t_first, "repeat_count_ms": 1e3 * t_again,
                        "count": first, "m_plus": trie.info["m_plus"]}
            if first != again:
                raise RuntimeError("counts differ between calls")
            log(f"[bench] rmat{scale} {how} build {1e3 * t_build:.1f} ms (median of {len(times)}), "
                f"first count {1e3 * t_first:.1f} ms, repeat {1e3 * t_again:.2f} ms")
            trie.free()
        row["speedup"] = row["host"]["build_ms"] / row["device"]["build_ms"]
        row["same_count"] = row["host"]["count"] == row["device"]["count"]
        rows.append(row)
        del src, dst
    if w.get("batch"):
        from paper_1503_02368_amd.workloads import WORKLOADS, make_batch
        bw = WORKLOADS["batch_triangles"]
        bt = load_tuning("batch_triangles")
        b = make_batch(bw)
        src = torch.from_numpy(np.ascontiguousarray(b.src).view(np.int32)).cuda()
        dst = torch.from_numpy(np.ascontiguousarray(b.dst).view(np.int32)).cuda()
        torch.cuda.synchronize()
        ctx.set_tuning(**dict(ctx.get_tuning(), **bt.get("tuning", {})))
        row = {"batch_graphs": b.n_graphs, "raw_pairs": int(b.src.size)}
        lay, tau = bt.get("layout", bw["layout"]), bt.get("tau", bw["tau"])
        for how in ("host", "device"):
            times = []
            for rep in range(max(1, min(args.steps, 2))):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if how == "host":
                    trie = ctx.build_batch(b, layout=lay, tau=tau)
                else:
                    trie = ctx.build_batch_device(b, src, dst, layout=lay, tau=tau)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                if rep < max(1, min(args.steps, 2)) - 1:
                    trie.free()
            t0 = time.perf_counter()
            first = int(ctx.count_batch(trie, eh.TRIANGLE).sum(dtype=np.uint64))
            t_first = time.perf_counter() - t0
            row[how] = {"build_ms": 1e3 * min(times), "first_count_ms": 1e3 * t_first,
                        "count": first}
            log(f"[bench] batch {how} build {1e3 * min(times):.0f} ms (best of {len(times)}), "
                f"first count {1e3 * t_first:.0f} ms")
            trie.free()
        row["speedup"] = row["host"]["build_ms"] / row["device"]["build_ms"]
        row["same_count"] = row["host"]["count"] == row["device"]["count"]
        rows.append(row)
        del src, dst
    top = rows[-1]
    return {
        "metric": metric, "value": top["raw_pairs"] / (top["device"]["build_ms"] / 1e3),
        "unit": "raw pairs/s (GPU trie build)", "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": top["device"]["build_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded generator)",
        "config": {"workload": name, "scales": w["scales"], "edge_factor": w["edge_factor"],
                   "layout": "hybrid", "tau": w["tau"],
                   "host_build": "eh_build_trie from host arrays (host build plus upload)",
                   "device_build": "eh_build_trie_device / eh_build_batch_device from pairs resident in HBM",
                   "value_is": "raw pairs per second of the last row's GPU build (the 20,000-graph batch)"},
        "table": rows,
        "same_counts": all(r["same_count"] for r in rows),
    }


# every arc evaluated (source staging), or each undirected edge once at its
# higher-ranked end and doubled (any other staging)
UNPRUNED_VARIANTS = {
    "source": dict(staging=1),
    "source_full_words": dict(staging=1, stage_words=0),
    "edge_once": dict(staging=2),
    "edge_once_full_words": dict(staging=2, stage_words=0),
    "edge_once_unroll4": dict(staging=2, stage_words=0, unroll=4),
    "edge_once_cursors": dict(staging=2, stage_words=0, dynamic=4, search_below=64),
    "pairwise_edge_once": dict(kernel=2, algo=0, group_lanes=0),
}


def bench_unpruned(name, w, args, ctx, eh, torch, metric):
    from paper_1503_02368_amd import inputs
    el = inputs.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
    base = dict(ctx.get_tuning())
    base.update(load_tuning("rmat20_triangles").get("tuning", {}))
    rows = {}
    pruned = ctx.build_edgelist(el, layout=w["layout"], tau=w["tau"])
    ctx.set_tuning(**base)
    ms_p, t_count = _time_counts(ctx, torch, pruned, 3, args.steps, args.warmup)
    rows["pruned_triangles"] = {"ms": ms_p, "count": t_count, "m_plus": pruned.info["m_plus"],
                                "b_merge": pruned.info["b_merge"]}
    log(f"[bench] pruned triangles {ms_p:.3f} ms, T = {t_count}")
    pruned.free()
    t0 = time.perf_counter()
    trie = ctx.build_edgelist(el, layout=w["layout"], tau=w["tau"], symmetric=True)
    info = trie.info
    log(f"[bench] symmetric trie in {time.perf_counter() - t0:.2f} s: {info}")
    best = None
    for vname, v in UNPRUNED_VARIANTS.items():
        t = dict(base)
        t.update(v)
        ctx.set_tuning(**t)
        ms, c6 = _time_counts(ctx, torch, trie, 3, args.steps, args.warmup)
        log(f"[bench] unpruned triangles, {vname}: {ms:.3f} ms, count {c6}")
        if best is None or ms < best[0]:
            best = (ms, vname, c6)
    ctx.set_tuning(**dict(base, **UNPRUNED_VARIANTS[best[1]]))
    lol = []
    lcount = None
    for _ in range(max(3, args.steps // 4)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lcount = ctx.count_lollipop(trie)
        lol.append(time.perf_counter() - t0)
    rows["unpruned_triangles"] = {"ms": best[0], "kernel_setting": best[1], "count": best[2],
                                  "m_plus": info["m_plus"], "b_merge": info["b_merge"],
                                  "max_degree": info["max_out_degree"]}
    rows["lollipop"] = {"ms": 1e3 * statistics.median(lol), "count": lcount,
                        "includes": "one edge-once launch weighted by degree, read-back"}
    log(f"[bench] Lollipop {rows['lollipop']['ms']:.3f} ms, count {lcount}")
    # the same ordered-triangle count as one pairwise intersection per arc over a
    # set store: a hub's set is met by probing its bitset with the smaller set
    h = trie.host_arrays()
    off = h["row"].astype(np.uint64)
    src = np.repeat(np.arange(off.size - 1, dtype=np.uint32), np.diff(off.astype(np.int64)))
    pair_rows = _layout_rows(ctx, eh, torch, off, h["col"], np.stack([src, h["col"]], axis=1),
                             args, best[2], w["tau"], {"graph": "unpruned"})
    del h, src
    rows["pairwise_by_layout"] = pair_rows
    parity = {"six_t": best[2] == 6 * t_count,
              "pairwise": all(r["correct"] for r in pair_rows)}
    k4 = unpruned_4cliques(ctx, eh, torch, args, w.get("k4_scale", 16), w["edge_factor"], base)
    rows["unpruned_4cliques"] = k4
    parity["twenty_four_k"] = k4["count_unpruned"] == 24 * k4["count_pruned"]
    if "oracle_k" in k4:
        parity["k4_oracle"] = k4["oracle_k"] == k4["count_pruned"]
    cpu = None
    if not args.no_cpu:
        import oracle
        g = oracle.Graph.from_edgelist(el)
        th = oracle.max_threads()
        t0 = time.perf_counter()
        six_t, _ = g.sym_triangles_by_first(threads=th)
        t_tri = time.perf_counter() - t0
        t0 = time.perf_counter()
        ref_l = g.sym_lollipop(threads=th)
        t_l = time.perf_counter() - t0
        parity.update(six_t_oracle=six_t == best[2], lollipop_oracle=ref_l == lcount)
        cpu = {"value": info["m_plus"] / t_tri, "unit": "stored edges/s", "cores": th,
               "kind": "oracle", "sample": f"whole graph: unpruned triangles {t_tri:.2f} s, "
                                           f"Lollipop {t_l:.2f} s"}
        log(f"[bench] oracle: unpruned triangles {t_tri:.2f} s, Lollipop {t_l:.2f} s")
    trie.free()
    ms = best[0]
    achieved = info["b_merge"] / (ms / 1e3) / 1e9
    res = {
        "metric": metric, "value": info["m_plus"] / (ms / 1e3), "unit": "stored edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": name, "scale": w["scale"], "edge_factor": w["edge_factor"],
                   "seed": w["seed"], "layout": "hybrid", "tau": w["tau"],
                   "relation": "both directions of every edge (unpruned)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0, "traffic": None,
                     "algorithmic_bytes_per_launch": info["b_merge"], "model": "B_merge (arcs)"},
        "table": rows,
        "parity_vs_oracle": all(parity.values()),
    }
    if cpu:
        res["cpu_baseline"] = cpu
    return res


def unpruned_4cliques(ctx, eh, torch, args, scale, edge_factor, base):
    """4-cliques on R-MAT at `scale` (seed = scale): pruned (K) beside the
    unpruned relation (24 K ordered tuples), whose hub roots keep S in HBM
    lists; times of single blocking counts (median of 3, plan cached)."""
    from paper_1503_02368_amd import inputs
    el = inputs.rmat(scale, edge_factor, seed=scale)
    out = {"graph": f"rmat{scale} edge factor {edge_factor}, seed {scale}"}
    ctx.set_tuning(**dict(base, kernel=1, staging=1, dynamic=4, grab=2, chunk_work=4096,
                          stage_words=0))
    for key, kw in (("pruned", {}), ("unpruned", {"symmetric": True})):
        trie = ctx.build_edgelist(el, layout=1, tau=32.0, **kw)
        try:
            c = ctx.count_4cliques(trie)   # builds the plan
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c2 = ctx.count_4cliques(trie)
                ts.append(time.perf_counter() - t0)
                if c2 != c:
                    raise RuntimeError("4-clique counts differ between repeats")
            out[f"ms_{key}"] = 1e3 * statistics.median(ts)
            out[f"count_{key}"] = c
            out[f"max_degree_{key}"] = trie.info["max_out_degree"]
            log(f"[bench] {key} 4-cliques on rmat{scale}: {out[f'ms_{key}']:.2f} ms, count {c}")
        finally:
            trie.free()
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        out["oracle_k"] = oracle.Graph.from_edgelist(el).count(4, threads=oracle.max_threads())
        out["oracle_s"] = time.perf_counter() - t0
    return out


# (name, layout, tau, tuning changes): each a performance choice; the count never changes
ABLATION = [
    ("hybrid, tuned", None, None, {}),
    ("uint only (-R)", 0, 32.0, {}),
    ("all bitset", 2, 32.0, {}),
    ("hybrid layout, bitset words never streamed", None, None, {"use_bitsets": 0}),
    ("pairwise, hybrid, merge or galloping", None, None, {"kernel": 2, "algo": 0, "group_lanes": 0}),
    ("pairwise, uint only, merge only (-RA)", 0, 32.0,
     {"kernel": 2, "algo": 1, "group_lanes": 0, "use_bitsets": 0}),
]


def bench_ablation(name, w, args, ctx, eh, torch, metric):
    from paper_1503_02368_amd import inputs
    el = inputs.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
    tuned = load_tuning("rmat20_triangles")
    base = dict(ctx.get_tuning())
    base.update(tuned.get("tuning", {}))
    rows = []
    counts = set()
    cache = {}
    for label, lay, tau, change in ABLATION:
        lay = tuned.get("layout", 1) if lay is None else lay
        tau = tuned.get("tau", 256.0) if tau is None else tau
        if (lay, tau) not in cache:
            for t in cache.values():
                t.free()
            cache.clear()
            cache[(lay, tau)] = ctx.build_edgelist(el, layout=lay, tau=tau)
        trie = cache[(lay, tau)]
        ctx.set_tuning(**dict(base, **change))
        ms, c = _time_counts(ctx, torch, trie, 3, args.steps, args.warmup)
        counts.add(c)
        info = trie.info
        rows.append({"variant": label, "layout": ["uint", "hybrid", "bitset_all"][lay], "tau": tau,
                     "ms": ms, "edges_per_s": info["m_plus"] / (ms / 1e3),
                     "b_merge_per_s_gbs": info["b_merge"] / (ms / 1e3) / 1e9,
                     "bitset_sets": info["n_bitset_sets"], "count": c})
        log(f"[bench] {label:45s} {ms:8.3f} ms  count {c}")
    for t in cache.values():
        t.free()
    ctx.set_tuning(**base)
    ref = rows[0]["ms"]
    for r in rows:
        r["slowdown_vs_tuned"] = r["ms"] / ref
    return {
        "metric": metric, "value": rows[0]["edges_per_s"], "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ref, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded generator)",
        "config": {"workload": name, "scale": w["scale"], "edge_factor": w["edge_factor"],
                   "seed": w["seed"], "value_is": "the tuned hybrid row"},
        "table": rows,
        "same_count": len(counts) == 1,
    }


SET_LAYOUTS = ("uint", "set", "bitset", "composite")
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def _time_pairs(ctx, torch, st, d_pairs, steps, warmup):
    """Average ms of one pairwise-intersection launch over `steps` launches on
    the context's stream, and the total."""
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = ctx.stream
    s.wait_stream(torch.cuda.current_stream())
    for _ in range(warmup):
        ctx.intersect_pairs_async(st, d_pairs, out)
    torch.cuda.synchronize()
    out.zero_()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s)
    for _ in range(steps):
        ctx.intersect_pairs_async(st, d_pairs, out)
    ev1.record(s)
    torch.cuda.synchronize()
    total, rem = divmod(int(out.cpu().numpy().view(np.uint64)[0]), steps)
    if rem:
        raise RuntimeError("accumulated total is not a multiple of the step count")
    return ev0.elapsed_time(ev1) / steps, total


def _layout_rows(ctx, eh, torch, off, members, pairs, args, expect, tau, extra,
                 layouts=SET_LAYOUTS):
    d_pairs = torch.from_numpy(np.ascontiguousarray(pairs, np.uint32).view(np.int32)).cuda()
    n_members = int(members.size)
    touched = int(np.sum(np.diff(off.astype(np.int64))[pairs.ravel()]))  # members over both sides
    rows = []
    for lay in layouts:
        t0 = time.perf_counter()
        st = ctx.build_sets(off, members, layout=eh.SET_LAYOUTS[lay], tau=tau)
        enc = time.perf_counter() - t0
        ms, tot = _time_pairs(ctx, torch, st, d_pairs, args.steps, args.warmup)
        i = st.info
        st.free()
        stored = i["device_bytes"] - 4 * (i["n_sets"] + 1)
        row = dict(extra, layout=lay, ms=ms, total=tot,
                   correct=None if expect is None else tot == expect,
                   members_per_s=touched / (ms / 1e3), store_bytes=stored,
                   store_read_gbs=stored / (ms / 1e3) / 1e9,
                   bytes_per_launch=stored + 8 * int(pairs.shape[0]), segments=i["n_segments"],
                   bitset_segments=i["n_bitset_segments"], uint_members=i["uint_members"],
                   bitset_words=i["bitset_words"], encode_s=enc)
        rows.append(row)
        log(f"[bench] {str(extra.get('dense_frac', extra.get('graph'))):8s} {lay:9s} {ms:9.3f} ms  {stored / 2**20:9.1f} MiB stored"
            f"  segments {i['n_segments']:>10d}  total {tot}{'' if tot == expect else ' MISMATCH'}")
    del d_pairs
    best = min(r["ms"] for r in rows)
    for r in rows:
        r["vs_best"] = r["ms"] / best
    return rows


def bench_composite(name, w, args, ctx, eh, torch, metric):
    """Section 4.3 layouts at relation (uint, bitset), set and block
    (composite) level: (1) batches of pairs of sets whose members lie partly
    in one shared dense region (the dense-region sweep of Figure 5); (2)
    triangle counting of R-MAT s20 as one pairwise intersection per oriented
    edge under each layout (the level comparison of Table 4), beside the
    staged kernel."""
    from paper_1503_02368_amd import inputs
    sweep = []
    for frac in w["fracs"]:
        sp = inputs.dense_region_sets(w["n_pairs"], w["size"], frac, domain=w["domain"],
                                      density=w["density"], seed=w["seed"])
        expect = None
        extra = {"dense_frac": frac}
        if not args.no_cpu:
            import oracle
            t0 = time.perf_counter()
            expect, _ = oracle.pair_intersections(sp.off, sp.members, sp.pairs)
            extra["oracle_s"] = time.perf_counter() - t0
        sweep += _layout_rows(ctx, eh, torch, sp.off, sp.members, sp.pairs, args, expect, 32.0,
                              extra, w.get("layouts", SET_LAYOUTS))
        del sp
    levels_out = None
    if w.get("levels", True):
        levels_out = _levels_rmat(name, w, args, ctx, eh, torch)
    head = [r for r in sweep if r["dense_frac"] == 0.5 and r["layout"] == "composite"][0]
    res = {
        "metric": "set members intersected per second (composite layout, half of each set dense)",
        "value": head["members_per_s"], "unit": "members/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic (seeded generator)",
        "config": {"workload": name, "n_pairs": w["n_pairs"], "size": w["size"],
                   "domain": w["domain"], "density": w["density"], "seed": w["seed"],
                   "block_ids": 256},
        "dense_region_sweep": sweep,
        "levels_rmat_triangles": levels_out,
        "all_correct": (all(r["correct"] for r in sweep)
                        and (levels_out is None or all(r["correct"] for r in levels_out["rows"])))
                       if not args.no_cpu else None,
    }
    # roofline of the reported cell: each set is in one pair, so a launch reads
    # every stored segment, member and word once, plus the pair list
    gbs = head["bytes_per_launch"] / (head["ms"] / 1e3) / 1e9
    traffic = measured_traffic("composite_half", SETS_SRC) if head["dense_frac"] == 0.5 else None
    res["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                       "bytes_per_launch": head["bytes_per_launch"]}
    if "oracle_s" in head:
        import oracle
        touched = head["members_per_s"] * head["ms"] / 1e3
        res["cpu_baseline"] = {"value": touched / head["oracle_s"], "unit": "members/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": "the whole cell (every pair, two-pointer merges)"}
    return res


def _levels_rmat(name, w, args, ctx, eh, torch):
    """Triangle counting of R-MAT as one pairwise intersection per oriented
    edge under each layout, beside the staged kernel."""
    from paper_1503_02368_amd import inputs
    # triangle counting as pairwise intersections of out-sets
    el = inputs.rmat(w["scale"], w["edge_factor"], seed=w["graph_seed"])
    tuned = load_tuning("rmat20_triangles")
    base = dict(ctx.get_tuning())
    base.update(tuned.get("tuning", {}))
    ctx.set_tuning(**base)
    tau = tuned.get("tau", 32.0)
    trie = ctx.build_edgelist(el, layout=tuned.get("layout", 1), tau=tau)
    staged_ms, t_count = _time_counts(ctx, torch, trie, 3, args.steps, args.warmup)
    h = trie.host_arrays()
    trie.free()
    off = h["row"].astype(np.uint64)
    rows_u = np.repeat(np.arange(off.size - 1, dtype=np.uint32), np.diff(off.astype(np.int64)))
    pairs = np.stack([rows_u, h["col"]], axis=1)
    m_plus = int(pairs.shape[0])
    levels = _layout_rows(ctx, eh, torch, off, h["col"], pairs, args, t_count, tau,
                          {"graph": f"rmat{w['scale']}"})
    for r in levels:
        r["edges_per_s"] = m_plus / (r["ms"] / 1e3)
        r["vs_staged"] = r["ms"] / staged_ms
    log(f"[bench] staged kernel on the same graph: {staged_ms:.3f} ms")
    return {"staged_ms": staged_ms, "count": t_count, "tau": tau, "rows": levels}


def serve_run(ctx, eh, trie, reqs, mode, policy=0, deadline_s=None):
    """Replays the arrival schedule; returns per-request latency (s), counts
    and whether each request was served.  deadline_s (serial only): requests
    not started by then are left unserved, their latency taken at that time."""
    n = len(reqs)
    lat = [0.0] * n
    counts = [0] * n
    done = [True] * n
    if mode == "serial":
        start = time.monotonic()
        for i, r in enumerate(reqs):
            due = start + r.t_arrival
            now = time.monotonic()
            if deadline_s is not None and now - start > deadline_s:
                for j in range(i, n):
                    done[j] = False
                    lat[j] = max(0.0, now - (start + reqs[j].t_arrival))
                break
            if now < due:
                time.sleep(due - now)
            counts[i] = ctx.count_rooted(trie, r.pattern, r.roots)
            lat[i] = time.monotonic() - due
        return lat, counts, done
    srv = ctx.server(trie, policy=policy)
    tickets = [None] * n
    start_ns = [0]
    submitted = threading.Event()

    def submitter():
        start_ns[0] = time.monotonic_ns()
        for i, r in enumerate(reqs):
            due = start_ns[0] + int(r.t_arrival * 1e9)
            now = time.monotonic_ns()
            if now < due:
                time.sleep((due - now) / 1e9)
            while True:
                try:
                    tickets[i] = srv.submit(r.pattern, r.roots)
                    break
                except eh.EHError as e:
                    if e.status != eh.EH_EBUSY:
                        raise
                    time.sleep(50e-6)
        submitted.set()

    th = threading.Thread(target=submitter)
    th.start()
    # completions arrive through the server's completion queue; a ticket can
    # come back before the submitter thread has recorded it, so results are
    # matched to requests lazily
    by_ticket = {}
    results = {}
    recorded = 0  # requests are submitted in order
    left = n
    last = time.monotonic()
    while left:
        if time.monotonic() - last > 120.0:
            srv.close()
            raise RuntimeError(f"served run made no progress for 120 s ({left} pending)")
        for t, res in srv.drain(1024, 20):
            results[t] = res
            last = time.monotonic()
        while recorded < n and tickets[recorded] is not None:
            by_ticket[tickets[recorded]] = recorded
            recorded += 1
        for t in [t for t in results if t in by_ticket]:
            res = results.pop(t)
            i = by_ticket[t]
            due = start_ns[0] + int(reqs[i].t_arrival * 1e9)
            lat[i] = (res.t_done_ns - due) / 1e9
            counts[i] = res.count
            left -= 1
    th.join()
    srv.close()
    return lat, counts, done
