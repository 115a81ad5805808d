"""Autotuner: picks the layout and kernel knobs per workload by measurement.

The paper's lower-bound "oracle optimizer" (section 4.4) ran every layout and
algorithm combination and kept the best; this tuner does the same over the
knobs of this engine, per workload, on the real GPU: set layout (uint only,
or the set optimizer at several tau), kernel (staged or pairwise), staging
side, bitset use, work-item size, persistent waves per CU, schedule, and for
the pairwise kernel lanes per pair, algorithm and the galloping ratio gamma.
The set optimizer's threshold tau and its added floor s_min (a set takes the
bitset layout only with at least s_min members) are searched with the layout.
Graph and batch workloads are timed per launch; the served workload by the
time a server takes to answer a burst of its request mix.

Counts never depend on these choices.  Every candidate's counts must equal
the reference -- the expected count when the caller supplies one (--expect,
for instance the CPU oracle's count of the workload), else the first
candidate's -- or the search stops with an error.  The winner is then built
again from scratch with its layout and counted once more; that count must
also equal the reference, and the tuning.json entry records which reference
it was checked against.

    python -m paper_1503_02368_amd.autotune --workload rmat20_triangles [--expect T] --out tuning.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning.json")

BASE = dict(kernel=1, staging=2, algo=0, gamma=32.0, chunk_work=4096, waves_per_cu=32,
            group_lanes=0, use_bitsets=1, dynamic=0, stage_words=0, xcds=0, unroll=8, grab=8,
            search_below=24, group=1, reverse=0, k4_local=1)
# schedules tried last: (dynamic, grab); 3 and 4 cut the items into one range per XCD,
# 5 deals items sorted by decreasing cost boustrophedon
SCHEDULES = [(1, 8), (2, 8), (3, 8), (4, 1), (4, 4), (4, 16), (5, 8)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Timer:
    def __init__(self, ctx, torch):
        self.ctx = ctx
        self.torch = torch
        self.out = torch.zeros(1, dtype=torch.int64, device="cuda")

    def graph(self, trie, pattern, reps=5):
        """(ms per launch, count) of `reps` accumulating launches after one warm-up."""
        torch, ctx, out = self.torch, self.ctx, self.out
        s = ctx.stream
        s.wait_stream(torch.cuda.current_stream())
        ctx.count_add_async(trie, pattern, out)   # warm-up (also builds the plan)
        torch.cuda.synchronize()
        out.zero_()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            ctx.count_add_async(trie, pattern, out)
        e1.record(s)
        torch.cuda.synchronize()
        total = int(out.cpu().numpy().view(np.uint64)[0])
        count, rem = divmod(total, reps)
        if rem:
            raise RuntimeError("accumulated count is not a multiple of the launch count")
        return e0.elapsed_time(e1) / reps, count


class Search:
    """Candidates and their times; every count must equal the reference: the
    caller's expected count when given, else the first candidate's."""

    def __init__(self, expect=None):
        self.ref = expect
        self.checked = "expected" if expect is not None else "first candidate"
        self.best = None
        self.table = []

    def record(self, cfg, ms, count):
        if self.ref is None:
            self.ref = count
        elif count != self.ref:
            raise RuntimeError(f"count {count} differs from the reference {self.ref} under {cfg}")
        self.table.append((ms, cfg))
        if self.best is None or ms < self.best[0]:
            self.best = (ms, cfg)
        log(f"[tune] {ms:8.3f} ms  {cfg}")


def tune_graph(el, pattern, layouts, ctx, torch, quick=False, expect=None):
    from paper_1503_02368_amd import eh
    timer = Timer(ctx, torch)
    S = Search(expect)
    for layout, tau, s_min in layouts:
        trie = ctx.build_edgelist(el, layout=layout, tau=tau, s_min=s_min)
        has_bits = trie.info["n_bitset_sets"] > 0
        try:
            kinds = [dict(kernel=1, staging=2), dict(kernel=1, staging=1)] if pattern == 3 else \
                [dict(kernel=1, staging=1), dict(kernel=1, staging=1, k4_local=0)]
            if pattern == 3:
                kinds.append(dict(kernel=2, group_lanes=0, algo=0))
            local = None
            for k, ub in itertools.product(kinds, [1, 0] if has_bits else [0]):
                cfg = dict(BASE, **k, use_bitsets=ub)
                ctx.set_tuning(**cfg)
                ms, c = timer.graph(trie, pattern)
                S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
                if local is None or ms < local[0]:
                    local = (ms, cfg)
            # refine the schedule of the best kernel on this layout
            chunks = [1024, 4096, 16384] if quick else [1024, 2048, 4096, 8192, 16384, 32768, 65536]
            waves = [16, 32] if quick else [8, 16, 24, 32, 40]
            words = [0, 512]
            unrolls = [4, 8] if pattern == 3 and local[1]["kernel"] == 1 else [8]
            for ch, wv, sw, un in itertools.product(chunks, waves, words, unrolls):
                cfg = dict(local[1], chunk_work=ch, waves_per_cu=wv, stage_words=sw, unroll=un)
                ctx.set_tuning(**cfg)
                ms, c = timer.graph(trie, pattern)
                S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
                if local is None or ms < local[0]:
                    local = (ms, cfg)
            for dyn, grab in SCHEDULES:
                cfg = dict(local[1], dynamic=dyn, grab=grab)
                ctx.set_tuning(**cfg)
                ms, c = timer.graph(trie, pattern)
                S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
                if ms < local[0]:
                    local = (ms, cfg)
            # the same schedule dealing the items from the last to the first
            cfg = dict(local[1], reverse=1)
            ctx.set_tuning(**cfg)
            ms, c = timer.graph(trie, pattern)
            S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
            if ms < local[0]:
                local = (ms, cfg)
            if local[1]["kernel"] == 1:
                for sb in (12, 16, 32, 48):
                    cfg = dict(local[1], search_below=sb)
                    ctx.set_tuning(**cfg)
                    ms, c = timer.graph(trie, pattern)
                    S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
                    if ms < local[0]:
                        local = (ms, cfg)
            if pattern == 3 and local[1]["kernel"] == 1 and local[1]["staging"] == 2:
                for grp, sw in itertools.product((2, 4), (0, 512)):
                    cfg = dict(local[1], group=grp, stage_words=sw)
                    ctx.set_tuning(**cfg)
                    ms, c = timer.graph(trie, pattern)
                    S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
            if local[1]["kernel"] == eh.KERNEL_PAIRWISE:
                for g, al, gm in itertools.product([4, 16, 64], [0, 1, 2], [8.0, 32.0, 128.0]):
                    cfg = dict(local[1], group_lanes=g, algo=al, gamma=gm)
                    ctx.set_tuning(**cfg)
                    ms, c = timer.graph(trie, pattern)
                    S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
        finally:
            trie.free()
    return S


def tune_batch(b, pattern, layouts, ctx, torch, quick=False, expect=None):
    """expect: the per-graph counts (uint64 array), or None."""
    S = Search(None if expect is None else tuple(int(x) for x in expect))
    G = b.n_graphs
    out = torch.zeros(G, dtype=torch.int64, device="cuda")
    for layout, tau, s_min in layouts:
        trie = ctx.build_batch(b, layout=layout, tau=tau, s_min=s_min)
        def run(cfg):
            ctx.set_tuning(**cfg)
            s = ctx.stream
            ctx.count_batch_async(trie, pattern, 0, G, out)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(3):
                ctx.count_batch_async(trie, pattern, 0, G, out)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            c = tuple(int(x) for x in out.cpu().numpy().view(np.uint64))
            S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, c)
            return ms

        try:
            chunks = [1024, 4096] if quick else [512, 1024, 2048, 4096, 8192, 16384]
            kinds = [dict(staging=2), dict(staging=1)]
            groups = (8,) if quick else (4, 8, 16)
            kinds += [dict(kernel=2, group_lanes=g, algo=al) for g in groups for al in (0, 1)]
            local = None
            for k, ch, (dyn, grab) in itertools.product(kinds, chunks, [(0, 8), (4, 16)]):
                cfg = dict(BASE, **k, chunk_work=ch, dynamic=dyn, grab=grab,
                           group=4 if k.get("staging") == 2 else 1)
                ms = run(cfg)
                if local is None or ms < local[0]:
                    local = (ms, cfg)
            unrolls = [4, 8] if local[1]["kernel"] == 1 else [8]
            words = [0, 512] if local[1]["kernel"] == 1 else [0]
            groups = [1, 2, 4] if local[1]["group"] > 1 else [1]
            for wv, un, sw, gr, (dyn, grab) in itertools.product([24, 32, 40], unrolls, words, groups,
                                                                  [(0, 8), (4, 4), (4, 16), (4, 64)]):
                cfg = dict(local[1], waves_per_cu=wv, unroll=un, stage_words=sw, group=gr,
                           dynamic=dyn, grab=grab)
                ms = run(cfg)
                if ms < local[0]:
                    local = (ms, cfg)
            if local[1]["kernel"] == 1:
                for sb in (12, 16, 32, 48):
                    run(dict(local[1], search_below=sb))
        finally:
            trie.free()
    return S


def served_requests(w, n, quick=False):
    """The request burst the served workload is tuned on."""
    from paper_1503_02368_amd import inputs
    return inputs.request_stream(n, rate_qps=5000, duration_s=0.25 if quick else 0.5,
                                 seed=w["seed"] + 1)


def tune_served(w, ctx, torch, quick=False, expect=None, el=None):
    """Served workload: the time to answer a burst of the benchmark's request
    mix (every request submitted at once) through one server per setting.
    expect: the per-request counts, or None."""
    from paper_1503_02368_amd import inputs
    if el is None:
        el = inputs.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
    reqs = served_requests(w, el.n, quick)
    S = Search(None if expect is None else tuple(int(x) for x in expect))
    for layout, tau, s_min in [(1, 32.0, 1)] if quick else [(1, 32.0, 1), (1, 256.0, 1), (1, 32.0, 16)]:
        trie = ctx.build_edgelist(el, layout=layout, tau=tau, s_min=s_min)

        def run(cfg):
            ctx.set_tuning(**cfg)
            srv = ctx.server(trie)
            try:
                t0 = time.perf_counter()
                tickets = [srv.submit(r.pattern, r.roots) for r in reqs]
                counts = tuple(srv.wait(t).count for t in tickets)
                ms = (time.perf_counter() - t0) * 1e3
            finally:
                srv.close()
            S.record(dict(layout=layout, tau=tau, s_min=s_min, tuning=cfg), ms, counts)
            return ms

        try:
            local = None
            for ch, sw, (dyn, grab) in itertools.product([4096, 32768, 131072], [0, 512],
                                                        [(0, 8), (4, 1), (4, 4)]):
                cfg = dict(BASE, staging=1, chunk_work=ch, stage_words=sw, dynamic=dyn, grab=grab)
                ms = run(cfg)
                if local is None or ms < local[0]:
                    local = (ms, cfg)
            for wv, un in itertools.product([24, 32, 40], [4, 8]):
                run(dict(local[1], waves_per_cu=wv, unroll=un))
        finally:
            trie.free()
    return S


def layouts_for(w, quick=False):
    """(layout, tau, s_min) candidates: the set optimizer at several tau, and
    its s_min floor at 1 (the paper's rule), 16 and 64."""
    if w["layout"] == 0:
        return [(0, 32.0, 1)]           # the workload fixes the uint-only layout
    if quick:
        return [(1, 32.0, 1), (1, 256.0, 1), (1, 256.0, 16)]
    return [(0, 32.0, 1), (1, 8.0, 1), (1, 32.0, 1), (1, 256.0, 1), (1, 32.0, 16),
            (1, 256.0, 16), (1, 256.0, 64)]


def verify(kind, w, data, cfg, pattern, ctx, torch, ref, quick=False):
    """Builds the winner's trie from scratch and counts once more with its
    tuning; returns the counts in the form of the search's reference."""
    ctx.set_tuning(**cfg["tuning"])
    if kind == "graph":
        trie = ctx.build_edgelist(data, layout=cfg["layout"], tau=cfg["tau"], s_min=cfg["s_min"])
        try:
            return Timer(ctx, torch).graph(trie, pattern, reps=1)[1]
        finally:
            trie.free()
    if kind == "batch":
        trie = ctx.build_batch(data, layout=cfg["layout"], tau=cfg["tau"], s_min=cfg["s_min"])
        try:
            return tuple(int(x) for x in ctx.count_batch(trie, pattern))
        finally:
            trie.free()
    trie = ctx.build_edgelist(data, layout=cfg["layout"], tau=cfg["tau"], s_min=cfg["s_min"])
    try:
        srv = ctx.server(trie)
        try:
            tickets = [srv.submit(r.pattern, r.roots) for r in served_requests(w, data.n, quick)]
            return tuple(srv.wait(t).count for t in tickets)
        finally:
            srv.close()
    finally:
        trie.free()


def tune_workload(name, w, ctx, torch, quick=False, expect=None, data=None):
    """Searches one workload and returns its tuning.json entry.  data replaces
    the workload's generated input (a graph, or a batch for batch workloads);
    expect is the reference count: an integer for a graph, per-graph counts
    for a batch, per-request counts for the served burst."""
    from paper_1503_02368_amd.workloads import make_batch, make_graph
    from paper_1503_02368_amd import inputs
    t0 = time.time()
    kind = w["kind"]
    if kind == "batch":
        data = make_batch(w) if data is None else data
        S = tune_batch(data, w["pattern"], layouts_for(w, quick), ctx, torch, quick, expect)
    elif kind == "graph":
        data = make_graph(w) if data is None else data
        S = tune_graph(data, w["pattern"], layouts_for(w, quick), ctx, torch, quick, expect)
    elif kind == "served":
        if data is None:
            data = inputs.rmat(w["scale"], w["edge_factor"], seed=w["seed"])
        S = tune_served(w, ctx, torch, quick, expect, el=data)
    else:
        raise ValueError(f"workload kind {kind} is not tuned")
    ms, cfg = S.best
    again = verify(kind, w, data, cfg, w.get("pattern", 3), ctx, torch, S.ref, quick)
    if again != S.ref:
        raise RuntimeError(f"{name}: the winner rebuilt from scratch counts {again}, "
                           f"not the reference {S.ref}")
    log(f"[tune] {name}: best {ms:.3f} ms with {cfg}; rebuilt and checked against the "
        f"{S.checked} count")
    return {"layout": cfg["layout"], "tau": cfg["tau"], "s_min": cfg["s_min"],
            "tuning": cfg["tuning"], "ms": ms, "candidates": len(S.table),
            "count": sum(S.ref) if isinstance(S.ref, tuple) else S.ref,
            "checked_against": S.checked, "searched_s": round(time.time() - t0, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", action="append", required=True)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--expect", type=int, default=None,
                    help="reference count of a single graph workload (e.g. the CPU oracle's)")
    args = ap.parse_args()
    if args.expect is not None and len(args.workload) != 1:
        ap.error("--expect needs exactly one --workload")
    import torch
    from paper_1503_02368_amd import eh
    from paper_1503_02368_amd.workloads import WORKLOADS
    ctx = eh.Context(0)
    # entries of other workloads are kept: from --out if it exists, else
    # from the package's tuning.json
    result = {}
    for src in (args.out, DEFAULT_OUT):
        if os.path.exists(src):
            with open(src) as f:
                result = json.load(f)
            break
    for name in args.workload:
        w = WORKLOADS[name]
        if w["kind"] not in ("graph", "batch", "served"):
            continue
        result[name] = tune_workload(name, w, ctx, torch, args.quick, args.expect)
        with open(args.out, "w") as f:
            json.dump(result, f, indent=1, sort_keys=True)
    ctx.close()


if __name__ == "__main__":
    main()
