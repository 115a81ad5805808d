"""GPU parity: every count from the HIP library equals the oracle's, bit for bit.

Counts are exact integers, so the bar is equality.  Layout (uint, hybrid,
all-bitset), kernel (staged, pairwise), staging side, intersection algorithm
and schedule are performance choices only (paper section 4); each is forced
here and must give the same count.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import inputs
from golden_io import all_fixtures, load

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(eh):
    c = eh.Context(0)
    yield c
    c.close()


def zoo():
    g = [inputs.complete(n) for n in (3, 4, 5, 17, 70)]
    g += [inputs.cycle(3), inputs.cycle(4), inputs.cycle(50), inputs.grid(6, 7), inputs.star(30),
          inputs.wheel(4), inputs.wheel(33), inputs.friendship(9), inputs.complete_bipartite(5, 8),
          inputs.random_tree(200, 1)]
    for p in all_fixtures():
        n, s, d, _ = load(p)
        g.append(inputs.EdgeList(n, s, d, p.rsplit("/", 1)[-1]))
    g += [inputs.gnp(40, p, s) for p in (0.2, 0.6, 0.95) for s in (1, 2)]
    g += [inputs.erdos_renyi_gnm(4096, 32768, seed=1)]
    g += [inputs.rmat(s, 16, seed=100 + s) for s in (8, 10, 12)]
    g += [inputs.messy(inputs.rmat(9, 16, seed=7), 3), inputs.relabel(inputs.rmat(10, 8, seed=8), 4)]
    g += [inputs.chung_lu(5000, 32, 2.1, seed=2, graph=1)]
    g += [inputs.disjoint_union(inputs.complete(30), inputs.rmat(9, 16, seed=9), inputs.wheel(12))]
    return g


ZOO = zoo()
_ORACLE = {}


def truth(el):
    key = el.name
    if key not in _ORACLE:
        g = oracle.Graph.from_edgelist(el)
        t = g.triangles(rooted=True)
        k = g.cliques4()
        _ORACLE[key] = (t["count"], k["count"], t["root"])
    return _ORACLE[key]


TUNINGS = {
    "staged_target": dict(kernel=1, staging=2, use_bitsets=1, dynamic=0, stage_words=0),
    "staged_source": dict(kernel=1, staging=1, use_bitsets=1, dynamic=1, stage_words=0),
    "staged_nobits": dict(kernel=1, staging=2, use_bitsets=0, dynamic=2, stage_words=0),
    "staged_half": dict(kernel=1, staging=1, use_bitsets=1, dynamic=2, stage_words=512),
    "staged_list": dict(kernel=1, staging=2, use_bitsets=1, dynamic=0, stage_words=8),
    "staged_global": dict(kernel=1, staging=1, use_bitsets=1, dynamic=1, stage_words=1),
    "pair_auto": dict(kernel=2, algo=0, use_bitsets=1, group_lanes=0, dynamic=0),
    "pair_merge4": dict(kernel=2, algo=1, use_bitsets=0, group_lanes=4, dynamic=1),
    "pair_search16": dict(kernel=2, algo=2, use_bitsets=0, group_lanes=16, dynamic=2),
    "pair_merge64": dict(kernel=2, algo=1, use_bitsets=1, group_lanes=64, dynamic=0),
    # partitioned schedules: 8 ranges interleaved per L2 domain; 5 ranges with
    # cursors taking 3 items per fetch (ranges of unequal size, stealing)
    "staged_part": dict(kernel=1, staging=2, use_bitsets=1, dynamic=3, xcds=0),
    "staged_steal": dict(kernel=1, staging=1, use_bitsets=1, dynamic=4, xcds=5, grab=3),
    "pair_steal": dict(kernel=2, algo=0, use_bitsets=1, group_lanes=8, dynamic=4, xcds=8, grab=1),
    # every streamed element's set found by binary search, or never
    "staged_search": dict(kernel=1, staging=2, use_bitsets=1, search_below=4096),
    "staged_search_src": dict(kernel=1, staging=1, use_bitsets=1, search_below=4096, stage_words=512),
    "staged_walk": dict(kernel=1, staging=2, use_bitsets=1, search_below=0),
    # half-size staged region: the 8-waves-per-SIMD triangle instance
    "staged_lean": dict(kernel=1, staging=2, use_bitsets=1, stage_words=512, dynamic=4, grab=5),
    # small items grouped 4 (or 2) to a wave, interleaved bitmaps
    "staged_group": dict(kernel=1, staging=2, use_bitsets=1, group=4, dynamic=4, grab=3),
    "staged_group_lean": dict(kernel=1, staging=2, use_bitsets=1, group=2, stage_words=512,
                              search_below=0),
    # items dealt from the last to the first
    "staged_reverse": dict(kernel=1, staging=2, use_bitsets=1, stage_words=512, dynamic=4, grab=2,
                           reverse=1),
    "staged_source_rev": dict(kernel=1, staging=1, use_bitsets=1, dynamic=0, reverse=1),
    # items sorted by decreasing estimated cost, dealt boustrophedon
    "staged_snake": dict(kernel=1, staging=2, use_bitsets=1, stage_words=512, dynamic=5),
    "staged_source_snake": dict(kernel=1, staging=1, use_bitsets=1, dynamic=5, chunk_work=512),
    "staged_group_snake": dict(kernel=1, staging=2, use_bitsets=1, group=4, dynamic=5),
}
DEFAULT = dict(kernel=1, staging=2, algo=0, gamma=32.0, chunk_work=4096, waves_per_cu=32,
               group_lanes=0, use_bitsets=1, dynamic=0, stage_words=0, xcds=0, unroll=8, grab=8,
               search_below=24, group=1, reverse=0, k4_local=1)


def tune(ctx, **kw):
    t = dict(DEFAULT)
    t.update(kw)
    ctx.set_tuning(**t)


LAYOUTS = [("hybrid32", 1, 32.0), ("uint", 0, 32.0), ("bitset_all", 2, 32.0), ("hybrid256", 1, 256.0),
           ("hybrid2", 1, 2.0)]


@pytest.mark.parametrize("lay", LAYOUTS, ids=lambda x: x[0])
@pytest.mark.parametrize("tname", list(TUNINGS))
def test_triangles_zoo(ctx, eh, tname, lay):
    tune(ctx, **TUNINGS[tname])
    for el in ZOO:
        T, _, _ = truth(el)
        trie = ctx.build_edgelist(el, layout=lay[1], tau=lay[2])
        try:
            got = ctx.count_triangles(trie)
        finally:
            trie.free()
        assert got == T, (el.name, tname, lay[0])


@pytest.mark.parametrize("lay", LAYOUTS[:3], ids=lambda x: x[0])
@pytest.mark.parametrize("tname", ["staged_source", "staged_nobits", "staged_list", "staged_global",
                                   "staged_half", "staged_steal", "staged_search_src",
                                   "staged_source_rev", "staged_source_snake"])
def test_4cliques_zoo(ctx, eh, tname, lay):
    tune(ctx, **TUNINGS[tname])
    for el in ZOO:
        _, K, _ = truth(el)
        trie = ctx.build_edgelist(el, layout=lay[1], tau=lay[2])
        try:
            got = ctx.count_4cliques(trie)
        finally:
            trie.free()
        assert got == K, (el.name, tname, lay[0])


def _k4_local_graphs():
    """Roots in every out-degree class of the induced-neighbourhood kernel
    (<= 128, <= 256, <= 512) and just beyond it (513), out-sets spanning more
    ids than its window, sinks and messy input."""
    star_of_cliques = inputs.disjoint_union(*[inputs.complete(6) for _ in range(4000)])
    # one vertex adjacent to a member of every clique: its out-set spans the ids
    hub = star_of_cliques.n
    src = np.concatenate([star_of_cliques.src, np.full(4000, hub, np.uint32)])
    dst = np.concatenate([star_of_cliques.dst, np.arange(0, 24000, 6, dtype=np.uint32)])
    spread = inputs.EdgeList(hub + 1, src, dst, "hub_over_4000_K6")
    return [inputs.complete(130), inputs.complete(257), inputs.complete(513), inputs.complete(514),
            inputs.disjoint_union(inputs.complete(200), inputs.rmat(12, 16, seed=81),
                                  inputs.complete(40)),
            inputs.rmat(14, 16, seed=82), inputs.gnp(3000, 0.05, seed=83),
            inputs.chung_lu(40000, 24, 2.1, seed=84), spread,
            inputs.messy(inputs.rmat(11, 16, seed=85), 3)]


@pytest.mark.parametrize("lay", [("uint", 0, 32.0), ("hybrid256", 1, 256.0), ("bitset_all", 2, 32.0)],
                         ids=lambda x: x[0])
def test_4cliques_induced_neighbourhoods(ctx, eh, lay):
    """4-cliques with roots counted over their induced out-neighbourhoods
    (k4_local = 1) equal the oracle's and the staged S-list kernel's
    (k4_local = 0), with and without streamed bitset words, under two
    schedules of the roots the first leaves to the second."""
    from math import comb
    for el in _k4_local_graphs():
        # complete graphs by the closed form C(n, 4), the rest by the oracle
        K = comb(el.n, 4) if el.name == f"K{el.n}" else oracle.Graph.from_edgelist(el).count(4)
        say("k4 local", lay[0], el.name, K)
        trie = ctx.build_edgelist(el, layout=lay[1], tau=lay[2])
        try:
            for kw in (dict(k4_local=1, staging=1, dynamic=0), dict(k4_local=1, use_bitsets=0),
                       dict(k4_local=1, dynamic=4, grab=2, chunk_work=512),
                       dict(k4_local=0, staging=1, dynamic=4, grab=2)):
                tune(ctx, **kw)
                assert ctx.count_4cliques(trie) == K, (el.name, kw)
        finally:
            trie.free()


def test_4cliques_induced_window_spill(ctx, eh):
    """Roots of out-degree 257..512 whose out-sets span more ids than the
    eight-wave class's 16,384-id window (a near-regular graph of 20,000
    vertices and mean degree 640: about 13.5 K such roots, a quarter of them
    with members below the window), counted whole and rooted (the items
    path), equal the oracle's."""
    el = inputs.chung_lu(20000, 640, 6.0, seed=86)
    g = oracle.Graph.from_edgelist(el)
    root = g.cliques4_rooted_at(np.arange(el.n, dtype=np.uint32))
    K = int(root.sum(dtype=np.uint64))
    assert K == g.count(4)
    trie = ctx.build_edgelist(el)
    try:
        assert 256 < trie.info["max_out_degree"] <= 512
        for kw in (dict(k4_local=1, staging=1, dynamic=0), dict(k4_local=1, use_bitsets=0)):
            tune(ctx, **kw)
            assert ctx.count_4cliques(trie) == K, kw
        tune(ctx, k4_local=1)
        sample = np.random.default_rng(7).choice(el.n, 3000, replace=False).astype(np.uint32)
        assert ctx.count_rooted(trie, eh.CLIQUE4, sample) == oracle.rooted_count(root, sample)
    finally:
        trie.free()


def test_4cliques_induced_accumulate_and_noalloc(ctx, eh):
    """The accumulating and allocation-free counts run both 4-clique launches
    of a plan whose roots are split between them."""
    import torch
    el = inputs.disjoint_union(inputs.complete(600), inputs.rmat(12, 16, seed=86))
    K = oracle.Graph.from_edgelist(el).count(4)
    tune(ctx, k4_local=1, staging=1, dynamic=4, grab=2)
    trie = ctx.build_edgelist(el)
    try:
        assert ctx.count_4cliques(trie) == K
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.stream.wait_stream(torch.cuda.current_stream())
        ctx.count_add_async(trie, eh.CLIQUE4, out)
        ctx.count_add_noalloc(trie, eh.CLIQUE4, out)
        torch.cuda.synchronize()
        assert int(out.cpu().numpy().view(np.uint64)[0]) == 2 * K
    finally:
        trie.free()


@pytest.mark.parametrize("dyn", [0, 4])
def test_4cliques_high_out_degree(ctx, eh, dyn):
    """Out-degrees above 512 and 1024, the S-list sizes of the 4-clique kernel
    instances: items whose root has a longer out-list run in a second launch.
    Complete graphs are pinned by closed forms (K = C(n, 4); all degrees tie,
    so rank = id and vertex i roots C(n-1-i, 3) 4-cliques); a disjoint union
    with a sparse graph adds the oracle's counts for the sparse part."""
    from math import comb
    tune(ctx, kernel=1, staging=1, dynamic=dyn, grab=2)
    for n in (600, 1100):
        trie = ctx.build_edgelist(inputs.complete(n))
        try:
            assert trie.info["max_out_degree"] == n - 1
            assert ctx.count_4cliques(trie) == comb(n, 4)
            roots = np.array([0, 1, 300, n // 2, n - 4, n - 1], np.uint32)  # a set: 300 may repeat
            want = sum(comb(n - 1 - int(i), 3) for i in np.unique(roots))
            assert ctx.count_rooted(trie, eh.CLIQUE4, roots) == want
        finally:
            trie.free()
    sparse = inputs.rmat(9, 16, seed=9)
    gs = oracle.Graph.from_edgelist(sparse).cliques4(rooted=True)
    k = 600
    un = inputs.disjoint_union(inputs.complete(k), sparse)
    trie = ctx.build_edgelist(un)
    srv = None
    try:
        assert ctx.count_4cliques(trie) == comb(k, 4) + gs["count"]

        def want(roots):
            return sum(comb(k - 1 - int(i), 3) if i < k else int(gs["root"][i - k]) for i in roots)

        key = inputs.stream_key(11, 3)
        sets = [np.array([0, 5, 599, 600, 601], np.uint32),
                (inputs.rand_u64(key, 0, 300) % np.uint64(un.n)).astype(np.uint32),
                np.arange(k, un.n, dtype=np.uint32), np.arange(0, 40, dtype=np.uint32)]
        for r in sets:
            assert ctx.count_rooted(trie, eh.CLIQUE4, r) == want(np.unique(r))
        srv = ctx.server(trie, step_items=512)
        tickets = [srv.submit(eh.CLIQUE4, r) for r in sets]
        for t, r in zip(tickets, sets):
            assert srv.wait(t).count == want(np.unique(r))
    finally:
        if srv is not None:
            srv.close()
        trie.free()


@pytest.mark.parametrize("tname", ["staged_source", "pair_auto", "staged_global"])
def test_per_root(ctx, eh, tname):
    tune(ctx, **TUNINGS[tname])
    for el in ZOO[-6:]:
        T, _, root = truth(el)
        trie = ctx.build_edgelist(el)
        try:
            tot, per = ctx.count_triangles(trie, per_root=True)
        finally:
            trie.free()
        assert tot == T
        np.testing.assert_array_equal(per, root)


@pytest.mark.parametrize("chunk", [64, 700, 100000])
def test_chunking_and_grid(ctx, eh, chunk):
    el = inputs.rmat(13, 16, seed=31)
    T, K, _ = truth(el)
    for wpc, dyn in ((4, 0), (32, 0), (1, 3), (1, 4), (32, 4)):
        for staging in (1, 2):
            tune(ctx, chunk_work=chunk, waves_per_cu=wpc, staging=staging, dynamic=dyn)
            trie = ctx.build_edgelist(el)
            try:
                assert ctx.count_triangles(trie) == T
                assert ctx.count_4cliques(trie) == K
            finally:
                trie.free()


def test_async_and_repeat(ctx, eh):
    import torch
    tune(ctx)
    el = inputs.rmat(14, 16, seed=14)
    T, K, _ = truth(el)
    trie = ctx.build_edgelist(el)
    try:
        out = torch.zeros(4, dtype=torch.int64, device="cuda")
        ctx.stream.wait_stream(torch.cuda.current_stream())
        for i in range(3):
            ctx.count_async(trie, eh.TRIANGLE, out[i:i + 1])
        ctx.count_async(trie, eh.CLIQUE4, out[3:4])
        ctx.stream.synchronize()
        v = out.cpu().numpy().view(np.uint64)
        assert list(v) == [T, T, T, K]
    finally:
        trie.free()


@pytest.mark.parametrize("k4l", [1, 0])
def test_rooted(ctx, eh, k4l):
    """Rooted counts; 4-clique roots of out-degree <= 512 by induced
    neighbourhoods (k4_local = 1) or all by the S-list kernel."""
    tune(ctx, k4_local=k4l)
    el = inputs.rmat(12, 16, seed=12)
    g = oracle.Graph.from_edgelist(el)
    rt = g.triangles(rooted=True)["root"]
    rk = g.cliques4(rooted=True)["root"]
    trie = ctx.build_edgelist(el)
    try:
        key = inputs.stream_key(3, 3)
        for i, size in enumerate((1, 7, 100, 1000, el.n)):
            roots = (inputs.rand_u64(key, 10000 * i, size) % np.uint64(el.n)).astype(np.uint32)
            assert ctx.count_rooted(trie, eh.TRIANGLE, roots) == oracle.rooted_count(rt, roots)
            assert ctx.count_rooted(trie, eh.CLIQUE4, roots) == oracle.rooted_count(rk, roots)
        allv = np.arange(el.n, dtype=np.uint32)
        assert ctx.count_rooted(trie, eh.TRIANGLE, allv) == int(rt.sum())
        with pytest.raises(eh.EHError):
            ctx.count_rooted(trie, eh.TRIANGLE, np.array([el.n], np.uint32))
        with pytest.raises(eh.EHError):
            ctx.count_rooted(trie, 5, np.array([0], np.uint32))
    finally:
        trie.free()


def small_batch(num=120, seed=4):
    return inputs.batch_chung_lu(num, seed=seed, n_hi=2048)


@pytest.mark.parametrize("tname", ["staged_target", "staged_source", "pair_auto", "staged_part",
                                   "staged_steal", "staged_search", "staged_lean", "staged_group",
                                   "staged_group_lean"])
def test_batch(ctx, eh, tname):
    tune(ctx, **TUNINGS[tname])
    b = small_batch()
    want_t = np.array([oracle.Graph.from_edgelist(b.graph(i)).triangles()["count"]
                       for i in range(b.n_graphs)], np.uint64)
    want_k = np.array([oracle.Graph.from_edgelist(b.graph(i)).cliques4()["count"]
                       for i in range(b.n_graphs)], np.uint64)
    trie = ctx.build_batch(b)
    try:
        assert trie.info["n_graphs"] == b.n_graphs
        np.testing.assert_array_equal(ctx.count_batch(trie, eh.TRIANGLE), want_t)
        np.testing.assert_array_equal(ctx.count_batch(trie, eh.CLIQUE4), want_k)
        # one launch per instance gives the same vector
        per = np.array([ctx.count_batch(trie, eh.TRIANGLE, i, 1)[0] for i in range(b.n_graphs)],
                       np.uint64)
        np.testing.assert_array_equal(per, want_t)
        np.testing.assert_array_equal(ctx.count_batch(trie, eh.TRIANGLE, 17, 40), want_t[17:57])
        with pytest.raises(eh.EHError):
            ctx.count_batch(trie, eh.TRIANGLE, b.n_graphs - 1, 2)
    finally:
        trie.free()


def test_batch_order_invariant(ctx, eh):
    tune(ctx)
    b = small_batch(60, seed=9)
    order = np.argsort(inputs.rand_u64(inputs.stream_key(1, 2), 0, b.n_graphs))
    srcs, dsts, off = [], [], [0]
    for i in order:
        g = b.graph(int(i))
        srcs.append(g.src)
        dsts.append(g.dst)
        off.append(off[-1] + g.m_raw)
    b2 = inputs.BatchEdges(b.n_vertices[order].copy(), np.array(off, np.uint64),
                           np.concatenate(srcs), np.concatenate(dsts), "perm")
    t1 = ctx.build_batch(b)
    t2 = ctx.build_batch(b2)
    try:
        a = ctx.count_batch(t1, eh.TRIANGLE)
        c = ctx.count_batch(t2, eh.TRIANGLE)
        np.testing.assert_array_equal(a[order], c)
    finally:
        t1.free()
        t2.free()


@pytest.mark.parametrize("policy,k4l", [(0, 1), (1, 1), (1, 0)])
def test_server_alone_equals_mix(ctx, eh, policy, k4l):
    """Each request alone = in the mix = the oracle's rooted count; 4-clique
    requests' roots of out-degree <= 512 by induced neighbourhoods (k4_local
    = 1: a request's items cut into the kernels' regions across steps) or
    all by the S-list kernel."""
    tune(ctx, k4_local=k4l)
    el = inputs.rmat(13, 16, seed=13)
    g = oracle.Graph.from_edgelist(el)
    roots_t = g.triangles(rooted=True)["root"]
    roots_k = g.cliques4(rooted=True)["root"]
    trie = ctx.build_edgelist(el)
    reqs = inputs.request_stream(el.n, rate_qps=1000, duration_s=0.06, seed=5, log2_lo=2, log2_hi=12)
    assert len(reqs) > 20
    want = [oracle.rooted_count(roots_t if r.pattern == 3 else roots_k, r.roots) for r in reqs]
    srv = ctx.server(trie, step_items=512, policy=policy)
    try:
        alone = []
        for r in reqs:
            t = srv.submit(r.pattern, r.roots)
            alone.append(srv.wait(t).count)
        tickets = [srv.submit(r.pattern, r.roots) for r in reqs]
        mix = [srv.wait(t).count for t in tickets]
        assert alone == want
        assert mix == want
        with pytest.raises(eh.EHError) as e:
            srv.poll(tickets[0])
        assert e.value.status == eh.EH_ENOTFOUND
    finally:
        srv.close()
    # back-pressure: a budget that holds one request at a time
    srv = ctx.server(trie, hbm_budget_bytes=1 << 16, max_active=2, step_items=64)
    try:
        small = [r for r in reqs if r.roots.size < 500][:10]
        tickets = [srv.submit(r.pattern, r.roots) for r in small]
        got = [srv.wait(t).count for t in tickets]
        assert got == [oracle.rooted_count(roots_t if r.pattern == 3 else roots_k, r.roots) for r in small]
        with pytest.raises(eh.EHError) as e:
            srv.submit(3, np.arange(el.n, dtype=np.uint32))
        assert e.value.status == eh.EH_ENOMEM
        with pytest.raises(eh.EHError):
            srv.submit(3, np.array([el.n + 5], np.uint32))
    finally:
        srv.close()
    trie.free()


def test_server_arena_first_fit(ctx, eh):
    """Admission by the HBM arena: requests of very different sizes under a
    budget a little above the largest one's items wait for extents to free up
    (first fit, merged on release) and still answer exactly; a request whose
    items exceed the arena is refused, and so is an arena of no item."""
    tune(ctx, staging=1)
    el = inputs.rmat(12, 16, seed=31)
    g = oracle.Graph.from_edgelist(el)
    rt = g.triangles(rooted=True)["root"]
    rk = g.cliques4(rooted=True)["root"]
    trie = ctx.build_edgelist(el)
    key = inputs.stream_key(31, 7)
    sizes = [int(x) for x in (inputs.rand_u64(key, 0, 40) % np.uint64(1200)) + np.uint64(1)]
    reqs = []
    for i, k in enumerate(sizes):
        roots = (inputs.rand_u64(inputs.stream_key(32, i), 0, k) % np.uint64(el.n)).astype(np.uint32)
        reqs.append((3 if i % 3 else 4, roots))
    want = [oracle.rooted_count(rt if p == 3 else rk, r) for p, r in reqs]
    everything = (4, np.arange(el.n, dtype=np.uint32))
    # the items of each request, from a server whose arena holds them all
    srv = ctx.server(trie)
    try:
        res = [srv.wait(srv.submit(p, r)) for p, r in reqs + [everything]]
    finally:
        srv.close()
    assert [x.count for x in res[:-1]] == want
    items = [x.items for x in res]
    budget = max(items[:-1]) + 3
    assert sum(items[:-1]) > 3 * budget   # most requests wait for room
    srv = ctx.server(trie, hbm_budget_bytes=16 * budget, max_active=8, step_items=300, policy=1)
    try:
        tickets = [srv.submit(p, r) for p, r in reqs]
        assert [srv.wait(t).count for t in tickets] == want
        if items[-1] > budget:
            with pytest.raises(eh.EHError) as e:
                srv.submit(*everything)
            assert e.value.status == eh.EH_ENOMEM
    finally:
        srv.close()
        trie.free()
    small = ctx.build_edgelist(inputs.complete(5))
    try:
        with pytest.raises(eh.EHError) as e:
            ctx.server(small, hbm_budget_bytes=8)
        assert e.value.status == eh.EH_EINVAL
    finally:
        small.free()


def test_full_size_rmat20_triangles(ctx, eh):
    """The measured workload: R-MAT scale 20, edge factor 16, hybrid layout."""
    tune(ctx)
    el = inputs.rmat(20, 16, seed=20)
    say("rmat20 generated")
    g = oracle.Graph.from_edgelist(el)
    T = g.triangles()["count"]
    say("oracle T", T)
    trie = ctx.build_edgelist(el)
    try:
        for tname in ("staged_target", "staged_source", "pair_auto", "staged_part", "staged_steal",
                      "staged_search", "staged_walk", "staged_lean", "staged_group",
                      "staged_group_lean"):
            tune(ctx, **TUNINGS[tname])
            got = ctx.count_triangles(trie)
            say(tname, got)
            assert got == T, tname
    finally:
        trie.free()


def test_server_drain(ctx, eh):
    """Completion-queue retrieval returns every request once, with exact counts."""
    tune(ctx)
    el = inputs.rmat(12, 16, seed=41)
    g = oracle.Graph.from_edgelist(el)
    rt = g.triangles(rooted=True)["root"]
    rk = g.cliques4(rooted=True)["root"]
    trie = ctx.build_edgelist(el)
    reqs = inputs.request_stream(el.n, rate_qps=2000, duration_s=0.05, seed=9, log2_lo=1, log2_hi=11)
    srv = ctx.server(trie, step_items=256)
    try:
        want = {}
        for r in reqs:
            t = srv.submit(r.pattern, r.roots)
            want[t] = oracle.rooted_count(rt if r.pattern == 3 else rk, r.roots)
        # one request retired by poll/wait must not come back from drain
        t0 = next(iter(want))
        assert srv.wait(t0).count == want.pop(t0)
        got = {}
        deadline = 200
        while len(got) < len(want) and deadline:
            for t, res in srv.drain(16, 50):
                assert t not in got
                got[t] = res.count
            deadline -= 1
        assert got == want
        assert srv.drain(8, 1) == []
    finally:
        srv.close()
        trie.free()


def test_server_concurrent_submitters(ctx, eh):
    """Several host threads submit and wait at once (submission only copies
    roots; expansion workers and the progress thread do the rest): every
    answer equals the oracle's."""
    import threading
    tune(ctx)
    el = inputs.rmat(12, 16, seed=43)
    g = oracle.Graph.from_edgelist(el)
    tabs = {3: g.triangles(rooted=True)["root"], 4: g.cliques4(rooted=True)["root"]}
    trie = ctx.build_edgelist(el)
    reqs = inputs.request_stream(el.n, rate_qps=4000, duration_s=0.05, seed=12, log2_lo=1, log2_hi=11)
    srv = ctx.server(trie, step_items=300)
    errors, got = [], {}

    def client(k):
        try:
            mine = reqs[k::4]
            tickets = [srv.submit(r.pattern, r.roots) for r in mine]
            for r, t in zip(mine, tickets):
                got[id(r)] = (srv.wait(t).count, oracle.rooted_count(tabs[r.pattern], r.roots))
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    try:
        threads = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(120)
        assert not errors, errors
        assert len(got) == len(reqs)
        assert all(a == b for a, b in got.values())
    finally:
        srv.close()
        trie.free()


def test_server_close_with_pending(ctx, eh):
    """Closing a server with requests still queued or being expanded returns
    (finishing admitted work, cancelling the rest), and a new server on the
    same trie answers correctly afterwards."""
    tune(ctx)
    el = inputs.rmat(13, 16, seed=44)
    g = oracle.Graph.from_edgelist(el)
    rk = g.cliques4(rooted=True)["root"]
    trie = ctx.build_edgelist(el)
    try:
        big = np.arange(el.n, dtype=np.uint32)
        srv = ctx.server(trie, step_items=64, max_active=2)
        for _ in range(40):
            srv.submit(eh.CLIQUE4, big)
        srv.close()
        srv = ctx.server(trie)
        try:
            t = srv.submit(eh.CLIQUE4, big[:1000])
            assert srv.wait(t).count == oracle.rooted_count(rk, big[:1000])
        finally:
            srv.close()
    finally:
        trie.free()


def _el(n, pairs, name):
    a = np.array(pairs, np.uint32).reshape(-1, 2)
    return inputs.EdgeList(n, a[:, 0].copy(), a[:, 1].copy(), name)


DEGENERATE = [
    (_el(0, [], "no vertices"), 0, 0),
    (_el(1, [], "one vertex"), 0, 0),
    (_el(7, [], "no edges"), 0, 0),
    (_el(3, [(0, 0), (1, 1), (2, 2)], "self-loops only"), 0, 0),
    (_el(2, [(0, 1), (1, 0), (0, 1)], "one edge, repeated"), 0, 0),
    (_el(5, [(0, 1), (1, 2), (2, 0)], "one triangle, isolated rest"), 1, 0),
    (inputs.complete(4), 4, 1),
]


@pytest.mark.parametrize("tname", ["staged_target", "staged_source", "pair_auto", "staged_lean",
                                   "staged_steal", "staged_group"])
def test_degenerate_inputs(ctx, eh, tname):
    """Empty and tiny graphs: zero vertices, no edges, self-loops only, one
    edge, one triangle with isolated vertices, K4 -- totals, per-root
    vectors, rooted requests and the server all give the exact answer."""
    tune(ctx, **TUNINGS[tname])
    for el, T, K in DEGENERATE:
        trie = ctx.build_edgelist(el)
        try:
            assert ctx.count_triangles(trie) == T, el.name
            assert ctx.count_4cliques(trie) == K, el.name
            if tname == "staged_source":
                tot, per = ctx.count_triangles(trie, per_root=True)
                assert tot == T and int(per.sum()) == T and per.size == el.n, el.name
            if el.n:
                allv = np.arange(el.n, dtype=np.uint32)
                assert ctx.count_rooted(trie, eh.TRIANGLE, allv) == T, el.name
                assert ctx.count_rooted(trie, eh.CLIQUE4, allv) == K, el.name
                srv = ctx.server(trie)
                try:
                    tickets = [srv.submit(eh.TRIANGLE, allv), srv.submit(eh.CLIQUE4, allv[:1])]
                    assert srv.wait(tickets[0]).count == T, el.name
                    assert srv.wait(tickets[1]).count == (K if el.n == 4 else 0), el.name
                finally:
                    srv.close()
        finally:
            trie.free()


def test_batch_with_empty_graphs(ctx, eh):
    """A batch mixing graphs with no vertices, no edges and tiny cliques with
    ordinary ones: every per-graph count is exact, one launch or one per graph."""
    tune(ctx)
    parts = [el for el, _, _ in DEGENERATE] + [inputs.rmat(9, 8, seed=5), inputs.complete(40)]
    parts = parts + parts[::-1]
    srcs, dsts, off, nv = [], [], [0], []
    for g in parts:
        srcs.append(g.src)
        dsts.append(g.dst)
        off.append(off[-1] + g.m_raw)
        nv.append(g.n)
    b = inputs.BatchEdges(np.array(nv, np.uint32), np.array(off, np.uint64),
                          np.concatenate(srcs), np.concatenate(dsts), "degenerate mix")
    want_t = np.array([oracle.Graph.from_edgelist(g).triangles()["count"] for g in parts], np.uint64)
    want_k = np.array([oracle.Graph.from_edgelist(g).cliques4()["count"] for g in parts], np.uint64)
    trie = ctx.build_batch(b)
    try:
        for dyn in (0, 4):
            tune(ctx, dynamic=dyn)
            np.testing.assert_array_equal(ctx.count_batch(trie, eh.TRIANGLE), want_t)
            np.testing.assert_array_equal(ctx.count_batch(trie, eh.CLIQUE4), want_k)
            per = np.array([ctx.count_batch(trie, eh.TRIANGLE, i, 1)[0] for i in range(len(parts))],
                           np.uint64)
            np.testing.assert_array_equal(per, want_t)
    finally:
        trie.free()


ORDER_GRAPHS = [inputs.rmat(12, 16, seed=41), inputs.relabel(inputs.rmat(11, 16, seed=42), 3),
                inputs.chung_lu(20000, 16, 1.8, seed=6), inputs.chung_lu(8000, 12, 2.6, seed=7),
                inputs.erdos_renyi_gnm(3000, 4000, seed=8),
                inputs.disjoint_union(inputs.complete(40), inputs.wheel(30), inputs.grid(9, 9))]
_ORDER_TRUTH = {}


def order_truth(el, order):
    key = (el.name, order)
    if key not in _ORDER_TRUTH:
        g = oracle.Graph.from_edgelist(el, order)
        t = g.triangles(rooted=True)
        off, _ = g.oriented()
        d = np.diff(off.astype(np.int64))
        dmax = int(d.max()) if d.size else 0
        k = g.cliques4(rooted=True)
        _ORDER_TRUTH[key] = (t, k, dmax)
    return _ORDER_TRUTH[key]


@pytest.mark.parametrize("order", ["rev_degree", "input", "bfs", "hybrid", "strong_runs"])
def test_node_orderings(ctx, eh, order):
    """Node orderings (appendix A): totals equal the oracle's under every
    ordering; per-root and rooted counts follow the ordering's ranks, which
    the oracle computes with its own code.  Out-degrees above 2048 (only
    possible away from degree order) keep the 4-clique S lists in HBM.""" 
    for el in ORDER_GRAPHS:
        t, k, dmax = order_truth(el, order)
        say("order", order, el.name, "dmax", dmax)
        trie = ctx.build_edgelist(el, order=eh.ORDERS[order])
        try:
            assert trie.info["max_out_degree"] == dmax
            for tname in ("staged_target", "staged_source", "staged_lean", "staged_group",
                          "pair_auto"):
                tune(ctx, **TUNINGS[tname])
                assert ctx.count_triangles(trie) == t["count"], (el.name, tname)
            tune(ctx, **TUNINGS["staged_source"])
            tot, per = ctx.count_triangles(trie, per_root=True)
            assert tot == t["count"]
            np.testing.assert_array_equal(per, t["root"])
            roots = np.arange(0, el.n, 7, dtype=np.uint32)
            assert ctx.count_rooted(trie, eh.TRIANGLE, roots) == oracle.rooted_count(t["root"], roots)
            for tname in ("staged_source", "staged_steal"):
                tune(ctx, **TUNINGS[tname])
                assert ctx.count_4cliques(trie) == k["count"], (el.name, tname)
            assert ctx.count_rooted(trie, eh.CLIQUE4, roots) == oracle.rooted_count(k["root"], roots)
        finally:
            trie.free()


def test_out_degree_beyond_16_bits(ctx, eh):
    """Wheel W_70000 under reverse degree order: the hub's out-set holds all
    70,000 rim vertices, beyond what target staging's 16-bit segment lengths
    describe, so triangle totals stage sources instead: W_k has k triangles,
    and no 4-clique (its hub's S lists are kept in HBM)."""
    k = 70000
    el = inputs.wheel(k)
    trie = ctx.build_edgelist(el, order=eh.ORDER_REV_DEGREE)
    try:
        assert trie.info["max_out_degree"] == k
        for tname in ("staged_target", "staged_lean", "staged_group", "staged_source", "pair_auto"):
            tune(ctx, **TUNINGS[tname])
            assert ctx.count_triangles(trie) == k, tname
        tune(ctx, **TUNINGS["staged_source"])
        assert ctx.count_4cliques(trie) == 0
    finally:
        trie.free()


@pytest.mark.parametrize("order", ["bfs", "hybrid", "rev_degree"])
def test_batch_node_orderings(ctx, eh, order):
    tune(ctx, **TUNINGS["staged_group"])
    b = small_batch(80, seed=13)
    want = [order_truth(b.graph(i), order) for i in range(b.n_graphs)]
    trie = ctx.build_batch(b, order=eh.ORDERS[order])
    try:
        np.testing.assert_array_equal(ctx.count_batch(trie, eh.TRIANGLE),
                                      np.array([w[0]["count"] for w in want], np.uint64))
        np.testing.assert_array_equal(ctx.count_batch(trie, eh.CLIQUE4),
                                      np.array([w[1]["count"] for w in want], np.uint64))
    finally:
        trie.free()


def _device_pairs(el):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(el.src).view(np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(el.dst).view(np.int32)).cuda())


def _same_trie(ctx, a, b, where):
    assert a.info == b.info, where
    ha, hb = a.host_arrays(), b.host_arrays()
    for k in ha:
        np.testing.assert_array_equal(ha[k], hb[k], err_msg=f"{where}: host {k}")
    da, db = ctx.device_arrays(a), ctx.device_arrays(b)
    for k in da:
        np.testing.assert_array_equal(da[k], db[k], err_msg=f"{where}: device {k}")


DEVICE_BUILD_GRAPHS = [inputs.rmat(12, 16, seed=51), inputs.messy(inputs.rmat(10, 8, seed=52), 5),
                       inputs.chung_lu(30000, 12, 2.1, seed=53), inputs.erdos_renyi_gnm(5000, 9000, seed=54),
                       inputs.complete(70), inputs.grid(20, 30), inputs.wheel(100),
                       inputs.disjoint_union(inputs.complete(33), inputs.star(40), inputs.path(1)),
                       inputs.EdgeList(9, np.arange(9, dtype=np.uint32), np.arange(9, dtype=np.uint32),
                                       "loops_only"),
                       inputs.EdgeList(2, np.array([0, 1, 1, 0], np.uint32), np.array([1, 0, 1, 1], np.uint32),
                                       "one_edge_repeated")]


@pytest.mark.parametrize("order", ["degree", "rev_degree", "input", "bfs", "hybrid", "strong_runs"])
@pytest.mark.parametrize("lay", LAYOUTS, ids=lambda x: x[0])
def test_device_build_matches_host_build(ctx, eh, order, lay):
    """The GPU trie build gives the host build's trie, array for array (index
    work: bit-exact), host copy and device arrays alike; ranks and the
    oriented CSR equal the oracle's; counts equal the oracle's."""
    tune(ctx, **TUNINGS["staged_lean"])
    for el in DEVICE_BUILD_GRAPHS:
        say("device build", order, lay[0], el.name)
        src, dst = _device_pairs(el)
        ht = ctx.build_edgelist(el, layout=lay[1], tau=lay[2], order=eh.ORDERS[order])
        dt = ctx.build_trie_device(el.n, src, dst, layout=lay[1], tau=lay[2], order=eh.ORDERS[order])
        try:
            _same_trie(ctx, dt, ht, f"{el.name} {order} {lay[0]}")
            t, k, dmax = order_truth(el, order)
            g = oracle.Graph.from_edgelist(el, order)
            off, nbr = g.oriented()
            h = dt.host_arrays()
            np.testing.assert_array_equal(h["rank"], g.rank())
            np.testing.assert_array_equal(h["row"], off.astype(np.uint32))
            np.testing.assert_array_equal(h["col"], nbr)
            assert ctx.count_triangles(dt) == t["count"]
            if lay[0] == "hybrid32":
                assert ctx.count_4cliques(dt) == k["count"]
        finally:
            dt.free()
            ht.free()


def test_device_build_rejects(ctx, eh):
    import torch
    src = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    dst = torch.tensor([1, 2, 3], dtype=torch.int32, device="cuda")
    with pytest.raises(eh.EHError) as e:
        ctx.build_trie_device(3, src, dst)            # id 3 >= n
    assert e.value.status == eh.EH_EINVAL
    for order in ("bfs", "hybrid", "strong_runs"):
        # traversal orderings: built on the GPU for a single graph, not for a batch
        t = ctx.build_trie_device(4, src, dst, order=eh.ORDERS[order])
        try:
            assert t.info["m_plus"] == 3
        finally:
            t.free()
        b = inputs.BatchEdges(np.array([4], np.uint32), np.array([0, 3], np.uint64),
                              np.array([0, 1, 2], np.uint32), np.array([1, 2, 3], np.uint32), "one")
        with pytest.raises(eh.EHError) as e:
            ctx.build_batch_device(b, src, dst, order=eh.ORDERS[order])
        assert e.value.status == eh.EH_EINVAL
    with pytest.raises(eh.EHError) as e:
        ctx.build_trie_device(0, src, dst)
    assert e.value.status == eh.EH_EINVAL
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    for n in (0, 1, 6):
        t = ctx.build_trie_device(n, empty, empty)
        try:
            assert t.info["n"] == n and t.info["m_plus"] == 0
            assert ctx.count_triangles(t) == 0 and ctx.count_4cliques(t) == 0
        finally:
            t.free()
    # the context stays usable after a rejected build
    t = ctx.build_trie_device(4, src, dst)
    try:
        assert t.info["m_plus"] == 3 and ctx.count_triangles(t) == 0
    finally:
        t.free()


def test_device_build_full_size_rmat20(ctx, eh):
    """R-MAT scale 20 built on the GPU: the host build's trie, array for array,
    and the oracle's ranks, rows and columns."""
    el = inputs.rmat(20, 16, seed=20)
    src, dst = _device_pairs(el)
    say("rmat20 pairs on device")
    dt = ctx.build_trie_device(el.n, src, dst)
    ht = ctx.build_edgelist(el)
    try:
        _same_trie(ctx, dt, ht, "rmat20")
        say("device build equals host build")
        g = oracle.Graph.from_edgelist(el)
        off, nbr = g.oriented()
        h = dt.host_arrays()
        np.testing.assert_array_equal(h["rank"], g.rank())
        np.testing.assert_array_equal(h["row"], off.astype(np.uint32))
        np.testing.assert_array_equal(h["col"], nbr)
        tune(ctx, **TUNINGS["staged_lean"])
        T = g.triangles()["count"]
        assert ctx.count_triangles(dt) == T
    finally:
        dt.free()
        ht.free()
    # the traversal orderings at full size: the GPU's parallel label sequences
    # equal the host's sequential traversals (themselves pinned to the oracle's
    # orderings on smaller graphs)
    for order in ("bfs", "hybrid", "strong_runs"):
        dt = ctx.build_trie_device(el.n, src, dst, order=eh.ORDERS[order])
        ht = ctx.build_edgelist(el, order=eh.ORDERS[order])
        try:
            _same_trie(ctx, dt, ht, f"rmat20 {order}")
            say("device build equals host build", order)
            tune(ctx, **TUNINGS["staged_source"])
            assert ctx.count_triangles(dt) == T
        finally:
            dt.free()
            ht.free()


SYM_GRAPHS = [inputs.rmat(12, 16, seed=71), inputs.chung_lu(6000, 12, 2.3, seed=72),
              inputs.messy(inputs.rmat(10, 8, seed=73), 2), inputs.gnp(60, 0.3, seed=74),
              inputs.complete(45), inputs.disjoint_union(inputs.wheel(25), inputs.star(12),
                                                         inputs.path(1), inputs.grid(5, 5)),
              inputs.chung_lu(30000, 8, 1.9, seed=75)]
_SYM_TRUTH = {}


def sym_truth(el):
    """6T, t(x) by id, 24K and the Lollipop count, from the oracle (pinned:
    the unpruned join equals 6T and 24K; t(x) = 2 c3(x))."""
    if el.name not in _SYM_TRUTH:
        g = oracle.Graph.from_edgelist(el)
        six_t, t = g.sym_triangles_by_first()
        _SYM_TRUTH[el.name] = (six_t, t, 24 * g.count(4), g.sym_lollipop())
    return _SYM_TRUTH[el.name]


@pytest.mark.parametrize("tname", ["staged_target", "staged_source", "staged_lean", "staged_group",
                                   "staged_search", "staged_steal", "pair_auto", "pair_merge4"])
def test_symmetric_triangles_and_lollipop(ctx, eh, tname):
    """Unpruned relation: the join's ordered triangles (6T), t(x) by first
    attribute, rooted counts, and the Lollipop count, under every kernel."""
    tune(ctx, **TUNINGS[tname])
    for el in SYM_GRAPHS:
        six_t, t, _, lolli = sym_truth(el)
        say("symmetric", tname, el.name)
        trie = ctx.build_edgelist(el, symmetric=True)
        try:
            assert ctx.count_triangles(trie) == six_t
            tot, per = ctx.count_triangles(trie, per_root=True)
            assert tot == six_t
            np.testing.assert_array_equal(per, t)
            roots = np.arange(1, el.n, 5, dtype=np.uint32)
            assert ctx.count_rooted(trie, eh.TRIANGLE, roots) == int(t[roots].sum(dtype=np.uint64))
            assert ctx.count_lollipop(trie) == lolli
        finally:
            trie.free()


@pytest.mark.parametrize("tname", ["staged_target", "staged_lean", "pair_auto"])
def test_symmetric_totals_each_edge_once(ctx, eh, tname):
    """Symmetric totals are counted over each undirected edge once and doubled
    (unless the tuning asks for source staging): overwrite and accumulate
    forms, against the oracle's 6T and the every-arc evaluation."""
    import torch
    for el in SYM_GRAPHS:
        six_t = sym_truth(el)[0]
        say("symmetric totals", tname, el.name)
        trie = ctx.build_edgelist(el, symmetric=True)
        try:
            tune(ctx, **TUNINGS[tname])
            d = torch.full((1,), 12345, dtype=torch.int64, device="cuda")
            ctx.stream.wait_stream(torch.cuda.current_stream())
            ctx.count_async(trie, eh.TRIANGLE, d)
            ctx.count_add_async(trie, eh.TRIANGLE, d)
            ctx.count_add_async(trie, eh.TRIANGLE, d)
            ctx.stream.synchronize()
            assert int(d.item()) == 3 * six_t
            tune(ctx, **dict(TUNINGS[tname], staging=eh.STAGE_SOURCE))
            assert ctx.count_triangles(trie) == six_t
        finally:
            trie.free()


@pytest.mark.parametrize("tname", ["staged_source", "staged_half", "staged_steal"])
def test_symmetric_4cliques(ctx, eh, tname):
    """Unpruned 4-cliques: 24K ordered tuples, with S in LDS lists up to
    degree 2048 and in HBM lists beyond."""
    tune(ctx, **TUNINGS[tname])
    for el in SYM_GRAPHS:
        _, _, k24, _ = sym_truth(el)
        trie = ctx.build_edgelist(el, symmetric=True)
        try:
            assert ctx.count_4cliques(trie) == k24, el.name
        finally:
            trie.free()


def test_symmetric_hub_of_100k(ctx, eh):
    """W_100000 unpruned: the hub's set has 100,000 members (composite
    staging, uint-bitset at scale); 6T = 6k, Lollipop = 2k^2 + 12k."""
    k = 100000
    trie = ctx.build_edgelist(inputs.wheel(k), symmetric=True)
    try:
        assert trie.info["max_out_degree"] == k
        for tname in ("staged_source", "staged_lean", "pair_auto", "staged_steal"):
            tune(ctx, **TUNINGS[tname])
            assert ctx.count_triangles(trie) == 6 * k, tname
            assert ctx.count_lollipop(trie) == 2 * k * k + 12 * k, tname
    finally:
        trie.free()


@pytest.mark.parametrize("tname", ["staged_target", "staged_nobits", "staged_list", "staged_lean",
                                   "staged_part", "staged_snake"])
def test_lollipop_edge_once(ctx, eh, tname):
    """The Lollipop count over each undirected edge {x, u} once, weighted by
    |N(x)| + |N(u)|, equals the oracle's and the every-arc evaluation (source
    staging: t(x) by first attribute, then degree-weighted): staged sets as
    bitmaps, composites with searched prefixes (8-word windows), with and
    without streamed bitset words, under four schedules."""
    graphs = SYM_GRAPHS + [inputs.rmat(14, 16, seed=141)]
    for el in graphs:
        lolli = sym_truth(el)[3]
        say("lollipop edge once", tname, el.name)
        trie = ctx.build_edgelist(el, symmetric=True)
        try:
            tune(ctx, **TUNINGS[tname])
            assert ctx.count_lollipop(trie) == lolli, el.name
            assert ctx.count_lollipop(trie) == lolli, el.name   # cached plan
            tune(ctx, **dict(TUNINGS[tname], staging=eh.STAGE_SOURCE))
            assert ctx.count_lollipop(trie) == lolli, el.name
        finally:
            trie.free()


def test_symmetric_batch_and_device_build(ctx, eh):
    tune(ctx, **TUNINGS["staged_steal"])
    b = small_batch(60, seed=17)
    want = [(6 * order_truth(b.graph(i), "degree")[0]["count"],
             24 * oracle.Graph.from_edgelist(b.graph(i)).count(4)) for i in range(b.n_graphs)]
    trie = ctx.build_batch(b, symmetric=True)
    try:
        np.testing.assert_array_equal(ctx.count_batch(trie, eh.TRIANGLE),
                                      np.array([w[0] for w in want], np.uint64))
        np.testing.assert_array_equal(ctx.count_batch(trie, eh.CLIQUE4),
                                      np.array([w[1] for w in want], np.uint64))
        with pytest.raises(eh.EHError) as e:
            ctx.count_lollipop(trie)
        assert e.value.status == eh.EH_ESTATE
    finally:
        trie.free()
    for el in SYM_GRAPHS[:4]:
        src, dst = _device_pairs(el)
        ht = ctx.build_edgelist(el, symmetric=True)
        dt = ctx.build_trie_device(el.n, src, dst, symmetric=True)
        try:
            _same_trie(ctx, dt, ht, el.name + " symmetric")
            assert ctx.count_lollipop(dt) == sym_truth(el)[3]
        finally:
            dt.free()
            ht.free()
    pruned = ctx.build_edgelist(SYM_GRAPHS[0])
    try:
        with pytest.raises(eh.EHError) as e:
            ctx.count_lollipop(pruned)
        assert e.value.status == eh.EH_ESTATE
    finally:
        pruned.free()


def _degenerate_mix():
    parts = [el for el, _, _ in DEGENERATE] + [inputs.rmat(9, 8, seed=5), inputs.complete(40)]
    parts = parts + parts[::-1]
    srcs, dsts, off, nv = [], [], [0], []
    for g in parts:
        srcs.append(g.src)
        dsts.append(g.dst)
        off.append(off[-1] + g.m_raw)
        nv.append(g.n)
    return inputs.BatchEdges(np.array(nv, np.uint32), np.array(off, np.uint64),
                             np.concatenate(srcs), np.concatenate(dsts), "degenerate mix")


@pytest.mark.parametrize("symmetric", [False, True])
@pytest.mark.parametrize("order", ["degree", "rev_degree", "input"])
def test_batch_device_build(ctx, eh, order, symmetric):
    """The batch trie built on the GPU equals the host batch build array for
    array, and its per-graph counts equal the oracle's."""
    import torch
    tune(ctx, **TUNINGS["staged_group"])
    for b in (small_batch(70, seed=21), _degenerate_mix()):
        say("batch device build", order, symmetric, b.name)
        src = torch.from_numpy(np.ascontiguousarray(b.src).view(np.int32)).cuda()
        dst = torch.from_numpy(np.ascontiguousarray(b.dst).view(np.int32)).cuda()
        ht = ctx.build_batch(b, order=eh.ORDERS[order], symmetric=symmetric)
        dt = ctx.build_batch_device(b, src, dst, order=eh.ORDERS[order], symmetric=symmetric)
        try:
            _same_trie(ctx, dt, ht, f"{b.name} {order} {symmetric}")
            mult = 6 if symmetric else 1
            want = np.array([mult * order_truth(b.graph(i), order)[0]["count"]
                             for i in range(b.n_graphs)], np.uint64)
            np.testing.assert_array_equal(ctx.count_batch(dt, eh.TRIANGLE), want)
        finally:
            dt.free()
            ht.free()
    # a local id at or beyond its graph's vertex count is refused
    b = small_batch(5, seed=22)
    bad_src = np.ascontiguousarray(b.src).copy()
    bad_src[int(b.edge_off[2])] = b.n_vertices[2]  # graph 2's first pair names id n_2
    src = torch.from_numpy(bad_src.view(np.int32)).cuda()
    dst = torch.from_numpy(np.ascontiguousarray(b.dst).view(np.int32)).cuda()
    with pytest.raises(eh.EHError) as e:
        ctx.build_batch_device(b, src, dst)
    assert e.value.status == eh.EH_EINVAL


def test_host_planner_path(ctx, eh, monkeypatch):
    """Target-staged triangle plans are built on the GPU unless EH_HOST_PLAN is
    set; the host planner (kept for grouped plans of a few large graphs) must
    give the same counts."""
    monkeypatch.setenv("EH_HOST_PLAN", "1")
    for tname in ("staged_target", "staged_lean", "staged_group", "staged_group_lean"):
        tune(ctx, **TUNINGS[tname])
        for el in ZOO[-8:]:
            T, _, _ = truth(el)
            trie = ctx.build_edgelist(el)
            try:
                assert ctx.count_triangles(trie) == T, (tname, el.name)
            finally:
                trie.free()
        b = small_batch(50, seed=23)
        want = np.array([oracle.Graph.from_edgelist(b.graph(i)).triangles()["count"]
                         for i in range(b.n_graphs)], np.uint64)
        trie = ctx.build_batch(b)
        try:
            np.testing.assert_array_equal(ctx.count_batch(trie, eh.TRIANGLE), want)
        finally:
            trie.free()


def test_out_degree_limits(ctx, eh):
    """K_2050: triangles at out-degree 2049 (C(n, 3)); 4-cliques C(n, 4),
    the root of out-degree 2049 with its S lists in HBM."""
    from math import comb
    tune(ctx)
    n = 2050
    trie = ctx.build_edgelist(inputs.complete(n))
    try:
        assert trie.info["max_out_degree"] == n - 1
        for tname in ("staged_target", "staged_source", "staged_lean", "pair_auto"):
            tune(ctx, **TUNINGS[tname])
            assert ctx.count_triangles(trie) == comb(n, 3), tname
        tune(ctx, **TUNINGS["staged_source"])
        assert ctx.count_4cliques(trie) == comb(n, 4)
        # vertex i roots C(n-1-i, 3)
        roots = np.array([5, 100, 2000], np.uint32)
        assert ctx.count_rooted(trie, eh.CLIQUE4, roots) == sum(comb(n - 1 - int(i), 3) for i in roots)
    finally:
        trie.free()


def test_graph_capture_replay(ctx, eh):
    """The one-launch batch count and an accumulating single-graph count are
    captured into a HIP graph (after warm-up calls have built their plans) and
    replayed several times, with eager counts and synchronizations in between;
    every replay gives the eager result.  The capture holds the cursor-reset
    and output-clearing kernels of schedule 4 (fill kernels, no memset nodes)."""
    import torch
    tune(ctx, dynamic=4, grab=4, group=4)
    b = small_batch(60, seed=21)
    want = np.array([oracle.Graph.from_edgelist(b.graph(i)).triangles()["count"]
                     for i in range(b.n_graphs)], np.uint64)
    el = inputs.rmat(12, 16, seed=22)
    T = oracle.Graph.from_edgelist(el).triangles()["count"]
    bt = ctx.build_batch(b)
    gt = ctx.build_edgelist(el)
    try:
        G = bt.info["n_graphs"]
        out_b = torch.zeros(G, dtype=torch.int64, device="cuda")
        out_t = torch.zeros(1, dtype=torch.int64, device="cuda")
        s = ctx.stream
        s.wait_stream(torch.cuda.current_stream())
        ctx.count_batch_async(bt, eh.TRIANGLE, 0, G, out_b)
        ctx.count_add_async(gt, eh.TRIANGLE, out_t)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ctx.count_batch_async(bt, eh.TRIANGLE, 0, G, out_b)
            ctx.count_add_async(gt, eh.TRIANGLE, out_t)
        out_b.zero_()
        out_t.zero_()
        torch.cuda.synchronize()
        for rep in range(3):
            g.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out_b.cpu().numpy().view(np.uint64), want)
            assert int(out_t.cpu().numpy().view(np.uint64)[0]) == (rep + 1) * T
            # eager work on the same context between replays
            assert ctx.count_triangles(gt) == T
            np.testing.assert_array_equal(ctx.count_batch(bt, eh.TRIANGLE), want)
        del g
    finally:
        bt.free()
        gt.free()


def test_graph_capture_replay_4cliques(ctx, eh):
    """A 4-clique count whose roots run on the induced-neighbourhood kernels
    (four launches, three on side streams forked from the captured stream and
    joined back by events) and on the S-list kernel is captured and replayed;
    every replay, with eager 4-clique counts on the same streams in between,
    adds the oracle's count."""
    import torch
    tune(ctx, k4_local=1, staging=1, dynamic=4, grab=2)
    el = inputs.disjoint_union(inputs.complete(600), inputs.rmat(13, 16, seed=23))
    K = oracle.Graph.from_edgelist(el).count(4)
    gt = ctx.build_edgelist(el)
    try:
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        s = ctx.stream
        s.wait_stream(torch.cuda.current_stream())
        ctx.count_add_async(gt, eh.CLIQUE4, out)
        torch.cuda.synchronize()
        assert int(out.cpu().numpy().view(np.uint64)[0]) == K
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            ctx.count_add_async(gt, eh.CLIQUE4, out)
        out.zero_()
        torch.cuda.synchronize()
        for rep in range(3):
            g.replay()
            torch.cuda.synchronize()
            assert int(out.cpu().numpy().view(np.uint64)[0]) == (rep + 1) * K
            assert ctx.count_4cliques(gt) == K
        del g
    finally:
        gt.free()


def test_randomized_parity(ctx, eh):
    """Seeded random graphs (R-MAT, G(n,p), Chung-Lu, unions, messy input)
    under seeded random settings of every tuning knob: each triangle and
    4-clique count equals the oracle's."""
    key = inputs.stream_key(77, 7)
    draws = inputs.rand_u64(key, 0, 100 * 32)
    pick = iter(int(x) for x in draws)

    def choice(xs):
        return xs[next(pick) % len(xs)]

    for case in range(100):
        kind = choice(["rmat", "gnp", "cl", "union", "messy"])
        seed = 1000 + case
        if kind == "rmat":
            el = inputs.rmat(choice([6, 8, 10, 11]), choice([4, 16]), seed=seed)
        elif kind == "gnp":
            el = inputs.gnp(choice([20, 60, 150]), choice([0.05, 0.3, 0.7]), seed)
        elif kind == "cl":
            el = inputs.chung_lu(choice([300, 2000]), choice([4.0, 24.0]), 2.1, seed=seed, graph=case)
        elif kind == "union":
            el = inputs.disjoint_union(inputs.complete(choice([5, 30])), inputs.rmat(8, 8, seed=seed))
        else:
            el = inputs.messy(inputs.rmat(9, 8, seed=seed), seed)
        t = dict(kernel=choice([1, 1, 2]), staging=choice([1, 2]), use_bitsets=choice([0, 1]),
                 dynamic=choice([0, 1, 2, 3, 4, 5]), grab=choice([1, 3, 16]), xcds=choice([0, 3, 8]),
                 stage_words=choice([0, 8, 96, 512]), search_below=choice([0, 12, 4096]),
                 group=choice([1, 2, 4]), chunk_work=choice([64, 1000, 32768]),
                 reverse=choice([0, 1]),
                 waves_per_cu=choice([1, 8, 32]), unroll=choice([4, 8]),
                 group_lanes=choice([0, 4, 64]), algo=choice([0, 1, 2]), k4_local=choice([0, 1]))
        tune(ctx, **t)
        layout, tau = choice([(0, 32.0), (1, 2.0), (1, 32.0), (1, 256.0), (2, 32.0)])
        T, K, _ = truth(el)
        trie = ctx.build_edgelist(el, layout=layout, tau=tau)
        try:
            assert ctx.count_triangles(trie) == T, (case, kind, t, layout, tau)
            assert ctx.count_4cliques(trie) == K, (case, kind, t, layout, tau)
        finally:
            trie.free()


def test_randomized_build_paths(ctx, eh):
    """Seeded random graphs under seeded random choices of node ordering,
    pruned or unpruned relation, host or GPU build and tuning knobs: totals,
    per-root vectors and (where out-degrees allow) 4-cliques equal the
    oracle's under that ordering's ranks (unpruned: 6T, 2 c3 by first
    attribute, 24K)."""
    import torch
    key = inputs.stream_key(78, 8)
    draws = inputs.rand_u64(key, 0, 40 * 32)
    pick = iter(int(x) for x in draws)

    def choice(xs):
        return xs[next(pick) % len(xs)]

    for case in range(40):
        kind = choice(["rmat", "gnp", "cl", "messy"])
        seed = 2000 + case
        if kind == "rmat":
            el = inputs.rmat(choice([7, 9, 11]), choice([4, 16]), seed=seed)
        elif kind == "gnp":
            el = inputs.gnp(choice([30, 90]), choice([0.1, 0.5]), seed)
        elif kind == "cl":
            el = inputs.chung_lu(choice([500, 3000]), choice([6.0, 20.0]), choice([1.9, 2.5]),
                                 seed=seed, graph=case)
        else:
            el = inputs.messy(inputs.rmat(8, 8, seed=seed), seed)
        order = choice(["degree", "rev_degree", "input", "bfs", "hybrid", "strong_runs"])
        symmetric = choice([False, False, True])
        device = choice([False, True])
        t = dict(kernel=choice([1, 1, 2]), staging=choice([1, 2]), use_bitsets=choice([0, 1]),
                 dynamic=choice([0, 2, 4]), stage_words=choice([0, 96, 512]),
                 group=choice([1, 2, 4]), chunk_work=choice([64, 4096]),
                 search_below=choice([0, 24]), unroll=choice([4, 8]), reverse=choice([0, 1]))
        tune(ctx, **t)
        layout, tau = choice([(0, 32.0), (1, 32.0), (1, 256.0), (2, 32.0)])
        where = (case, kind, order, symmetric, device, t, layout, tau)
        say("random build path", where)
        if symmetric:
            six_t, t_first, k24, _ = sym_truth(el)
            want_t, want_root = six_t, t_first
        else:
            tr, kr, _ = order_truth(el, order)
            want_t, want_root = tr["count"], tr["root"]
            k24 = kr["count"]
        if device:
            src, dst = _device_pairs(el)
            trie = ctx.build_trie_device(el.n, src, dst, layout=layout, tau=tau,
                                         order=eh.ORDERS[order], symmetric=symmetric)
        else:
            trie = ctx.build_edgelist(el, layout=layout, tau=tau, order=eh.ORDERS[order],
                                      symmetric=symmetric)
        try:
            assert ctx.count_triangles(trie) == want_t, where
            tot, per = ctx.count_triangles(trie, per_root=True)
            assert tot == want_t, where
            np.testing.assert_array_equal(per, want_root, err_msg=str(where))
            assert ctx.count_4cliques(trie) == k24, where
        finally:
            trie.free()
