"""4-cliques rooted at hubs: roots whose out-set exceeds the 2048-entry LDS
list keep S = N+(u) & N+(v) in HBM (section 5.3's K4 plan; appendix A,
"pruning symmetric queries": the unpruned relation has hub lists of 10^4 and
more members).  Every count equals the oracle's: 24K on symmetric tries,
K on pruned tries under an ordering that leaves a hub's whole neighbourhood in
its out-set, rooted counts under that ordering, and closed forms."""
from math import comb

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import inputs

pytestmark = pytest.mark.gpu

STEAL = dict(kernel=1, staging=1, dynamic=4, grab=2, chunk_work=4096, stage_words=0)
STATIC = dict(kernel=1, staging=1, dynamic=0, chunk_work=1024, stage_words=512)
TUNINGS = [STEAL, STATIC]


@pytest.fixture(scope="module")
def ctx(eh):
    c = eh.Context(0)
    yield c
    c.close()


def hub_over(el, seed=0):
    """el plus one vertex adjacent to every vertex of el."""
    hub = el.n
    others = np.arange(el.n, dtype=np.uint32)
    src = np.concatenate([el.src, np.full(el.n, hub, np.uint32)])
    dst = np.concatenate([el.dst, others])
    return inputs.EdgeList(el.n + 1, src, dst, f"hub_over_{el.name}")


def cliques_with_hub():
    """Disjoint cliques K_12 .. K_40 and a random graph, all under one hub."""
    parts = [inputs.complete(k) for k in (12, 20, 33, 40)] + [inputs.gnp(200, 0.1, seed=3),
                                                              inputs.rmat(11, 8, seed=4)]
    return hub_over(inputs.disjoint_union(*parts))


def test_wheel_100k_unpruned_and_reverse_degree(ctx, eh):
    """W_100000 has no 4-clique (its rim is a cycle); its hub's list holds
    100,000 members, unpruned and, pruned under reverse degree order, as an
    out-set."""
    k = 100000
    el = inputs.wheel(k)
    for kw in (dict(symmetric=True), dict(order=eh.ORDER_REV_DEGREE)):
        trie = ctx.build_edgelist(el, **kw)
        try:
            assert trie.info["max_out_degree"] == k
            for t in TUNINGS:
                ctx.set_tuning(**t)
                assert ctx.count_4cliques(trie) == 0, (kw, t)
        finally:
            trie.free()


def test_complete_graph_beyond_lds_list(ctx, eh):
    """K_2050: the root of rank 0 has out-degree 2049; C(n, 4) in all, and
    vertex of rank i roots C(n-1-i, 3)."""
    n = 2050
    trie = ctx.build_edgelist(inputs.complete(n))
    try:
        for t in TUNINGS:
            ctx.set_tuning(**t)
            assert ctx.count_4cliques(trie) == comb(n, 4), t
        roots = np.array([0, 5, 100, 2000], np.uint32)
        assert ctx.count_rooted(trie, eh.CLIQUE4, roots) == sum(comb(n - 1 - int(i), 3) for i in roots)
    finally:
        trie.free()


@pytest.mark.parametrize("make", [cliques_with_hub,
                                  lambda: inputs.chung_lu(50000, 16, 1.9, seed=91)],
                         ids=["cliques_under_hub", "chung_lu_1.9_hub_13k"])
def test_hub_graphs(ctx, eh, make):
    el = make()
    g = oracle.Graph.from_edgelist(el)
    K = g.count(4)
    print(el.name, "K", K, flush=True)
    # unpruned: 24 K ordered tuples
    trie = ctx.build_edgelist(el, symmetric=True)
    try:
        assert trie.info["max_out_degree"] > 2048
        for t in TUNINGS:
            ctx.set_tuning(**t)
            assert ctx.count_4cliques(trie) == 24 * K, t
    finally:
        trie.free()
    # pruned under reverse degree order: the hub roots its whole neighbourhood
    go = oracle.Graph.from_edgelist(el, "rev_degree")
    rk = go.cliques4(rooted=True)
    assert rk["count"] == K
    trie = ctx.build_edgelist(el, order=eh.ORDER_REV_DEGREE)
    try:
        assert trie.info["max_out_degree"] > 2048
        for t in TUNINGS:
            ctx.set_tuning(**t)
            assert ctx.count_4cliques(trie) == K, t
        roots = np.arange(0, el.n, 5, dtype=np.uint32)
        roots[0] = el.n - 1
        assert ctx.count_rooted(trie, eh.CLIQUE4, roots) == oracle.rooted_count(rk["root"], roots)
    finally:
        trie.free()


def test_server_hub_requests(ctx, eh):
    """Served 4-clique requests rooted at a hub, under reverse degree order,
    alone and mixed with triangle requests."""
    el = cliques_with_hub()
    go = oracle.Graph.from_edgelist(el, "rev_degree")
    rt = go.triangles(rooted=True)["root"]
    rk = go.cliques4(rooted=True)["root"]
    ctx.set_tuning(**STEAL)
    trie = ctx.build_edgelist(el, order=eh.ORDER_REV_DEGREE)
    srv = ctx.server(trie, step_items=256)
    try:
        hub = el.n - 1
        reqs = [(4, np.array([hub], np.uint32)), (3, np.array([hub, 1, 2], np.uint32)),
                (4, np.arange(0, el.n, 3, dtype=np.uint32)), (4, np.array([5, hub, 7], np.uint32))]
        tickets = [srv.submit(p, r) for p, r in reqs]
        got = [srv.wait(t).count for t in tickets]
        want = [oracle.rooted_count(rk if p == 4 else rt, r) for p, r in reqs]
        assert got == want
        assert want[0] > 0
    finally:
        srv.close()
        trie.free()


def test_noalloc_uses_plan_lists(ctx, eh):
    """The allocation-free count runs the HBM-list launch from the lists the
    plan allocated on its first count."""
    import torch
    el = inputs.chung_lu(50000, 16, 1.9, seed=91)
    K = oracle.Graph.from_edgelist(el).count(4)
    ctx.set_tuning(**STEAL)
    trie = ctx.build_edgelist(el, order=eh.ORDER_REV_DEGREE)
    try:
        assert ctx.count_4cliques(trie) == K
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.stream.wait_stream(torch.cuda.current_stream())
        ctx.count_add_noalloc(trie, eh.CLIQUE4, out)
        ctx.count_add_noalloc(trie, eh.CLIQUE4, out)
        torch.cuda.synchronize()
        assert int(out.cpu().numpy().view(np.uint64)[0]) == 2 * K
    finally:
        trie.free()
