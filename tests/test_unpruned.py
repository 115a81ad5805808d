"""Pins for the oracle on the unpruned symmetric relation (appendix A,
pruning symmetric queries) and the Lollipop query of section 5.3, against
brute force over ordered tuples, closed forms and the pruned oracle's own
per-vertex counts; and the host build of symmetric tries against the
oracle's graph."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import eh, inputs


def adjacency(el):
    adj = [set() for _ in range(el.n)]
    for a, b in zip(el.src.tolist(), el.dst.tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def brute_lollipop(el):
    """Ordered (x, y, z, w) with xy, yz, xz, xw all edges (w may equal y or z:
    a join does not ask for distinct values)."""
    adj = adjacency(el)
    n = el.n
    total = 0
    for x, y, z in itertools.product(range(n), repeat=3):
        if y in adj[x] and z in adj[y] and z in adj[x]:
            total += len(adj[x])
    return total


@pytest.mark.parametrize("n,p,seed", [(8, 0.5, 1), (11, 0.4, 2), (13, 0.7, 3), (9, 0.95, 4)])
def test_lollipop_brute_force(n, p, seed):
    el = inputs.gnp(n, p, seed=seed)
    g = oracle.Graph.from_edgelist(el)
    assert g.sym_lollipop() == brute_lollipop(el)
    assert g.sym_lollipop(threads=1) == g.sym_lollipop(threads=4)


def test_lollipop_messy_input():
    el = inputs.messy(inputs.gnp(10, 0.5, seed=5), 3)
    assert oracle.Graph.from_edgelist(el).sym_lollipop() == brute_lollipop(inputs.gnp(10, 0.5, seed=5))


@pytest.mark.parametrize("n", [3, 4, 5, 9, 20])
def test_lollipop_complete_closed_form(n):
    # each x: (n-1)(n-2) ordered (y, z), n-1 choices of w
    g = oracle.Graph.from_edgelist(inputs.complete(n))
    assert g.sym_lollipop() == n * (n - 1) ** 2 * (n - 2)


@pytest.mark.parametrize("k", [4, 5, 12, 101])
def test_lollipop_wheel_closed_form(k):
    # hub: 2k ordered triangles, degree k; each rim vertex: 4 and degree 3
    g = oracle.Graph.from_edgelist(inputs.wheel(k))
    assert g.sym_lollipop() == 2 * k * k + 12 * k


def test_lollipop_triangle_free():
    for el in (inputs.star(20), inputs.grid(5, 6), inputs.cycle(9), inputs.complete_bipartite(4, 7)):
        assert oracle.Graph.from_edgelist(el).sym_lollipop() == 0


@pytest.mark.parametrize("el", [inputs.rmat(11, 16, seed=61), inputs.chung_lu(4000, 10, 2.2, seed=62),
                                inputs.erdos_renyi_gnm(2000, 9000, seed=63)], ids=lambda e: e.name)
def test_by_first_attribute_against_pruned_counts(el):
    """t(x) on the unpruned relation is twice the triangles containing x, as
    the pruned oracle counts them; the Lollipop count is the degree-weighted
    sum of t."""
    g = oracle.Graph.from_edgelist(el)
    r = g.triangles(per_vertex=True)
    total, t = g.sym_triangles_by_first()
    np.testing.assert_array_equal(t, 2 * r["per_vertex"])
    assert total == 6 * r["count"] == g.sym_ordered_triangles()
    deg = g.degree().astype(np.uint64)
    assert g.sym_lollipop() == int((t * deg).sum(dtype=np.uint64))


@pytest.mark.parametrize("order", ["degree", "rev_degree", "input"])
@pytest.mark.parametrize("el", [inputs.rmat(10, 16, seed=64), inputs.messy(inputs.rmat(9, 8, seed=65), 2),
                                inputs.disjoint_union(inputs.wheel(30), inputs.star(9), inputs.path(1))],
                         ids=lambda e: e.name)
def test_host_symmetric_trie(el, order):
    """The symmetric trie holds, in rank space, every undirected edge in both
    directions, rows ascending; the set optimizer applies to the full sets."""
    h = eh.host_trie(el.n, el.src, el.dst, order=eh.ORDERS[order], symmetric=True)
    g = oracle.Graph.from_edgelist(el, order)
    rank = g.rank().astype(np.int64)
    a, b = g.edges()
    ra, rb = rank[a], rank[b]
    src = np.concatenate([ra, rb])
    dst = np.concatenate([rb, ra])
    o = np.lexsort((dst, src))
    row = np.zeros(el.n + 1, np.int64)
    np.add.at(row, src + 1, 1)
    np.testing.assert_array_equal(h["row"], np.cumsum(row).astype(np.uint32))
    np.testing.assert_array_equal(h["col"], dst[o].astype(np.uint32))
    assert h["m_plus"] == 2 * g.m
    d = np.diff(h["row"].astype(np.int64))
    assert h["max_out_degree"] == (d.max() if d.size else 0)
    assert h["b_merge"] == int(sum(4 * (d[u] + d[v]) for u, v in zip(src.tolist(), dst.tolist())))
    for r in range(el.n):
        seg = h["col"][h["row"][r]:h["row"][r + 1]]
        if h["bs_off"][r] != 0xFFFFFFFF:
            assert (int(seg[-1]) - int(seg[0]) + 1) <= 32.0 * seg.size
