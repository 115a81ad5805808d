"""Pins for the oracle's node orderings (appendix A, node ordering; section
2.2 dictionary encoding) against facts they do not compute themselves:
sequences worked out by hand from the definitions, scipy's breadth-first
traversal, structural properties, and brute-force counts under the ranks."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import oracle
from oracle.orderings import ORDERS, ranks, sequence
from paper_1503_02368_amd import inputs


def _el(n, pairs):
    a = np.array([p[0] for p in pairs], np.uint32)
    b = np.array([p[1] for p in pairs], np.uint32)
    return inputs.EdgeList(n, a, b, "hand")


# Worked by hand from the definitions (ties and traversal details as read in
# oracle/orderings.py).
# P5: the path 0-1-2-3-4, degrees 1 2 2 2 1.
P5 = _el(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
P5_SEQ = {"degree": [3, 2, 1, 4, 0], "rev_degree": [0, 4, 1, 2, 3], "input": [0, 1, 2, 3, 4],
          "bfs": [1, 0, 2, 3, 4], "hybrid": [1, 2, 3, 0, 4], "strong_runs": [1, 0, 2, 3, 4]}
# H8: hub 0 with leaves 1 2 3, hub 4 with 3 5 6, and 7 hanging off 1.
# Degrees: 0:3 1:2 2:1 3:2 4:3 5:1 6:1 7:1.  BFS from 0 reaches 7 (via 1)
# before 4 (via 3); strong runs labels 4's run right after 0's.
H8 = _el(8, [(0, 1), (0, 2), (0, 3), (4, 3), (4, 5), (4, 6), (1, 7)])
H8_SEQ = {"degree": [4, 0, 3, 1, 7, 6, 5, 2], "rev_degree": [2, 5, 6, 7, 1, 3, 0, 4],
          "input": list(range(8)), "bfs": [0, 1, 2, 3, 7, 4, 5, 6],
          "hybrid": [0, 4, 1, 3, 2, 7, 5, 6], "strong_runs": [0, 1, 2, 3, 4, 5, 6, 7]}
# G7: triangle {5,0,1} plus leaf 2 on 5, and a separate triangle {3,4,6}.
G7 = _el(7, [(5, 0), (5, 1), (5, 2), (0, 1), (3, 4), (4, 6), (3, 6)])
G7_SEQ = {"degree": [5, 6, 4, 3, 1, 0, 2], "rev_degree": [2, 0, 1, 3, 4, 6, 5],
          "input": list(range(7)), "bfs": [5, 0, 1, 2, 3, 4, 6],
          "hybrid": [5, 0, 1, 3, 4, 6, 2], "strong_runs": [5, 0, 1, 2, 3, 4, 6]}


@pytest.mark.parametrize("el,expect", [(P5, P5_SEQ), (H8, H8_SEQ), (G7, G7_SEQ)],
                         ids=["P5", "H8", "G7"])
def test_hand_worked_sequences(el, expect):
    g = oracle.Graph.from_edgelist(el)
    for order in ORDERS:
        assert sequence(g, order) == expect[order], order
        r = ranks(g, order)
        # label l goes to rank n - 1 - l
        assert [int(r[v]) for v in expect[order]] == list(range(el.n - 1, -1, -1))


def test_degree_order_is_the_default_ranking():
    for el in (inputs.rmat(10, 8, seed=7), inputs.chung_lu(2000, 12, 2.3, seed=5)):
        g = oracle.Graph.from_edgelist(el)
        np.testing.assert_array_equal(ranks(g, "degree"), g.rank())


GRAPHS = [inputs.rmat(10, 8, seed=11), inputs.chung_lu(2500, 6, 2.5, seed=3),
          inputs.erdos_renyi_gnm(600, 700, seed=4),  # many components and isolated vertices
          inputs.disjoint_union(inputs.star(7), inputs.cycle(9), inputs.complete(5),
                                inputs.path(1), inputs.grid(3, 4))]


def _csr(g):
    a, b = g.edges()
    m = sp.coo_matrix((np.ones(2 * a.size), (np.r_[a, b], np.r_[b, a])), shape=(g.n, g.n)).tocsr()
    m.sort_indices()
    return m


@pytest.mark.parametrize("el", GRAPHS, ids=lambda e: e.name)
def test_bfs_against_scipy(el):
    """Each component is one contiguous run: scipy's breadth-first order from
    the component's vertex of highest degree (lowest id on ties), and the
    runs come in order of that root's (degree descending, id ascending)."""
    g = oracle.Graph.from_edgelist(el)
    deg = g.degree().astype(np.int64)
    seq = sequence(g, "bfs")
    assert sorted(seq) == list(range(g.n))
    m = _csr(g)
    ncomp, comp = csgraph.connected_components(m, directed=False)
    pos = 0
    prev_key = None
    while pos < g.n:
        root = seq[pos]
        members = np.nonzero(comp == comp[root])[0]
        best = min(members.tolist(), key=lambda v: (-deg[v], v))
        assert root == best
        key = (-deg[root], root)
        assert prev_key is None or prev_key < key
        prev_key = key
        expect = csgraph.breadth_first_order(m, root, directed=False, return_predecessors=False)
        assert seq[pos:pos + members.size] == expect.tolist()
        pos += members.size


@pytest.mark.parametrize("el", GRAPHS, ids=lambda e: e.name)
def test_hybrid_is_stable_degree_sort_of_bfs(el):
    g = oracle.Graph.from_edgelist(el)
    deg = g.degree().astype(np.int64)
    bfs_pos = {v: i for i, v in enumerate(sequence(g, "bfs"))}
    hyb = sequence(g, "hybrid")
    assert sorted(hyb) == list(range(g.n))
    for x, y in zip(hyb, hyb[1:]):
        assert deg[x] > deg[y] or (deg[x] == deg[y] and bfs_pos[x] < bfs_pos[y])


@pytest.mark.parametrize("el", GRAPHS, ids=lambda e: e.name)
def test_strong_runs_properties(el):
    """The highest-degree vertex's run comes first (the vertex, then its
    neighbours ascending), and every vertex is labelled no later than the
    run of its highest-degree neighbour."""
    g = oracle.Graph.from_edgelist(el)
    deg = g.degree().astype(np.int64)
    seq = sequence(g, "strong_runs")
    assert sorted(seq) == list(range(g.n))
    m = _csr(g)
    nbrs = lambda v: m.indices[m.indptr[v]:m.indptr[v + 1]].tolist()
    first = min(range(g.n), key=lambda v: (-deg[v], v))
    assert seq[:1 + deg[first]] == [first] + nbrs(first)
    label = {v: i for i, v in enumerate(seq)}
    visit = sorted(range(g.n), key=lambda v: (-deg[v], v))
    vpos = {v: i for i, v in enumerate(visit)}
    # labels handed out before visiting vertex number k: its run ends at most at
    # 1 + sum of (1 + degree) over the vertices visited up to k
    bound = np.cumsum([1 + deg[v] for v in visit])
    for v in range(g.n):
        if deg[v] == 0:
            continue
        h = min(nbrs(v), key=lambda w: vpos[w])
        assert label[v] < bound[min(vpos[h], vpos[v])]


def brute_rooted(el, rank):
    """T, K and per-root counts by subsets; root = vertex of smallest rank."""
    n = el.n
    adj = [set() for _ in range(n)]
    for a, b in zip(el.src.tolist(), el.dst.tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    r3 = np.zeros(n, np.uint64)
    r4 = np.zeros(n, np.uint64)
    for k, out in ((3, r3), (4, r4)):
        for t in itertools.combinations(range(n), k):
            if all(y in adj[x] for x, y in itertools.combinations(t, 2)):
                out[min(t, key=lambda v: rank[v])] += 1
    return r3, r4


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("n,p,seed", [(12, 0.5, 1), (18, 0.35, 2), (22, 0.6, 3)])
def test_rooted_counts_by_brute_force(order, n, p, seed):
    el = inputs.gnp(n, p, seed=seed)
    g = oracle.Graph.from_edgelist(el, order)
    r3, r4 = brute_rooted(el, g.rank())
    t = g.triangles(rooted=True)
    k = g.cliques4(rooted=True)
    np.testing.assert_array_equal(t["root"], r3)
    np.testing.assert_array_equal(k["root"], r4)
    assert t["count"] == int(r3.sum()) and k["count"] == int(r4.sum())


@pytest.mark.parametrize("el", GRAPHS + [inputs.rmat(11, 16, seed=2)], ids=lambda e: e.name)
def test_counts_do_not_depend_on_ordering(el):
    base = oracle.Graph.from_edgelist(el)
    T, K = base.count(3), base.count(4)
    assert 3 * T == base.sym_triangle_sum()
    for order in ORDERS:
        g = oracle.Graph.from_edgelist(el, order)
        off, nbr = g.oriented()
        rows = np.repeat(np.arange(g.n), np.diff(off.astype(np.int64)))
        assert np.all(nbr.astype(np.int64) > rows)  # directed low -> high rank
        assert g.count(3) == T and g.count(4) == K


def test_rerank_rejects_non_permutations():
    g = oracle.Graph.from_edgelist(inputs.cycle(5))
    with pytest.raises(ValueError):
        g.rerank(np.array([0, 1, 2, 3, 3], np.uint32))
    with pytest.raises(ValueError):
        g.rerank(np.array([0, 1, 2, 3, 5], np.uint32))
    with pytest.raises(ValueError):
        sequence(g, "shingle")
    assert g.count(3) == 0
