"""Pins for the CPU oracle against facts it does not compute itself.

Brute force over vertex subsets, linear algebra (trace(A^3) = 6T), textbook
graph counts (tests/golden), closed forms on families of graphs, and
invariants that the method fixes (paper section 2.1 and appendix A: ordering
and pruning change speed, never the set of results).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import inputs
from golden_io import all_fixtures, load


def brute(el):
    """All 3- and 4-subsets, adjacency-set test; roots by (degree, id) rank."""
    n = el.n
    adj = [set() for _ in range(n)]
    for a, b in zip(el.src.tolist(), el.dst.tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    deg = [len(s) for s in adj]
    key = lambda v: (deg[v], v)
    T = K = 0
    root3 = np.zeros(n, np.uint64)
    root4 = np.zeros(n, np.uint64)
    c3 = np.zeros(n, np.uint64)
    c4 = np.zeros(n, np.uint64)
    for t in itertools.combinations(range(n), 3):
        if all(y in adj[x] for x, y in itertools.combinations(t, 2)):
            T += 1
            root3[min(t, key=key)] += 1
            for v in t:
                c3[v] += 1
    for q in itertools.combinations(range(n), 4):
        if all(y in adj[x] for x, y in itertools.combinations(q, 2)):
            K += 1
            root4[min(q, key=key)] += 1
            for v in q:
                c4[v] += 1
    return T, K, root3, root4, c3, c4


def full(el):
    g = oracle.Graph.from_edgelist(el)
    t = g.triangles(rooted=True, per_vertex=True)
    k = g.cliques4(rooted=True, per_vertex=True)
    return g, t, k


@pytest.mark.parametrize("n,p,seed", [(n, p, s) for n in (6, 11, 17, 24)
                                      for p in (0.15, 0.4, 0.7, 0.95) for s in (1, 2)])
def test_brute_force_random(n, p, seed):
    el = inputs.gnp(n, p, seed)
    T, K, r3, r4, c3, c4 = brute(el)
    g, t, k = full(el)
    assert t["count"] == T and k["count"] == K
    np.testing.assert_array_equal(t["root"], r3)
    np.testing.assert_array_equal(k["root"], r4)
    np.testing.assert_array_equal(t["per_vertex"], c3)
    np.testing.assert_array_equal(k["per_vertex"], c4)


@pytest.mark.parametrize("n,p,seed", [(n, p, s) for n in (9, 20, 26) for p in (0.3, 0.8) for s in (1, 2)])
def test_4cliques_rooted_at_brute_force(n, p, seed):
    """4-cliques rooted at a chosen vertex subset (repeats in the list
    ignored) against brute force over 4-subsets; unlisted ids stay 0."""
    el = inputs.gnp(n, p, seed)
    _, _, _, r4, _, _ = brute(el)
    g = oracle.Graph.from_edgelist(el)
    pick = np.arange(0, n, 3, dtype=np.uint32)
    got = g.cliques4_rooted_at(np.concatenate([pick, pick[:2]]))
    want = np.zeros(n, np.uint64)
    want[pick] = r4[pick]
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(g.cliques4_rooted_at(np.arange(n)), r4)
    with pytest.raises(ValueError):
        g.cliques4_rooted_at([n])


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_messy_input(seed):
    el = inputs.messy(inputs.gnp(16, 0.5, seed), seed)
    T, K, r3, r4, _, _ = brute(el)
    _, t, k = full(el)
    assert (t["count"], k["count"]) == (T, K)
    np.testing.assert_array_equal(t["root"], r3)
    np.testing.assert_array_equal(k["root"], r4)


@pytest.mark.parametrize("n,p,seed", [(150, 0.1, 1), (200, 0.3, 2), (90, 0.8, 3)])
def test_trace_formula(n, p, seed):
    """trace(A^3) = 6T for the symmetric 0/1 adjacency matrix A."""
    el = inputs.gnp(n, p, seed)
    A = np.zeros((n, n), dtype=np.int64)
    A[el.src, el.dst] = 1
    A[el.dst, el.src] = 1
    np.fill_diagonal(A, 0)
    six_t = int(np.trace(A @ A @ A))
    assert oracle.Graph.from_edgelist(el).triangles()["count"] * 6 == six_t


@pytest.mark.parametrize("path", all_fixtures(), ids=lambda p: p.rsplit("/", 1)[-1])
def test_golden(path):
    n, s, d, expect = load(path)
    g = oracle.Graph(n, s, d)
    assert g.triangles()["count"] == expect["T"]
    assert g.cliques4()["count"] == expect["K"]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 33, 64, 101])
def test_complete_closed_form(n):
    g = oracle.Graph.from_edgelist(inputs.complete(n))
    t = g.triangles()
    assert t["count"] == math.comb(n, 3)
    assert g.cliques4()["count"] == math.comb(n, 4)
    # byte model on K_n: out-degrees are n-1, ..., 0; every pair sums two of them
    assert t["bytes"] == 2 * n * (n - 1) ** 2


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 9, 33, 64, 101])
def test_complete_byte_models(n):
    """The byte models on K_n, summed by hand over its ranks 0..n-1, where
    N+(r) = {r+1, ..., n-1}.

    B_K4: for x<y<z, |S_xy| = n-1-y and |N+(z)| = n-1-z; the triple sum of
    y + z is C(n,3) (3(n-1)/2 - (n-3)/4), which gives (3n-5) C(n,3) beside
    B_merge = 2n(n-1)^2.
    B_K4_held: the pair (x,y) extends iff y <= n-3; with k = n-1-y its reads
    are 12 + 4k, its level-2 reads 2k^2 + 6k, and each x <= n-4 adds
    16 + 4(n-1-x): 4 C(n+3,4) + 2n(n-1) - 24n for n >= 3.
    B_target: held sets y = 1..n-2 (n-2 of them, (n-1)(n-2)/2 members); y has
    y in-edges, each streaming the n-1-y members above y, C(n,3) in all.
    """
    g = oracle.Graph.from_edgelist(inputs.complete(n))
    k = g.cliques4()
    assert k["bytes"] == 2 * n * (n - 1) ** 2 + (3 * n - 5) * math.comb(n, 3)
    want_held = 4 * math.comb(n + 3, 4) + 2 * n * (n - 1) - 24 * n if n >= 3 else 0
    assert k["held_bytes"] == want_held
    # its element tests: y extended pairs end at y, each testing k = n-1-y
    # members of N+(y) and, for z in S_xy = {y+1, ..., n-1}, k(k-1)/2 more
    assert k["held_tests"] == sum(y * math.comb(n - y, 2) for y in range(1, n - 2))
    r = g.target_reads()
    if n >= 2:
        assert r["held_sets"] == n - 2
        assert r["held_members"] == r["parts"] == (n - 1) * (n - 2) // 2
        assert r["streamed"] == math.comb(n, 3)
        assert r["bytes"] == 6 * (n - 1) * (n - 2) + 32 * (n - 2) + 4 * math.comb(n, 3)
    else:
        assert r["bytes"] == 0


def brute_bytes(el):
    """The byte models by brute force over rank-ordered vertex triples, with
    ranks and out-sets derived here from the adjacency sets."""
    n = el.n
    adj = [set() for _ in range(n)]
    for a, b in zip(el.src.tolist(), el.dst.tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    order = sorted(range(n), key=lambda v: (len(adj[v]), v))
    rk = {v: i for i, v in enumerate(order)}
    up = {v: {w for w in adj[v] if rk[w] > rk[v]} for v in range(n)}
    d = {v: len(up[v]) for v in range(n)}
    b_merge = sum(4 * (d[x] + d[y]) for x in range(n) for y in up[x])
    b_k4 = b_merge
    held = tests = 0
    extended_roots = set()
    for x in range(n):
        for y in up[x]:
            after = sum(1 for w in up[x] if rk[w] > rk[y])
            ext = after >= 2 and d[y] >= 2
            s = up[x] & up[y]
            if ext:
                extended_roots.add(x)
                held += 12 + 4 * d[y]
                tests += d[y]
            for z in s:                     # triangle x < y < z in rank order
                b_k4 += 4 * (len(s) + d[z])
                if ext and len(s) >= 2:
                    held += 8 + 4 * d[z]
                    tests += d[z]
    held += sum(16 + 4 * d[x] for x in extended_roots)
    # target staging: y held when some x -> y exists and N+(y) is not empty
    tgt = 0
    for y in range(n):
        ins = [x for x in range(n) if y in up[x]]
        if ins and d[y] > 0:
            tgt += 32 + 4 * d[y]
            for x in ins:
                tgt += 8 + 4 * sum(1 for w in up[x] if rk[w] > rk[y])
    return b_merge, b_k4, held, tgt, tests


@pytest.mark.parametrize("n,p,seed", [(n, p, s) for n in (7, 13, 22, 30)
                                      for p in (0.2, 0.5, 0.85) for s in (1, 2)])
def test_byte_models_brute_force(n, p, seed):
    el = inputs.gnp(n, p, seed)
    g = oracle.Graph.from_edgelist(el)
    b_merge, b_k4, held, tgt, tests = brute_bytes(el)
    assert g.triangles()["bytes"] == b_merge
    k = g.cliques4()
    assert (k["bytes"], k["held_bytes"], k["held_tests"]) == (b_k4, held, tests)
    assert g.target_reads()["bytes"] == tgt


@pytest.mark.parametrize("seed", range(3))
def test_byte_models_messy_and_sparse(seed):
    """Sinks (empty out-sets), isolated vertices and messy input."""
    el = inputs.messy(inputs.disjoint_union(inputs.gnp(18, 0.3, seed), inputs.star(6),
                                            inputs.path(5)), seed)
    g = oracle.Graph.from_edgelist(el)
    b_merge, b_k4, held, tgt, _ = brute_bytes(el)
    k = g.cliques4()
    assert (g.triangles()["bytes"], k["bytes"], k["held_bytes"]) == (b_merge, b_k4, held)
    assert g.target_reads()["bytes"] == tgt


def test_batch_oracle_equals_single_graphs():
    """The parallel batch count is the single-graph count of each graph, in
    any order of the graphs."""
    b = inputs.batch_chung_lu(60, seed=11)
    counts, bm, bt = oracle.batch_triangles(b.n_vertices, b.edge_off, b.src, b.dst)
    for i in range(60):
        g = oracle.Graph.from_edgelist(b.graph(i))
        t = g.triangles()
        assert (int(counts[i]), int(bm[i])) == (t["count"], t["bytes"])
        assert int(bt[i]) == g.target_reads()["bytes"]
    perm = np.random.default_rng(3).permutation(60)
    nv = np.asarray(b.n_vertices)[perm]
    parts_s = [b.graph(i).src for i in perm]
    parts_d = [b.graph(i).dst for i in perm]
    off = np.concatenate([[0], np.cumsum([len(x) for x in parts_s])]).astype(np.uint64)
    c2, _, _ = oracle.batch_triangles(nv, off, np.concatenate(parts_s), np.concatenate(parts_d))
    np.testing.assert_array_equal(c2, counts[perm])
    with pytest.raises(ValueError):
        oracle.batch_triangles([3], [0, 1], np.array([0], np.uint32), np.array([3], np.uint32))


@pytest.mark.parametrize("el", [inputs.grid(7, 9), inputs.complete_bipartite(6, 9), inputs.star(40),
                                inputs.random_tree(300, 3), inputs.path(50), inputs.cycle(4),
                                inputs.cycle(5), inputs.cycle(97)], ids=lambda e: e.name)
def test_triangle_free(el):
    g = oracle.Graph.from_edgelist(el)
    assert g.triangles()["count"] == 0
    assert g.cliques4()["count"] == 0


def test_small_families():
    assert oracle.Graph.from_edgelist(inputs.cycle(3)).triangles()["count"] == 1
    for k in (4, 5, 6, 11, 50):
        g = oracle.Graph.from_edgelist(inputs.wheel(k))
        assert g.triangles()["count"] == k
        assert g.cliques4()["count"] == 0
    g = oracle.Graph.from_edgelist(inputs.wheel(3))   # W3 is K4
    assert (g.triangles()["count"], g.cliques4()["count"]) == (4, 1)
    for k in (1, 2, 7, 30):
        g = oracle.Graph.from_edgelist(inputs.friendship(k))
        assert (g.triangles()["count"], g.cliques4()["count"]) == (k, 0)


@pytest.mark.parametrize("seed", range(3))
def test_invariants_er(seed):
    el = inputs.erdos_renyi_gnm(600, 9000, seed)
    g, t, k = full(el)
    T, K = t["count"], k["count"]
    assert T > 0
    assert int(t["per_vertex"].sum()) == 3 * T
    assert int(k["per_vertex"].sum()) == 4 * K
    assert int(t["root"].sum()) == T and int(k["root"].sum()) == K
    assert g.sym_triangle_sum() == 3 * T
    assert g.sym_4clique_sum() == 6 * K
    assert g.sym_ordered_triangles() == 6 * T
    assert g.sym_ordered_4cliques() == 24 * K


def test_invariants_rmat():
    el = inputs.rmat(11, 16, seed=7)
    g, t, k = full(el)
    T, K = t["count"], k["count"]
    assert T > 1000 and K > 1000
    assert int(t["per_vertex"].sum()) == 3 * T
    assert int(k["per_vertex"].sum()) == 4 * K
    assert g.sym_triangle_sum() == 3 * T
    assert g.sym_4clique_sum() == 6 * K
    # ordering only changes speed: relabelled copies give the same totals
    for s in (1, 2):
        g2 = oracle.Graph.from_edgelist(inputs.relabel(el, s))
        assert g2.triangles()["count"] == T and g2.cliques4()["count"] == K
    # messy writing of the same graph
    g3 = oracle.Graph.from_edgelist(inputs.messy(el, 5))
    assert g3.m == g.m
    t3 = g3.triangles(rooted=True)
    assert t3["count"] == T
    np.testing.assert_array_equal(t3["root"], t["root"])


def test_disjoint_union_additive():
    parts = [inputs.gnp(30, 0.5, 1), inputs.complete(12), inputs.wheel(9), inputs.rmat(8, 8, seed=2)]
    tot_t = sum(oracle.Graph.from_edgelist(p).triangles()["count"] for p in parts)
    tot_k = sum(oracle.Graph.from_edgelist(p).cliques4()["count"] for p in parts)
    g = oracle.Graph.from_edgelist(inputs.disjoint_union(*parts))
    assert g.triangles()["count"] == tot_t
    assert g.cliques4()["count"] == tot_k


def test_rooted_partition_additive():
    el = inputs.rmat(10, 16, seed=3)
    g = oracle.Graph.from_edgelist(el)
    for pat, fn in ((3, g.triangles), (4, g.cliques4)):
        r = fn(rooted=True)
        key = inputs.stream_key(9, pat)
        part = (inputs.rand_u64(key, 0, el.n) % np.uint64(3)).astype(np.int64)
        sums = [oracle.rooted_count(r["root"], np.nonzero(part == i)[0]) for i in range(3)]
        assert sum(sums) == r["count"]
        assert oracle.rooted_count(r["root"], np.arange(el.n)) == r["count"]
        # duplicates in a root list are ignored
        assert oracle.rooted_count(r["root"], [5, 5, 7, 7]) == oracle.rooted_count(r["root"], [5, 7])


def test_range_split_matches_whole():
    el = inputs.rmat(10, 16, seed=4)
    g = oracle.Graph.from_edgelist(el)
    whole = g.triangles()
    mid = el.n // 3
    a = g.triangles(x_begin=0, x_end=mid)
    b = g.triangles(x_begin=mid)
    assert a["count"] + b["count"] == whole["count"]
    assert a["bytes"] + b["bytes"] == whole["bytes"]
    assert a["edges"] + b["edges"] == g.m


def test_orientation_properties():
    el = inputs.rmat(12, 16, seed=5)
    g = oracle.Graph.from_edgelist(el)
    off, nbr = g.oriented()
    rank = g.rank()
    deg = g.degree()
    assert int(off[-1]) == g.m
    # rank is a permutation ordered by (degree, id)
    order = np.argsort(rank)
    assert np.array_equal(np.sort(rank), np.arange(el.n))
    d_sorted = deg[order]
    assert np.all(np.diff(d_sorted.astype(np.int64)) >= 0)
    same = np.diff(d_sorted.astype(np.int64)) == 0
    assert np.all(np.diff(order.astype(np.int64))[same] > 0)
    # rows point upward, are strictly increasing, out-degree <= sqrt(2m)
    dplus = np.diff(off.astype(np.int64))
    rows = np.repeat(np.arange(el.n), dplus)
    assert np.all(nbr.astype(np.int64) > rows)
    for r in range(el.n):
        seg = nbr[off[r]:off[r + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)
    assert dplus.max() <= math.isqrt(2 * g.m) + 1


def test_empty_and_rejects():
    g = oracle.Graph(5, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert g.m == 0 and g.triangles()["count"] == 0 and g.cliques4()["count"] == 0
    g = oracle.Graph(3, np.array([0, 1, 2], np.uint32), np.array([0, 1, 2], np.uint32))
    assert g.m == 0
    with pytest.raises(ValueError):
        oracle.Graph(3, np.array([0], np.uint32), np.array([3], np.uint32))


def test_threads_agree():
    el = inputs.rmat(12, 16, seed=6)
    g = oracle.Graph.from_edgelist(el)
    a = g.triangles(threads=1)["count"]
    b = g.triangles(threads=4)["count"]
    assert a == b
    assert g.cliques4(threads=1)["count"] == g.cliques4(threads=3)["count"]
