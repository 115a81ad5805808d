"""Seeded synthetic graph inputs.

This module only draws raw edge lists (pairs of uint32 vertex ids, possibly
with duplicates, both directions and self-loops) and request streams.  It holds
none of the counting method's arithmetic: no cleaning, ranking, orientation,
layout choice or intersection.  Both the CPU oracle's tests and the GPU path
consume the arrays it returns, so both sides always see the same input.

Randomness comes from one counter-based generator, splitmix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
value for (key, counter) is the splitmix64 output function applied to
key + (counter + 1) * 0x9E3779B97F4A7C15.  Keys are derived from
(seed, stream) by the same mixer, so every graph of a batch and every draw is
addressable without sequential state.

Workload recipes (the paper measures on real social/citation graphs that are
not available here; these synthetic families stand in for them):

* R-MAT(scale, edge_factor, a, b, c, d): edge_factor * 2**scale samples, each
  choosing one quadrant per level with probabilities (a, b, c, d) quantised to
  1/65536; no noise, no vertex permutation.
* Erdos-Renyi G(n, M): M distinct unordered pairs drawn uniformly.
* Chung-Lu power law: round(n*dbar/2) endpoint pairs; each end is floor(x),
  x drawn by inverse CDF from the density proportional to
  (x+1)**(-1/(gamma-1)) on [0, n).
* Batched Chung-Lu: n_i = round(exp U[ln 64, ln 16384]),
  dbar_i = exp U[ln 8, ln 64], gamma = 2.1, one key per graph.
* Small structured graphs (complete, grid, cycle, wheel, ...) for pins.
* Sets with a dense region (pairwise intersection by layout): 2 P sets of
  `size` distinct ids in [0, domain).  Pair p = (2p, 2p+1) shares one region
  [c_p, c_p + r) with c_p uniform; each of its sets holds
  k_d = round(dense_frac * size) ids of the region (r = the larger of k_d and
  ceil(k_d / density)) and size - k_d ids of the rest of the domain, each part
  by jittered sampling: the part's range is cut into as many equal strata as
  it has members and each stratum gives one uniform id.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    """splitmix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _mix_int(x: int) -> int:
    x &= _MASK64
    x ^= x >> 30
    x = (x * 0xBF58476D1CE4E5B9) & _MASK64
    x ^= x >> 27
    x = (x * 0x94D049BB133111EB) & _MASK64
    x ^= x >> 31
    return x


def stream_key(seed: int, stream: int = 0) -> int:
    """Key for stream `stream` of seed `seed` (both non-negative ints)."""
    k = _mix_int((seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) & _MASK64)
    return _mix_int((k ^ ((stream + 1) * 0xD1B54A32D192ED03)) & _MASK64)


def rand_u64(key: int, start: int, count: int) -> np.ndarray:
    """Counter-based uint64 draws for counters start .. start+count-1."""
    ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + ctr * _GOLDEN
        return _mix(z)


def rand_uniform(key: int, start: int, count: int) -> np.ndarray:
    """Uniform float64 in [0, 1) with 53 random bits."""
    return (rand_u64(key, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ---------------------------------------------------------------------------
# Graph families
# ---------------------------------------------------------------------------

@dataclass
class EdgeList:
    """Raw directed pairs on vertices 0..n-1 (duplicates / loops allowed)."""
    n: int
    src: np.ndarray  # uint32
    dst: np.ndarray  # uint32
    name: str = ""

    @property
    def m_raw(self) -> int:
        return int(self.src.shape[0])


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0, chunk: int = 1 << 20) -> EdgeList:
    """R-MAT generator (Chakrabarti, Zhan, Faloutsos 2004), no noise.

    Each 64-bit draw supplies four 16-bit level choices; quadrant (row, col)
    is (0,0) below a, (0,1) below a+b, (1,0) below a+b+c, else (1,1).  The row
    bit goes to src and the column bit to dst, most significant level first.
    """
    import concurrent.futures as cf
    import os
    n = 1 << scale
    m = edge_factor * n
    key = stream_key(seed, 0x52AA7)
    ta = np.uint64(round(a * 65536))
    tb = np.uint64(round((a + b) * 65536))
    tc = np.uint64(round((a + b + c) * 65536))
    draws_per = (scale + 3) // 4
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)

    def fill(s0):
        cnt = min(chunk, m - s0)
        r = rand_u64(key, s0 * draws_per, cnt * draws_per).reshape(cnt, draws_per)
        s = np.zeros(cnt, dtype=np.uint64)
        d = np.zeros(cnt, dtype=np.uint64)
        lvl = 0
        for k in range(draws_per):
            col = r[:, k]
            for j in range(4):
                if lvl == scale:
                    break
                u = (col >> np.uint64(16 * j)) & np.uint64(0xFFFF)
                rowbit = (u >= tb).astype(np.uint64)
                colbit = (((u >= ta) & (u < tb)) | (u >= tc)).astype(np.uint64)
                s = (s << np.uint64(1)) | rowbit
                d = (d << np.uint64(1)) | colbit
                lvl += 1
        src[s0:s0 + cnt] = s.astype(np.uint32)
        dst[s0:s0 + cnt] = d.astype(np.uint32)

    starts = list(range(0, m, chunk))
    nt = min(16, os.cpu_count() or 1)
    if len(starts) <= 1 or nt == 1:
        for s0 in starts:
            fill(s0)
    else:
        with cf.ThreadPoolExecutor(max_workers=nt) as ex:
            list(ex.map(fill, starts))
    return EdgeList(n, src, dst, f"rmat{scale}_ef{edge_factor}_s{seed}")


def _pair_from_index(k: np.ndarray, n: int):
    """Map k in [0, n(n-1)/2) to the k-th pair (i<j) in row-major order."""
    kf = k.astype(np.float64)
    # i = largest i with i*(2n-i-1)/2 <= k
    i = np.floor(((2 * n - 1) - np.sqrt((2 * n - 1) ** 2 - 8 * kf)) / 2).astype(np.int64)
    i = np.clip(i, 0, n - 2)
    base = i * (2 * n - i - 1) // 2
    # fix float rounding at the boundaries
    over = base > k
    while over.any():
        i[over] -= 1
        base = i * (2 * n - i - 1) // 2
        over = base > k
    nxt = (i + 1) * (2 * n - i - 2) // 2
    under = nxt <= k
    while under.any():
        i[under] += 1
        base = i * (2 * n - i - 1) // 2
        nxt = (i + 1) * (2 * n - i - 2) // 2
        under = nxt <= k
    j = k - base + i + 1
    return i, j


def erdos_renyi_gnm(n: int, m: int, seed: int = 0) -> EdgeList:
    """G(n, M): M distinct unordered pairs, uniformly at random.

    Draws candidate pair indices in counter order and keeps the first M
    distinct ones.
    """
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("m exceeds the number of pairs")
    key = stream_key(seed, 0xE5)
    got = np.empty(0, dtype=np.int64)
    start = 0
    while True:
        want = max(2 * (m - got.size), 1024)
        u = rand_u64(key, start, want)
        start += want
        cand = (u % np.uint64(total)).astype(np.int64)
        allc = np.concatenate([got, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        got = allc[first]
        if got.size >= m:
            got = got[:m]
            break
    i, j = _pair_from_index(got, n)
    return EdgeList(n, i.astype(np.uint32), j.astype(np.uint32), f"er{n}_m{m}_s{seed}")


def _powerlaw_ends(n: np.ndarray, u: np.ndarray, gamma: float, gidx=None) -> np.ndarray:
    """floor(x) for x with density proportional to (x+1)^(-1/(gamma-1)) on [0, n).

    n holds one size per graph and gidx maps each draw u to its graph (None:
    one graph).  Inverse CDF: x = (1 + u((n+1)^b - 1))^(1/b) - 1, b = 1 - 1/(gamma-1).
    """
    beta = 1.0 - 1.0 / (gamma - 1.0)
    nf = np.asarray(n, dtype=np.float64)
    sel = (lambda a: a) if gidx is None else (lambda a: a[gidx])
    if abs(beta) < 1e-12:
        x = np.expm1(u * sel(np.log1p(nf)))
    else:
        top = np.expm1(beta * np.log1p(nf))   # (n+1)^b - 1
        x = np.expm1(np.log1p(u * sel(top)) * (1.0 / beta))
    e = np.floor(x).astype(np.int64)
    np.clip(e, 0, sel(np.asarray(n, dtype=np.int64)) - 1, out=e)
    return e


def _chung_lu_many(ns, ds, gamma, seed, graph_ids, chunk=1 << 22, threads=None):
    """Endpoint pairs of several Chung-Lu graphs; returns (src, dst, edge_off).

    Graphs are cut into chunks of about `chunk` draws that a thread pool fills
    (numpy releases the GIL); every draw is addressed by (graph, counter), so
    the result does not depend on the chunking or the thread count.
    """
    import concurrent.futures as cf
    import os
    ns = np.asarray(ns, dtype=np.int64)
    ms = np.rint(ns * np.asarray(ds, dtype=np.float64) / 2.0).astype(np.int64)
    off = np.zeros(ns.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(ms).astype(np.uint64)
    src = np.empty(int(off[-1]), dtype=np.uint32)
    dst = np.empty(int(off[-1]), dtype=np.uint32)
    keys = np.array([stream_key(seed, 0xC1000000 + int(g)) for g in graph_ids], dtype=np.uint64)
    spans = []
    g0 = 0
    while g0 < ns.size:
        g1, tot = g0, 0
        while g1 < ns.size and (tot == 0 or tot + 2 * ms[g1] <= chunk):
            tot += 2 * int(ms[g1])
            g1 += 1
        spans.append((g0, g1, tot))
        g0 = g1

    def fill(span):
        g0, g1, tot = span
        if tot == 0:
            return
        cnt = 2 * ms[g0:g1]
        gidx = np.repeat(np.arange(g0, g1), cnt)
        starts = np.repeat(np.cumsum(cnt) - cnt, cnt)
        ctr = (np.arange(tot, dtype=np.int64) - starts + 1).astype(np.uint64)
        with np.errstate(over="ignore"):
            z = _mix(keys[gidx] + ctr * _GOLDEN)
        u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        ends = _powerlaw_ends(ns, u, gamma, gidx).astype(np.uint32)
        a = int(off[g0])
        src[a:a + tot // 2] = ends[0::2]
        dst[a:a + tot // 2] = ends[1::2]

    nt = threads or min(16, os.cpu_count() or 1)
    if len(spans) == 1 or nt == 1:
        for sp in spans:
            fill(sp)
    else:
        with cf.ThreadPoolExecutor(max_workers=nt) as ex:
            list(ex.map(fill, spans))
    return src, dst, off


def chung_lu(n: int, avg_degree: float, gamma: float = 2.1, seed: int = 0,
             graph: int = 0) -> EdgeList:
    """Chung-Lu style power-law graph: round(n*dbar/2) endpoint pairs, each end
    floor(x) with x drawn from the density proportional to (x+1)^(-1/(gamma-1))
    on [0, n) (vertex i's expected degree falls off as i^(-1/(gamma-1)))."""
    s, d, _ = _chung_lu_many([n], [avg_degree], gamma, seed, [graph])
    return EdgeList(n, s, d, f"cl{n}_d{avg_degree:.2f}_g{gamma}_s{seed}_{graph}")


@dataclass
class BatchEdges:
    """Many independent raw edge lists, concatenated."""
    n_vertices: np.ndarray   # uint32 [G]
    edge_off: np.ndarray     # uint64 [G+1] into src/dst
    src: np.ndarray          # uint32, local ids per graph
    dst: np.ndarray
    name: str = ""

    @property
    def n_graphs(self) -> int:
        return int(self.n_vertices.shape[0])

    def graph(self, i: int) -> EdgeList:
        a, b = int(self.edge_off[i]), int(self.edge_off[i + 1])
        return EdgeList(int(self.n_vertices[i]), self.src[a:b], self.dst[a:b], f"{self.name}[{i}]")


def batch_sizes(num_graphs: int, seed: int, n_lo: int = 64, n_hi: int = 16384,
                d_lo: float = 8.0, d_hi: float = 64.0):
    """Per-graph (n_i, dbar_i): log-uniform n and mean degree."""
    key = stream_key(seed, 0xBA7C4)
    u = rand_uniform(key, 0, 2 * num_graphs).reshape(num_graphs, 2)
    n = np.rint(np.exp(math.log(n_lo) + u[:, 0] * (math.log(n_hi) - math.log(n_lo)))).astype(np.int64)
    d = np.exp(math.log(d_lo) + u[:, 1] * (math.log(d_hi) - math.log(d_lo)))
    d = np.minimum(d, (n - 1).astype(np.float64))
    return n, d


def batch_chung_lu(num_graphs: int, seed: int = 4, gamma: float = 2.1, n_lo: int = 64,
                   n_hi: int = 16384, d_lo: float = 8.0, d_hi: float = 64.0) -> BatchEdges:
    """Graph g is chung_lu(n_g, dbar_g, gamma, seed, g) with (n_g, dbar_g) from batch_sizes."""
    n, d = batch_sizes(num_graphs, seed, n_lo, n_hi, d_lo, d_hi)
    src, dst, off = _chung_lu_many(n, d, gamma, seed, np.arange(num_graphs))
    return BatchEdges(n.astype(np.uint32), off, src, dst, f"batch_cl{num_graphs}_s{seed}")


# ---------------------------------------------------------------------------
# Small structured graphs
# ---------------------------------------------------------------------------

def _el(n, pairs, name):
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return EdgeList(n, p[:, 0].astype(np.uint32), p[:, 1].astype(np.uint32), name)


def complete(n: int) -> EdgeList:
    i, j = np.triu_indices(n, 1)
    return EdgeList(n, i.astype(np.uint32), j.astype(np.uint32), f"K{n}")


def complete_bipartite(a: int, b: int) -> EdgeList:
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return EdgeList(a + b, i.ravel().astype(np.uint32), j.ravel().astype(np.uint32), f"K{a},{b}")


def grid(rows: int, cols: int) -> EdgeList:
    pairs = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                pairs.append((v, v + 1))
            if r + 1 < rows:
                pairs.append((v, v + cols))
    return _el(rows * cols, pairs, f"grid{rows}x{cols}")


def cycle(n: int) -> EdgeList:
    return _el(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}")


def path(n: int) -> EdgeList:
    return _el(n, [(i, i + 1) for i in range(n - 1)], f"P{n}")


def star(k: int) -> EdgeList:
    return _el(k + 1, [(0, i) for i in range(1, k + 1)], f"S{k}")


def wheel(k: int) -> EdgeList:
    """k-cycle rim on 1..k plus hub 0."""
    pairs = [(0, i) for i in range(1, k + 1)]
    pairs += [(i, i % k + 1) for i in range(1, k + 1)]
    return _el(k + 1, pairs, f"W{k}")


def friendship(k: int) -> EdgeList:
    """k triangles sharing the single vertex 0."""
    pairs = []
    for t in range(k):
        a, b = 1 + 2 * t, 2 + 2 * t
        pairs += [(0, a), (0, b), (a, b)]
    return _el(2 * k + 1, pairs, f"F{k}")


def random_tree(n: int, seed: int = 0) -> EdgeList:
    key = stream_key(seed, 0x7EE)
    u = rand_u64(key, 0, max(n - 1, 0))
    pairs = [(i, int(u[i - 1] % np.uint64(i))) for i in range(1, n)]
    return _el(n, pairs, f"tree{n}_s{seed}")


def gnp(n: int, p: float, seed: int = 0) -> EdgeList:
    """G(n, p) over unordered pairs (for small pins)."""
    i, j = np.triu_indices(n, 1)
    u = rand_uniform(stream_key(seed, 0x6A9), 0, i.size)
    keep = u < p
    return EdgeList(n, i[keep].astype(np.uint32), j[keep].astype(np.uint32), f"gnp{n}_{p}_s{seed}")


def disjoint_union(*graphs: EdgeList) -> EdgeList:
    srcs, dsts, base = [], [], 0
    for g in graphs:
        srcs.append(g.src.astype(np.int64) + base)
        dsts.append(g.dst.astype(np.int64) + base)
        base += g.n
    s = np.concatenate(srcs) if srcs else np.zeros(0, np.int64)
    d = np.concatenate(dsts) if dsts else np.zeros(0, np.int64)
    return EdgeList(base, s.astype(np.uint32), d.astype(np.uint32), "+".join(g.name for g in graphs))


def relabel(g: EdgeList, seed: int = 0) -> EdgeList:
    """Apply a seeded random permutation to the vertex ids."""
    key = stream_key(seed, 0x9E7)
    perm = np.argsort(rand_u64(key, 0, g.n), kind="stable").astype(np.uint32)
    return EdgeList(g.n, perm[g.src], perm[g.dst], g.name + f"_perm{seed}")


def messy(g: EdgeList, seed: int = 0) -> EdgeList:
    """Same simple graph, written badly: reversed copies, duplicates, loops, shuffled."""
    key = stream_key(seed, 0x3E55)
    m = g.m_raw
    s = np.concatenate([g.src, g.dst, g.src])
    d = np.concatenate([g.dst, g.src, g.dst])
    if g.n > 0:
        loops = (rand_u64(key, 0, max(m // 4, 1)) % np.uint64(g.n)).astype(np.uint32)
        s = np.concatenate([s, loops])
        d = np.concatenate([d, loops])
    order = np.argsort(rand_u64(key, 1 << 40, s.size), kind="stable")
    return EdgeList(g.n, s[order].astype(np.uint32), d[order].astype(np.uint32), g.name + "_messy")


# ---------------------------------------------------------------------------
# Request streams for the served workload
# ---------------------------------------------------------------------------

@dataclass
class Request:
    t_arrival: float          # seconds from stream start
    pattern: int              # 3 = triangle, 4 = 4-clique
    roots: np.ndarray         # uint32 original vertex ids (distinct)


def request_stream(n_vertices: int, rate_qps: float, duration_s: float, seed: int = 5,
                   k4_share: float = 0.2, log2_lo: float = 8.0, log2_hi: float = 16.0,
                   max_requests: int | None = None):
    """Open-loop Poisson arrivals with log-uniform root-set sizes."""
    key = stream_key(seed, 0x5E4E)
    reqs = []
    t = 0.0
    i = 0
    while True:
        u = rand_uniform(key, 4 * i, 3)
        t += -math.log(1.0 - u[0]) / rate_qps
        if t >= duration_s or (max_requests is not None and i >= max_requests):
            break
        size = int(round(2.0 ** (log2_lo + u[1] * (log2_hi - log2_lo))))
        size = max(1, min(size, n_vertices))
        pat = 4 if u[2] < k4_share else 3
        rk = stream_key(seed, 0x100000000 + i)
        if 4 * size > n_vertices:
            # dense root sets: first `size` ids of a seeded permutation
            perm = np.argsort(rand_u64(rk, 0, n_vertices), kind="stable")
            reqs.append(Request(t, pat, perm[:size].astype(np.uint32)))
            i += 1
            continue
        # sparse root sets: draw with oversampling, keep first `size` distinct in draw order
        got = np.empty(0, np.uint32)
        start = 0
        while got.size < size:
            want = 2 * (size - got.size) + 16
            cand = (rand_u64(rk, start, want) % np.uint64(n_vertices)).astype(np.uint32)
            start += want
            allc = np.concatenate([got, cand])
            _, first = np.unique(allc, return_index=True)
            first.sort()
            got = allc[first]
        reqs.append(Request(t, pat, got[:size].copy()))
        i += 1
    return reqs


# ---------------------------------------------------------------------------
# Sets with a dense region
# ---------------------------------------------------------------------------

@dataclass
class SetPairs:
    """Sets members[off[i]:off[i+1]] (ascending, distinct) and pairs [P, 2] of set indices."""
    off: np.ndarray      # uint64 [n_sets + 1]
    members: np.ndarray  # uint32
    pairs: np.ndarray    # uint32 [P, 2]
    name: str = ""

    @property
    def n_sets(self) -> int:
        return int(self.off.size - 1)


def _jittered(key: int, n_sets: int, k: int, span: int) -> np.ndarray:
    """[n_sets, k] ascending distinct values in [0, span): value i of a set is
    uniform in the i-th of k equal strata of [0, span)."""
    if k == 0:
        return np.empty((n_sets, 0), np.int64)
    lo = (np.arange(k, dtype=np.int64) * span) // k
    width = np.diff(np.append(lo, span))
    u = rand_uniform(key, 0, n_sets * k).reshape(n_sets, k)
    return lo + np.minimum((u * width).astype(np.int64), width - 1)


def dense_region_sets(n_pairs: int, size: int, dense_frac: float, domain: int = 1 << 21,
                      density: float = 0.5, seed: int = 0) -> SetPairs:
    """2 n_pairs sets with a dense region shared by the two sets of a pair."""
    k_d = int(round(dense_frac * size))
    k_s = size - k_d
    r = max(k_d, int(math.ceil(k_d / density))) if k_d else 0
    if k_s > domain - r:
        raise ValueError("domain too small for the sparse members")
    n_sets = 2 * n_pairs
    c = (rand_u64(stream_key(seed, 1), 0, n_pairs) % np.uint64(domain - r + 1)).astype(np.int64)
    cs = np.repeat(c, 2)[:, None]
    dense = _jittered(stream_key(seed, 2), n_sets, k_d, r) + cs
    sparse = _jittered(stream_key(seed, 3), n_sets, k_s, domain - r)
    sparse = np.where(sparse >= cs, sparse + r, sparse)
    members = np.sort(np.concatenate([dense, sparse], axis=1), axis=1).astype(np.uint32).ravel()
    off = np.arange(n_sets + 1, dtype=np.uint64) * np.uint64(size)
    sets = np.arange(n_sets, dtype=np.uint32)
    pairs = np.stack([sets[0::2], sets[1::2]], axis=1)
    return SetPairs(off, members, pairs, f"dense_region_{n_pairs}x{size}_f{dense_frac:g}")
