"""CPU oracle for triangle and 4-clique counting -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does, and this package imports
nothing from it: the two share no code.  The arithmetic lives in
``eh_oracle.c`` (plain C, OpenMP over outer vertices); this module only
compiles it with gcc and marshals arrays through ctypes.

Definitions (paper section 2.1 Generic-Join; section 3.3 triangle loop nest;
section 5.2 pruning each undirected edge once by degree-assigned ids):
self-loops are dropped and every other pair is an undirected edge; T counts
3-vertex subsets that are triangles, K counts 4-vertex cliques; the root of
an instance is its vertex of smallest rank, rank = (degree asc, id asc), or
the ranks of another node ordering (appendix A; ``orderings.py``).  Pairwise
set intersection (section 4.2) counts |A & B| for given pairs of sorted sets.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile eh_oracle.c into liboracle.so with gcc -O2 -fopenmp."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                    "-o", tmp, _SRC], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.orc_graph_new.restype = vp
        lib.orc_graph_new.argtypes = [ctypes.c_uint32, ctypes.c_uint64, _u32p, _u32p,
                                      ctypes.POINTER(ctypes.c_int)]
        lib.orc_graph_free.argtypes = [vp]
        lib.orc_graph_rerank.restype = ctypes.c_int
        lib.orc_graph_rerank.argtypes = [vp, _u32p]
        lib.orc_num_edges.restype = ctypes.c_uint64
        lib.orc_num_edges.argtypes = [vp]
        lib.orc_get_edges.argtypes = [vp, _u32p, _u32p]
        lib.orc_get_rank.argtypes = [vp, _u32p]
        lib.orc_get_degree.argtypes = [vp, _u32p]
        lib.orc_get_oriented.argtypes = [vp, _u64p, _u32p]
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_triangles_range.restype = ctypes.c_uint64
        lib.orc_triangles_range.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                            _u64p, _u64p, _u64p, _u64p]
        lib.orc_4cliques_range.restype = ctypes.c_uint64
        lib.orc_4cliques_range.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                           _u64p, _u64p, _u64p, _u64p, _u64p]
        lib.orc_4cliques_rooted_at.restype = ctypes.c_uint64
        lib.orc_4cliques_rooted_at.argtypes = [vp, _u32p, ctypes.c_uint64, ctypes.c_int, _u64p]
        lib.orc_target_reads.restype = ctypes.c_uint64
        lib.orc_target_reads.argtypes = [vp, _u64p]
        lib.orc_batch_triangles.restype = ctypes.c_int
        lib.orc_batch_triangles.argtypes = [ctypes.c_uint32, _u32p, _u64p, _u32p, _u32p,
                                            ctypes.c_int, _u64p, _u64p, _u64p]
        for name in ("orc_sym_triangle_sum", "orc_sym_4clique_sum", "orc_sym_ordered_triangles",
                     "orc_sym_ordered_4cliques"):
            f = getattr(lib, name)
            f.restype = ctypes.c_uint64
            f.argtypes = [vp]
        lib.orc_sym_triangles_by_first.restype = ctypes.c_uint64
        lib.orc_sym_triangles_by_first.argtypes = [vp, ctypes.c_int, _u64p]
        lib.orc_sym_lollipop.restype = ctypes.c_uint64
        lib.orc_sym_lollipop.argtypes = [vp, ctypes.c_int]
        lib.orc_pair_intersections.restype = ctypes.c_uint64
        lib.orc_pair_intersections.argtypes = [ctypes.c_uint32, _u64p, _u32p, ctypes.c_uint64,
                                               _u32p, ctypes.c_int, _u64p]
        _lib = lib
        return lib


def _p32(a):
    return a.ctypes.data_as(_u32p)


def _p64(a):
    return None if a is None else a.ctypes.data_as(_u64p)


def max_threads() -> int:
    return int(_load().orc_max_threads())


class Graph:
    """The cleaned, ranked and oriented graph the oracle counts on."""

    def __init__(self, n: int, src, dst, order: str | None = None):
        lib = _load()
        self._lib = lib
        src = np.ascontiguousarray(src, dtype=np.uint32)
        dst = np.ascontiguousarray(dst, dtype=np.uint32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        err = ctypes.c_int(0)
        self._h = lib.orc_graph_new(int(n), int(src.size), _p32(src), _p32(dst), ctypes.byref(err))
        if not self._h:
            raise ValueError("vertex id out of range" if err.value == 1 else "oracle out of memory")
        self.n = int(n)
        self.m = int(lib.orc_num_edges(self._h))
        if order is not None and order != "degree":
            from oracle.orderings import ranks
            self.rerank(ranks(self, order))

    def rerank(self, rank) -> None:
        """Ranks vertices by rank[id] (a permutation) instead of (degree, id)."""
        rank = np.ascontiguousarray(rank, dtype=np.uint32)
        if rank.shape != (self.n,):
            raise ValueError("rank needs one entry per vertex")
        st = self._lib.orc_graph_rerank(self._h, _p32(rank))
        if st:
            raise ValueError("rank is not a permutation" if st == 1 else "oracle out of memory")

    @classmethod
    def from_edgelist(cls, el, order: str | None = None) -> "Graph":
        return cls(el.n, el.src, el.dst, order)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_graph_free(h)
            self._h = None

    # -- structure ---------------------------------------------------------
    def edges(self):
        a = np.empty(self.m, np.uint32)
        b = np.empty(self.m, np.uint32)
        self._lib.orc_get_edges(self._h, _p32(a), _p32(b))
        return a, b

    def rank(self):
        r = np.empty(self.n, np.uint32)
        self._lib.orc_get_rank(self._h, _p32(r))
        return r

    def degree(self):
        d = np.empty(self.n, np.uint32)
        self._lib.orc_get_degree(self._h, _p32(d))
        return d

    def oriented(self):
        """(off uint64[n+1], nbr uint32[m]) of the rank-space oriented CSR."""
        off = np.empty(self.n + 1, np.uint64)
        nbr = np.empty(self.m, np.uint32)
        self._lib.orc_get_oriented(self._h, _p64(off), _p32(nbr))
        return off, nbr

    # -- counts --------------------------------------------------------------
    def _run(self, fn, threads, rooted, per_vertex, x_begin, x_end, held=False):
        root = np.zeros(self.n, np.uint64) if rooted else None
        cv = np.zeros(self.n, np.uint64) if per_vertex else None
        b = ctypes.c_uint64(0)
        e = ctypes.c_uint64(0)
        h = (ctypes.c_uint64 * 2)()
        xe = self.n if x_end is None else int(x_end)
        extra = (h,) if held else ()
        total = fn(self._h, int(x_begin), xe, int(threads), _p64(root), _p64(cv), ctypes.byref(b),
                   ctypes.byref(e), *extra)
        out = {"count": int(total), "root": root, "per_vertex": cv, "bytes": int(b.value),
               "edges": int(e.value)}
        if held:
            out["held_bytes"] = int(h[0])
            out["held_tests"] = int(h[1])
        return out

    def triangles(self, threads: int = 0, rooted: bool = False, per_vertex: bool = False,
                  x_begin: int = 0, x_end: int | None = None) -> dict:
        """T; optional per-root (by original id) and per-vertex containment counts.

        ``bytes`` is B_merge over the visited oriented edges, ``edges`` their number.
        """
        return self._run(self._lib.orc_triangles_range, threads, rooted, per_vertex, x_begin, x_end)

    def cliques4(self, threads: int = 0, rooted: bool = False, per_vertex: bool = False,
                 x_begin: int = 0, x_end: int | None = None) -> dict:
        """K; ``bytes`` is B_K4 over the visited oriented edges, ``held_bytes``
        B_K4_held (the reads when N+(x) and S_xy are held on chip) and
        ``held_tests`` its element tests (the streamed members)."""
        return self._run(self._lib.orc_4cliques_range, threads, rooted, per_vertex, x_begin, x_end,
                         held=True)

    def cliques4_rooted_at(self, ids, threads: int = 0) -> np.ndarray:
        """Per original id, the 4-cliques rooted there (vertex of smallest rank),
        computed only for the ids listed (repeats ignored); 0 elsewhere."""
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        root = np.zeros(self.n, np.uint64)
        tot = self._lib.orc_4cliques_rooted_at(self._h, _p32(ids), ids.size, int(threads), _p64(root))
        if tot == 2**64 - 1:
            raise ValueError("id out of range, or oracle out of memory")
        return root

    def target_reads(self) -> dict:
        """B_target: the reads of the triangle sum with N+(y) of the middle
        attribute held and only the part of N+(x) above y streamed per in-edge
        x -> y.  Returns the bytes and their four parts."""
        out = np.zeros(4, np.uint64)
        b = int(self._lib.orc_target_reads(self._h, _p64(out)))
        if b == 2**64 - 1:
            raise MemoryError("oracle out of memory")
        return {"bytes": b, "held_sets": int(out[0]), "held_members": int(out[1]),
                "parts": int(out[2]), "streamed": int(out[3])}

    def count(self, pattern: int, threads: int = 0) -> int:
        if pattern == 3:
            return self.triangles(threads)["count"]
        if pattern == 4:
            return self.cliques4(threads)["count"]
        raise ValueError("pattern must be 3 or 4")

    # -- cross-checks without orientation -------------------------------------
    def sym_triangle_sum(self) -> int:
        return int(self._lib.orc_sym_triangle_sum(self._h))

    def sym_4clique_sum(self) -> int:
        return int(self._lib.orc_sym_4clique_sum(self._h))

    def sym_ordered_triangles(self) -> int:
        return int(self._lib.orc_sym_ordered_triangles(self._h))

    def sym_ordered_4cliques(self) -> int:
        return int(self._lib.orc_sym_ordered_4cliques(self._h))

    # -- the unpruned relation (appendix A, pruning symmetric queries) ----------
    def sym_triangles_by_first(self, threads: int = 0):
        """(6T, t) with t[x] the ordered triangles (x, y, z), by original id."""
        t = np.zeros(self.n, np.uint64)
        total = int(self._lib.orc_sym_triangles_by_first(self._h, int(threads), _p64(t)))
        return total, t

    def sym_lollipop(self, threads: int = 0) -> int:
        """COUNT(*) of Lollipop(x,y,z,w) :- R(x,y),S(y,z),T(x,z),U(x,w), unpruned."""
        return int(self._lib.orc_sym_lollipop(self._h, int(threads)))


def pair_intersections(off, members, pairs, threads: int = 0):
    """|A & B| per pair (section 4.2; layout-independent, section 4.3): set i is
    members[off[i]:off[i+1]], sorted without repeats; pairs is [n, 2] of set
    indices.  Returns (total, per-pair uint64 counts)."""
    off = np.ascontiguousarray(off, dtype=np.uint64)
    members = np.ascontiguousarray(members, dtype=np.uint32)
    pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros(pairs.shape[0], np.uint64)
    tot = _load().orc_pair_intersections(off.size - 1, _p64(off), _p32(members), pairs.shape[0],
                                         _p32(pairs), int(threads), _p64(out))
    if tot == 2**64 - 1:
        raise ValueError("a pair names a set index out of range")
    return int(tot), out


def batch_triangles(n_vertices, edge_off, src, dst, threads: int = 0):
    """Per-graph T of many independent graphs, graphs counted in parallel:
    graph i has n_vertices[i] vertices and the raw pairs src/dst[edge_off[i]:
    edge_off[i+1]] with local ids.  Returns (counts, b_merge, b_target), each
    uint64 per graph."""
    nv = np.ascontiguousarray(n_vertices, dtype=np.uint32)
    off = np.ascontiguousarray(edge_off, dtype=np.uint64)
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    if off.size != nv.size + 1 or src.shape != dst.shape or int(off[-1]) > src.size:
        raise ValueError("batch arrays do not agree")
    counts = np.zeros(nv.size, np.uint64)
    bm = np.zeros(nv.size, np.uint64)
    bt = np.zeros(nv.size, np.uint64)
    st = _load().orc_batch_triangles(nv.size, _p32(nv), _p64(off), _p32(src), _p32(dst),
                                     int(threads), _p64(counts), _p64(bm), _p64(bt))
    if st == 1:
        raise ValueError("vertex id out of range")
    if st == 2:
        raise MemoryError("oracle out of memory")
    return counts, bm, bt


def rooted_count(root_by_id: np.ndarray, roots) -> int:
    """Instances whose root lies in the set of `roots` (duplicates ignored)."""
    r = np.unique(np.asarray(roots, dtype=np.int64))
    return int(root_by_id[r].sum(dtype=np.uint64))
