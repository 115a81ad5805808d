"""Node orderings for the oracle -- TEST INFRASTRUCTURE ONLY.

Plain Python, written from the paper's appendix A ("node ordering") and the
dictionary encoding of section 2.2.  An ordering is the sequence in which
vertices receive their labels 0, 1, 2, ...; the paper prunes a symmetric
relation by keeping each edge from the larger label to the smaller.  The
oracle ranks vertex v as n - 1 - label(v) and directs edges from lower to
higher rank, which keeps exactly those edges and every set's gaps.

Readings where the appendix is silent (ties, traversal details):

* degree       degree descending, ties by id descending, so that the ranks
               are (degree ascending, id ascending), the default ranking;
* rev_degree   degree ascending, ties by id ascending;
* input        label = id;
* bfs          breadth-first discovery order; each traversal starts at the
               unvisited vertex of highest degree (ties: lowest id), and the
               neighbours of a vertex are discovered in ascending id order;
* hybrid       the BFS sequence, then a stable sort by degree descending;
* strong_runs  vertices visited by degree descending (ties id ascending); a
               visited vertex takes the next label if it has none, then its
               unlabelled neighbours take the next labels, ascending id.
"""
from __future__ import annotations

from collections import deque

import numpy as np

ORDERS = ("degree", "rev_degree", "input", "bfs", "hybrid", "strong_runs")


def _adjacency(g) -> list[list[int]]:
    """Neighbour lists of the oracle graph's simple undirected edges, ascending."""
    a, b = g.edges()
    adj: list[list[int]] = [[] for _ in range(g.n)]
    for x, y in zip(a.tolist(), b.tolist()):
        adj[x].append(y)
        adj[y].append(x)
    for row in adj:
        row.sort()
    return adj


def _bfs(n: int, adj, deg) -> list[int]:
    seq: list[int] = []
    seen = [False] * n
    for root in sorted(range(n), key=lambda v: (-deg[v], v)):
        if seen[root]:
            continue
        seen[root] = True
        queue = deque([root])
        while queue:
            v = queue.popleft()
            seq.append(v)
            for w in adj[v]:
                if not seen[w]:
                    seen[w] = True
                    queue.append(w)
    return seq


def _strong_runs(n: int, adj, deg) -> list[int]:
    seq: list[int] = []
    labelled = [False] * n
    for v in sorted(range(n), key=lambda v: (-deg[v], v)):
        if not labelled[v]:
            labelled[v] = True
            seq.append(v)
        for w in adj[v]:
            if not labelled[w]:
                labelled[w] = True
                seq.append(w)
    return seq


def sequence(g, order: str) -> list[int]:
    """The vertices of oracle graph g in the order they receive labels."""
    n = g.n
    deg = g.degree().tolist()
    if order == "degree":
        return sorted(range(n), key=lambda v: (-deg[v], -v))
    if order == "rev_degree":
        return sorted(range(n), key=lambda v: (deg[v], v))
    if order == "input":
        return list(range(n))
    if order in ("bfs", "hybrid"):
        seq = _bfs(n, _adjacency(g), deg)
        if order == "hybrid":
            seq = sorted(seq, key=lambda v: -deg[v])  # Python's sort is stable
        return seq
    if order == "strong_runs":
        return _strong_runs(n, _adjacency(g), deg)
    raise ValueError(f"unknown ordering {order!r}")


def ranks(g, order: str) -> np.ndarray:
    """rank[id] = n - 1 - label(id) under the ordering."""
    seq = sequence(g, order)
    r = np.empty(g.n, dtype=np.uint32)
    r[np.asarray(seq, dtype=np.int64)] = np.arange(g.n - 1, -1, -1, dtype=np.uint32)
    return r
