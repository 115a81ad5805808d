"""Pins for the oracle's pairwise set intersection (section 4.2; its result
does not depend on the layout of section 4.3) against facts it does not
compute itself: brute force over Python sets, closed forms for arithmetic
progressions, numpy's intersect1d, and the triangle count by brute force.
Also the seeded dense-region set generator's recipe."""
import math

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import inputs


def _csr(sets):
    off = np.zeros(len(sets) + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in sets])
    members = np.concatenate([np.asarray(sorted(s), np.uint32) for s in sets]) if sets else \
        np.empty(0, np.uint32)
    return off, members.astype(np.uint32)


def _random_sets(seed, n_sets, max_size, domain):
    rng = np.random.default_rng(seed)
    sets = []
    for _ in range(n_sets):
        k = int(rng.integers(0, max_size + 1))
        sets.append(set(rng.choice(domain, size=min(k, domain), replace=False).tolist()))
    return sets


def test_oracle_brute_force_small():
    sets = _random_sets(1, 40, 30, 80) + [set(), set(range(80)), {0}, {79}]
    off, members = _csr(sets)
    rng = np.random.default_rng(2)
    pairs = rng.integers(0, len(sets), size=(600, 2)).astype(np.uint32)
    pairs = np.concatenate([pairs, [[40, 41], [41, 41], [42, 41], [43, 43], [5, 5]]]).astype(np.uint32)
    tot, per = oracle.pair_intersections(off, members, pairs)
    expect = [len(sets[a] & sets[b]) for a, b in pairs.tolist()]
    assert per.tolist() == expect and tot == sum(expect)


@pytest.mark.parametrize("a,b,n", [(2, 3, 1000), (4, 6, 4097), (7, 7, 300), (1, 5, 10 ** 5),
                                   (256, 96, 1 << 20), (33, 1, 1)])
def test_oracle_arithmetic_progressions(a, b, n):
    """Multiples of a and of b below n meet in the multiples of lcm(a, b)."""
    A = np.arange(0, n, a, dtype=np.uint32)
    B = np.arange(0, n, b, dtype=np.uint32)
    off = np.array([0, A.size, A.size + B.size], np.uint64)
    tot, per = oracle.pair_intersections(off, np.concatenate([A, B]), [[0, 1], [1, 0]])
    lcm = a * b // math.gcd(a, b)
    assert per.tolist() == [(n - 1) // lcm + 1] * 2 and tot == 2 * ((n - 1) // lcm + 1)


def test_oracle_matches_numpy_on_dense_regions():
    sp = inputs.dense_region_sets(24, 1500, 0.6, domain=1 << 18, seed=3)
    _, per = oracle.pair_intersections(sp.off, sp.members, sp.pairs)
    for p, (a, b) in enumerate(sp.pairs.tolist()):
        A = sp.members[sp.off[a]:sp.off[a + 1]]
        B = sp.members[sp.off[b]:sp.off[b + 1]]
        assert per[p] == np.intersect1d(A, B, assume_unique=True).size


def test_oracle_triangles_as_pair_intersections():
    """Summed over oriented edges (u, v), |N+(u) & N+(v)| is the triangle count
    (section 3.3), which brute force over vertex triples fixes."""
    el = inputs.gnp(40, 0.3, seed=4)
    g = oracle.Graph.from_edgelist(el)
    off, nbr = g.oriented()
    rows = np.repeat(np.arange(g.n), np.diff(off.astype(np.int64)))
    tot, _ = oracle.pair_intersections(off, nbr, np.stack([rows, nbr], axis=1))
    adj = set()
    for x, y in zip(el.src.tolist(), el.dst.tolist()):
        if x != y:
            adj.add((x, y))
            adj.add((y, x))
    brute = sum(1 for x in range(40) for y in range(x + 1, 40) for z in range(y + 1, 40)
                if (x, y) in adj and (y, z) in adj and (x, z) in adj)
    assert tot == brute


def test_oracle_rejects_out_of_range_pairs():
    off, members = _csr([{1, 2}, {2}])
    with pytest.raises(ValueError):
        oracle.pair_intersections(off, members, [[0, 2]])


def test_generator_recipe():
    sp = inputs.dense_region_sets(6, 512, 0.5, domain=1 << 16, density=0.5, seed=9)
    assert sp.n_sets == 12 and sp.members.size == 12 * 512
    for j in range(sp.n_sets):
        m = sp.members[sp.off[j]:sp.off[j + 1]].astype(np.int64)
        assert np.all(np.diff(m) > 0) and m[-1] < 1 << 16
    # the two sets of a pair share the dense region of 512 ids holding 256 of each
    a = sp.members[0:512].astype(np.int64)
    b = sp.members[512:1024].astype(np.int64)
    lo = max(a[np.argmax(np.diff(a) <= 2)], b[np.argmax(np.diff(b) <= 2)]) - 2
    assert np.sum((a >= lo) & (a < lo + 520)) >= 250 and np.sum((b >= lo) & (b < lo + 520)) >= 250
    again = inputs.dense_region_sets(6, 512, 0.5, domain=1 << 16, density=0.5, seed=9)
    assert np.array_equal(again.members, sp.members)


# ---- properties over generated sets (hypothesis) ---------------------------------

from hypothesis import given, settings, strategies as hs

_sets = hs.lists(hs.sets(hs.integers(0, 2 ** 32 - 1), max_size=60), min_size=1, max_size=8)


@settings(max_examples=150, deadline=None)
@given(_sets, hs.data())
def test_oracle_inclusion_exclusion(sets, data):
    """|A & B| = |A| + |B| - |A | B|, with the union from numpy; the count is
    symmetric and |A & A| = |A|."""
    off, members = _csr(sets)
    k = len(sets)
    pairs = data.draw(hs.lists(hs.tuples(hs.integers(0, k - 1), hs.integers(0, k - 1)),
                               min_size=1, max_size=20))
    both = [(a, b) for a, b in pairs] + [(b, a) for a, b in pairs] + [(a, a) for a in range(k)]
    tot, per = oracle.pair_intersections(off, members, np.array(both, np.uint32))
    for (a, b), c in zip(both, per.tolist()):
        A = np.asarray(sorted(sets[a]), np.uint32)
        B = np.asarray(sorted(sets[b]), np.uint32)
        assert c == A.size + B.size - np.union1d(A, B).size
    assert tot == int(per.sum())
