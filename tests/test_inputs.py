"""Seeded generators: reproducible, in range, with the requested shapes."""
import hashlib
import math

import numpy as np

from paper_1503_02368_amd import inputs


def digest(el):
    return hashlib.sha256(el.src.tobytes() + el.dst.tobytes()).hexdigest()


def test_splitmix_reference_values():
    # splitmix64 seeded with 0 yields these first outputs (published test vector
    # of the generator's reference implementation)
    out = inputs.rand_u64(0, 0, 3)
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rmat_reproducible_and_in_range():
    a = inputs.rmat(10, 8, seed=3)
    b = inputs.rmat(10, 8, seed=3)
    c = inputs.rmat(10, 8, seed=4)
    assert digest(a) == digest(b) != digest(c)
    assert a.m_raw == 8 * 1024
    assert a.src.max() < 1024 and a.dst.max() < 1024
    # quadrant frequencies of the top level follow (a, b, c, d)
    top_s = a.src >> 9
    top_d = a.dst >> 9
    frac = np.array([np.mean((top_s == i) & (top_d == j)) for i in (0, 1) for j in (0, 1)])
    assert np.allclose(frac, [0.57, 0.19, 0.19, 0.05], atol=0.03)


def test_rmat_chunking_invariant():
    a = inputs.rmat(9, 4, seed=1, chunk=1 << 22)
    b = inputs.rmat(9, 4, seed=1, chunk=100)
    assert digest(a) == digest(b)


def test_er_gnm():
    el = inputs.erdos_renyi_gnm(4096, 32768, seed=1)
    assert el.m_raw == 32768
    assert np.all(el.src < el.dst) and el.dst.max() < 4096
    keys = el.src.astype(np.int64) * 4096 + el.dst
    assert np.unique(keys).size == 32768
    assert digest(el) == digest(inputs.erdos_renyi_gnm(4096, 32768, seed=1))


def test_pair_index_bijection():
    n = 37
    k = np.arange(n * (n - 1) // 2, dtype=np.int64)
    i, j = inputs._pair_from_index(k, n)
    ref = np.array([(a, b) for a in range(n) for b in range(a + 1, n)])
    assert np.array_equal(i, ref[:, 0]) and np.array_equal(j, ref[:, 1])


def test_chung_lu_and_batch():
    el = inputs.chung_lu(1000, 16.0, 2.1, seed=1, graph=2)
    assert el.m_raw == 8000 and el.src.max() < 1000
    # heavier weights on low ids
    assert np.mean(el.src < 100) > 0.3
    b = inputs.batch_chung_lu(12, seed=4)
    assert b.n_graphs == 12 and int(b.edge_off[-1]) == b.src.size
    n, d = inputs.batch_sizes(2000, seed=4)
    assert n.min() >= 64 and n.max() <= 16384
    assert d.min() >= 8 - 1e-9 and d.max() <= 64 + 1e-9
    # log-uniform: median near the geometric mean of the bounds
    assert abs(math.log(np.median(n)) - math.log(math.sqrt(64 * 16384))) < 0.3
    for g in range(12):
        sub = b.graph(g)
        assert sub.src.size == 0 or sub.src.max() < sub.n


def test_request_stream():
    reqs = inputs.request_stream(1 << 12, rate_qps=1000, duration_s=0.5, seed=5)
    assert 300 < len(reqs) < 700
    ts = [r.t_arrival for r in reqs]
    assert all(x < y for x, y in zip(ts, ts[1:]))
    for r in reqs:
        assert r.pattern in (3, 4)
        assert np.unique(r.roots).size == r.roots.size
        assert 1 <= r.roots.size <= 1 << 12
        assert r.roots.max() < 1 << 12
