"""Host half of the library (no GPU): the ABI loads and exports every symbol
of include/eh.h, and the trie it builds is the oracle's graph, oriented and
laid out as the set optimizer specifies."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import eh, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "eh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eh_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = eh.load()
    decl = declared_symbols()
    assert len(decl) >= 20
    assert sorted(eh.SYMBOLS) == decl
    for name in decl:
        assert getattr(lib, name) is not None
        ctypes.cast(getattr(lib, name), ctypes.c_void_p)


def test_status_strings():
    lib = eh.load()
    assert lib.eh_status_str(0) == b"ok"
    assert lib.eh_status_str(-1) == b"invalid argument"
    assert lib.eh_abi_version() == eh.ABI_VERSION
    with open(os.path.join(ROOT, "include", "eh.h")) as f:
        assert int(re.search(r"#define EH_ABI_VERSION (\d+)", f.read()).group(1)) == eh.ABI_VERSION


GRAPHS = [inputs.rmat(10, 16, seed=3), inputs.messy(inputs.rmat(9, 8, seed=4), 2),
          inputs.erdos_renyi_gnm(512, 4000, seed=2), inputs.complete(40), inputs.grid(10, 12),
          inputs.wheel(20), inputs.chung_lu(3000, 24, 2.1, seed=1, graph=3)]


@pytest.mark.parametrize("el", GRAPHS, ids=lambda e: e.name)
def test_trie_matches_oracle(el):
    h = eh.host_trie(el.n, el.src, el.dst)
    g = oracle.Graph.from_edgelist(el)
    off, nbr = g.oriented()
    assert h["m_plus"] == g.m
    np.testing.assert_array_equal(h["rank"], g.rank())
    np.testing.assert_array_equal(h["row"], off.astype(np.uint32))
    np.testing.assert_array_equal(h["col"], nbr)
    assert h["b_merge"] == g.triangles()["bytes"]
    assert h["b_target"] == g.target_reads()["bytes"]
    d = np.diff(h["row"].astype(np.int64))
    assert h["max_out_degree"] == (d.max() if d.size else 0)


ORDER_GRAPHS = [inputs.rmat(10, 16, seed=3), inputs.messy(inputs.rmat(9, 8, seed=4), 2),
                inputs.chung_lu(3000, 24, 2.1, seed=1, graph=3),
                inputs.disjoint_union(inputs.wheel(9), inputs.star(5), inputs.path(4),
                                      inputs.complete(1), inputs.grid(4, 5))]


@pytest.mark.parametrize("order", sorted(eh.ORDERS))
@pytest.mark.parametrize("el", ORDER_GRAPHS, ids=lambda e: e.name)
def test_node_orderings_match_oracle(el, order):
    """Ranks (index work: bit-exact) and the oriented trie under each node
    ordering of appendix A equal the oracle's, computed by its own code."""
    h = eh.host_trie(el.n, el.src, el.dst, order=eh.ORDERS[order])
    g = oracle.Graph.from_edgelist(el, order)
    off, nbr = g.oriented()
    np.testing.assert_array_equal(h["rank"], g.rank())
    np.testing.assert_array_equal(h["row"], off.astype(np.uint32))
    np.testing.assert_array_equal(h["col"], nbr)
    assert h["b_merge"] == g.triangles()["bytes"]
    assert h["b_target"] == g.target_reads()["bytes"]
    d = np.diff(h["row"].astype(np.int64))
    assert h["max_out_degree"] == (d.max() if d.size else 0)


def test_symmetric_trie_has_no_target_model():
    el = inputs.rmat(9, 16, seed=5)
    assert eh.host_trie(el.n, el.src, el.dst, symmetric=True)["b_target"] == 0
    assert eh.host_trie(el.n, el.src, el.dst)["b_target"] > 0


def expand_bitset(h, r):
    w = h["bs_words"][h["bs_off"][r]: h["bs_off"][r] + h["bs_nw"][r]]
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return np.nonzero(bits)[0].astype(np.int64) + int(h["bs_base"][r])


@pytest.mark.parametrize("tau,s_min", [(2.0, 1), (32.0, 1), (256.0, 1), (32.0, 16), (1e9, 1)])
def test_density_rule_and_bitset_contents(tau, s_min):
    el = inputs.rmat(11, 16, seed=5)
    h = eh.host_trie(el.n, el.src, el.dst, layout=eh.LAYOUT_HYBRID, tau=tau, s_min=s_min)
    row, col = h["row"].astype(np.int64), h["col"].astype(np.int64)
    n_bs = 0
    for r in range(h["n"]):
        seg = col[row[r]:row[r + 1]]
        has = h["bs_off"][r] != 0xFFFFFFFF
        if seg.size == 0:
            assert not has
            continue
        rng = seg[-1] - seg[0] + 1
        want = seg.size >= s_min and rng <= tau * seg.size
        assert has == want
        if has:
            n_bs += 1
            assert h["bs_base"][r] % 32 == 0 and h["bs_base"][r] <= seg[0]
            np.testing.assert_array_equal(expand_bitset(h, r), seg)
    assert n_bs == h["n_bitset_sets"]


def test_layout_extremes():
    el = inputs.rmat(9, 16, seed=6)
    u = eh.host_trie(el.n, el.src, el.dst, layout=eh.LAYOUT_UINT)
    assert u["n_bitset_sets"] == 0 and u["bitset_words"] == 0
    b = eh.host_trie(el.n, el.src, el.dst, layout=eh.LAYOUT_BITSET_ALL)
    nonempty = int((np.diff(b["row"].astype(np.int64)) > 0).sum())
    assert b["n_bitset_sets"] == nonempty
    for r in range(b["n"]):
        if b["row"][r + 1] > b["row"][r]:
            np.testing.assert_array_equal(expand_bitset(b, r), b["col"][b["row"][r]:b["row"][r + 1]])


def test_invalid_and_empty():
    with pytest.raises(eh.EHError) as e:
        eh.host_trie(4, np.array([0, 1], np.uint32), np.array([1, 4], np.uint32))
    assert e.value.status == eh.EH_EINVAL
    with pytest.raises(eh.EHError) as e:
        eh.host_trie(4, np.array([0], np.uint32), np.array([1], np.uint32), order=6)
    assert e.value.status == eh.EH_EINVAL
    for order in eh.ORDERS.values():
        h = eh.host_trie(5, np.zeros(0, np.uint32), np.zeros(0, np.uint32), order=order)
        assert h["m_plus"] == 0 and h["n"] == 5
        assert sorted(h["rank"].tolist()) == list(range(5))
    h = eh.host_trie(7, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert h["m_plus"] == 0 and h["n"] == 7
    h = eh.host_trie(3, np.array([1, 2], np.uint32), np.array([1, 2], np.uint32))
    assert h["m_plus"] == 0
