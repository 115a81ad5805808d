"""Set stores (section 4.3 layouts at relation, set and block level) without a
GPU: the library's host encoding decoded back to its input and checked
against each layout's rule."""
import numpy as np
import pytest

from paper_1503_02368_amd import eh, inputs

LAYOUTS = {"uint": eh.SETS_UINT, "set": eh.SETS_SET, "bitset": eh.SETS_BITSET,
           "composite": eh.SETS_COMPOSITE}


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


# ---- host encoding ------------------------------------------------------------

def _decode(h, n_sets):
    """The members of each set, read back from segments, members and words."""
    bl = h["block_log"]
    wpb = 1 << (bl - 5)
    out = []
    for i in range(n_sets):
        got = []
        for s in range(h["seg_off"][i], h["seg_off"][i + 1]):
            b0, b1, start, w = (int(x) for x in h["seg"][s])
            if w & 0x80000000:
                words = h["words"][start:start + (b1 - b0 + 1) * wpb]
                bits = np.unpackbits(words.view(np.uint8), bitorder="little")
                ids = np.nonzero(bits)[0] + (b0 << bl)
                assert ids.size == w & 0x7FFFFFFF
                got.append(ids)
            else:
                vals = h["vals"][start:start + w].astype(np.int64)
                assert vals.size == 0 or (vals[0] >> bl == b0 and vals[-1] >> bl == b1)
                got.append(vals)
        out.append(np.concatenate(got).astype(np.int64) if got else np.empty(0, np.int64))
    return out


def _check_rules(h, sets, layout, bl, block_min, tau=32.0):
    seg = h["seg"].astype(np.int64)
    for i, s in enumerate(sets):
        segs = seg[h["seg_off"][i]:h["seg_off"][i + 1]]
        m = np.asarray(sorted(s), np.int64)
        if m.size == 0:
            assert segs.shape[0] == 0
            continue
        assert np.all(segs[1:, 0] > segs[:-1, 1])  # ascending, disjoint in blocks
        kind = (segs[:, 3] & 0x80000000) != 0
        if layout == "uint":
            assert segs.shape[0] == 1 and not kind[0]
        elif layout == "set":
            dense = (m[-1] - m[0] + 1) <= tau * m.size
            assert segs.shape[0] == 1 and kind[0] == dense
            assert segs[0, 0] == m[0] >> bl and segs[0, 1] == m[-1] >> bl
        else:
            blocks, counts = np.unique(m >> bl, return_counts=True)
            dense_blocks = set(blocks.tolist()) if layout == "bitset" else \
                set(blocks[counts >= block_min].tolist())
            stored = set()
            for (b0, b1, _, _), k in zip(segs.tolist(), kind.tolist()):
                if k:
                    stored |= set(range(b0, b1 + 1))
            assert stored == dense_blocks
            # maximal runs: neighbours differ in kind, or are bitset runs with a gap
            for t in range(1, segs.shape[0]):
                if kind[t] == kind[t - 1]:
                    assert kind[t] and segs[t, 0] > segs[t - 1, 1] + 1


CASES = [
    ("random", lambda: _random_sets(5, 60, 300, 5000)),
    ("dense_region", lambda: [set(x.tolist()) for x in np.split(
        inputs.dense_region_sets(8, 700, 0.5, domain=1 << 17, seed=2).members, 16)]),
    ("edges", lambda: [set(), {0}, {2 ** 32 - 1}, set(range(256)), set(range(255, 513)),
                       {2 ** 32 - 2, 2 ** 32 - 1, 0, 1}, set(range(2 ** 32 - 300, 2 ** 32)),
                       set(range(0, 4096, 2)), set(range(0, 1 << 16, 97))]),
]


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("bl", [5, 8, 12])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_host_encoding_decodes_and_follows_rules(layout, bl, case):
    sets = case[1]()
    off, members = _csr(sets)
    block_min = 3
    h = eh.host_sets(off, members, layout=LAYOUTS[layout], block_log=bl, block_min=block_min)
    assert h["n_sets"] == len(sets) and h["n_members"] == members.size
    assert h["n_segments"] == h["seg"].shape[0]
    assert h["uint_members"] + sum(int(w) & 0x7FFFFFFF for w in h["seg"][:, 3]
                                   if int(w) & 0x80000000) == members.size
    for got, s in zip(_decode(h, len(sets)), sets):
        assert got.tolist() == sorted(s)
    _check_rules(h, sets, layout, bl, block_min)


def test_default_block_min_and_sizes():
    sets = [set(range(0, 256, 32)), set(range(0, 256, 37)), set(range(1000, 1256))]
    off, members = _csr(sets)
    h = eh.host_sets(off, members, layout=eh.SETS_COMPOSITE)  # 256-id blocks, dense at 8
    kinds = [bool(int(w) & 0x80000000) for w in h["seg"][:, 3]]
    assert kinds == [True, False, True]
    # 8 members in block 0; 7 in block 0; 24 + 232 in blocks 3 and 4 (one run)
    assert h["bitset_blocks"] == 3 and h["bitset_words"] == 3 * 8
    assert h["n_segments"] == 3 and h["uint_members"] == 7


def test_host_encoding_rejects_bad_input():
    good_off, good = _csr([{1, 5}, {2}])
    with pytest.raises(eh.EHError):
        eh.host_sets(good_off, np.array([5, 1, 2], np.uint32))          # not ascending
    with pytest.raises(eh.EHError):
        eh.host_sets(good_off, np.array([1, 1, 2], np.uint32))          # repeat
    with pytest.raises(eh.EHError):
        eh.host_sets(good_off, good, layout=4)
    for bl in (4, 17):
        with pytest.raises(eh.EHError):
            eh.host_sets(good_off, good, block_log=bl)
    with pytest.raises(eh.EHError):
        eh.host_sets(np.array([1, 2, 3], np.uint64), good)              # off[0] != 0
    with pytest.raises(eh.EHError):
        eh.host_sets(np.array([0, 2, 1, 3], np.uint64), good)          # decreasing
    h = eh.host_sets(np.zeros(1, np.uint64), np.empty(0, np.uint32))    # no sets
    assert h["n_sets"] == 0 and h["n_segments"] == 0


# ---- generated sets (hypothesis) ---------------------------------------------------

from hypothesis import given, settings, strategies as hs


@settings(max_examples=120, deadline=None)
@given(hs.lists(hs.one_of(hs.sets(hs.integers(0, 2 ** 32 - 1), max_size=40),
                          hs.builds(lambda lo, n, step: set(range(lo, lo + n * step, step)),
                                    hs.integers(0, 2 ** 20), hs.integers(0, 600),
                                    hs.integers(1, 4))),
                min_size=0, max_size=6),
       hs.sampled_from(list(LAYOUTS)), hs.integers(5, 16), hs.integers(0, 40))
def test_host_encoding_generated(sets, layout, bl, block_min):
    """Any sets, layout, block size and density threshold: the encoding decodes
    to its input and follows the layout's rule."""
    off, members = _csr(sets)
    h = eh.host_sets(off, members, layout=LAYOUTS[layout], block_log=bl, block_min=block_min)
    for got, s in zip(_decode(h, len(sets)), sets):
        assert got.tolist() == sorted(s)
    _check_rules(h, sets, layout, bl, block_min if block_min else (1 << bl) // 32)
