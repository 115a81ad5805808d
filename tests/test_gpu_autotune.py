"""The autotuner (the brute-force "oracle optimizer" of section 4.4 applied to
this engine's knobs) in quick mode on small inputs: every candidate is
checked against the CPU oracle's count, the winner is rebuilt and checked
again, and the entry it writes reproduces the oracle's count when a caller
builds and counts with it, as the benchmark does."""
import json

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(eh):
    c = eh.Context(0)
    yield c
    c.close()


def test_tune_graph_entry_reproduces_oracle(ctx, eh, tmp_path):
    import torch
    from paper_1503_02368_amd import autotune
    from paper_1503_02368_amd.workloads import WORKLOADS
    el = inputs.rmat(11, 16, seed=61)
    T = oracle.Graph.from_edgelist(el).triangles()["count"]
    entry = autotune.tune_workload("small", WORKLOADS["rmat20_triangles"], ctx, torch, quick=True,
                                   expect=T, data=el)
    assert entry["count"] == T and entry["checked_against"] == "expected"
    assert {l[2] for l in autotune.layouts_for(WORKLOADS["rmat20_triangles"], True)} >= {1, 16}
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps({"small": entry}))
    e = json.loads(path.read_text())["small"]
    ctx.set_tuning(**e["tuning"])
    trie = ctx.build_edgelist(el, layout=e["layout"], tau=e["tau"], s_min=e["s_min"])
    try:
        assert ctx.count_triangles(trie) == T
    finally:
        trie.free()
    # a reference that no candidate can reach stops the search
    with pytest.raises(RuntimeError):
        autotune.tune_workload("small", WORKLOADS["rmat20_triangles"], ctx, torch, quick=True,
                               expect=T + 1, data=el)


def test_tune_4cliques_and_batch(ctx, eh):
    import torch
    from paper_1503_02368_amd import autotune
    from paper_1503_02368_amd.workloads import WORKLOADS
    el = inputs.rmat(10, 16, seed=62)
    K = oracle.Graph.from_edgelist(el).cliques4()["count"]
    entry = autotune.tune_workload("k4", WORKLOADS["rmat18_4cliques"], ctx, torch, quick=True,
                                   expect=K, data=el)
    assert entry["count"] == K
    b = inputs.batch_chung_lu(40, seed=63, n_hi=2048)
    want, _, _ = oracle.batch_triangles(b.n_vertices, b.edge_off, b.src, b.dst)
    entry = autotune.tune_workload("b", WORKLOADS["batch_triangles"], ctx, torch, quick=True,
                                   expect=want, data=b)
    assert entry["count"] == int(want.sum())
    ctx.set_tuning(**entry["tuning"])
    trie = ctx.build_batch(b, layout=entry["layout"], tau=entry["tau"], s_min=entry["s_min"])
    try:
        assert np.array_equal(np.asarray(ctx.count_batch(trie, eh.TRIANGLE), np.uint64), want)
    finally:
        trie.free()


def test_tune_served(ctx, eh):
    import torch
    from paper_1503_02368_amd import autotune
    from paper_1503_02368_amd.workloads import WORKLOADS
    w = WORKLOADS["served"]
    el = inputs.rmat(12, 16, seed=64)
    g = oracle.Graph.from_edgelist(el)
    rt = g.triangles(rooted=True)["root"]
    rk = g.cliques4(rooted=True)["root"]
    reqs = autotune.served_requests(w, el.n, quick=True)
    want = [oracle.rooted_count(rt if r.pattern == 3 else rk, r.roots) for r in reqs]
    entry = autotune.tune_workload("served_small", w, ctx, torch, quick=True, expect=want, data=el)
    assert entry["count"] == sum(want)
