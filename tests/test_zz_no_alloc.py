"""The allocation-free counting entry point (eh_count_add_noalloc) against
eh_count_add_async: identical counts on two calls in a row, the second on a
smaller input, under the schedules that use work cursors and the static ones,
for triangles and 4-cliques on pruned tries and the half count of a symmetric
trie; and both equal the CPU oracle's counts."""
import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import inputs

pytestmark = pytest.mark.gpu


def _u64(t):
    return int(t.cpu().numpy().view(np.uint64)[0])


@pytest.mark.parametrize("dynamic", [0, 1, 4])
@pytest.mark.parametrize("symmetric", [False, True])
def test_noalloc_equals_async(eh, dynamic, symmetric):
    import torch
    ctx = eh.Context(0)
    try:
        ctx.set_tuning(kernel=1, staging=2, dynamic=dynamic, grab=4, chunk_work=2048)
        big = inputs.rmat(12, 16, seed=81)
        small = inputs.rmat(9, 8, seed=82)
        for el in (big, small):  # the second call has the smaller input
            g = oracle.Graph.from_edgelist(el)
            want = {3: g.triangles()["count"], 4: g.cliques4()["count"]}
            if symmetric:
                want = {3: 6 * want[3], 4: 24 * want[4]}
            trie = ctx.build_edgelist(el, symmetric=symmetric)
            try:
                for pattern in (3, 4):
                    ref = torch.zeros(1, dtype=torch.int64, device="cuda")
                    got = torch.zeros(1, dtype=torch.int64, device="cuda")
                    ctx.stream.wait_stream(torch.cuda.current_stream())
                    ctx.count_add_async(trie, pattern, ref)   # also caches the plan
                    for _ in range(2):
                        ctx.count_add_noalloc(trie, pattern, got)
                    torch.cuda.synchronize()
                    assert _u64(ref) == want[pattern], (el.name, pattern)
                    assert _u64(got) == 2 * want[pattern], (el.name, pattern)
            finally:
                trie.free()
    finally:
        ctx.close()


def test_noalloc_needs_cached_plan(eh):
    import torch
    ctx = eh.Context(0)
    try:
        el = inputs.rmat(10, 16, seed=83)
        trie = ctx.build_edgelist(el)
        try:
            out = torch.zeros(1, dtype=torch.int64, device="cuda")
            with pytest.raises(eh.EHError) as e:
                ctx.count_add_noalloc(trie, 3, out)
            assert e.value.status == eh.EH_ESTATE
            ctx.count_triangles(trie)
            ctx.count_add_noalloc(trie, 3, out)
            torch.cuda.synchronize()
            assert _u64(out) == oracle.Graph.from_edgelist(el).triangles()["count"]
            with pytest.raises(eh.EHError) as e:
                ctx.count_add_noalloc(trie, 5, out)
            assert e.value.status == eh.EH_EINVAL
        finally:
            trie.free()
    finally:
        ctx.close()
