"""Allocation failures forced from the host: an allocator that fails on its
k-th call, for every k a build-and-count sequence reaches.  Each call either
succeeds with the oracle's counts or returns EH_ENOMEM; afterwards no device
memory is left allocated beyond what the context holds, nothing is freed
twice, and the context keeps working.  No kernel is made to fail: a refused
allocation ends the call before anything is launched on the missing buffer."""
import sys

import numpy as np
import pytest

import oracle
from paper_1503_02368_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class FailingAllocator:
    """torch's caching allocator, refusing every call from the fail_at-th on."""

    def __init__(self, torch, device=0):
        self.torch = torch
        self.device = device
        self.fail_at = None
        self.calls = 0
        self.refused = 0
        self.live = {}
        self.bad_frees = 0

    def arm(self, k):
        self.calls = 0
        self.refused = 0
        self.fail_at = k

    def disarm(self):
        self.fail_at = None

    def alloc(self, nbytes, stream):
        self.calls += 1
        if self.fail_at is not None and self.calls >= self.fail_at:
            self.refused += 1
            return None
        p = self.torch.cuda.caching_allocator_alloc(nbytes, self.device, stream)
        self.live[p] = nbytes
        return p

    def free(self, ptr, stream):
        if ptr not in self.live:
            self.bad_frees += 1
            return
        del self.live[ptr]
        self.torch.cuda.caching_allocator_delete(ptr)


EL = inputs.rmat(10, 8, seed=3)


@pytest.fixture(scope="module")
def truth():
    g = oracle.Graph.from_edgelist(EL)
    return g.count(3), g.count(4)


def _host_build_and_count(eh, ctx, torch):
    trie = ctx.build_edgelist(EL)
    try:
        return ctx.count_triangles(trie), ctx.count_4cliques(trie)
    finally:
        trie.free()


def _device_build_and_count(eh, ctx, torch):
    src = torch.from_numpy(np.ascontiguousarray(EL.src).view(np.int32)).cuda()
    dst = torch.from_numpy(np.ascontiguousarray(EL.dst).view(np.int32)).cuda()
    ctx.stream.wait_stream(torch.cuda.current_stream())
    trie = ctx.build_trie_device(EL.n, src, dst)
    try:
        return ctx.count_triangles(trie), ctx.count_4cliques(trie)
    finally:
        trie.free()


@pytest.mark.parametrize("how", ["host", "device"])
def test_every_allocation_failure_is_clean(eh, truth, how):
    import torch
    fa = FailingAllocator(torch)
    ctx = eh.Context(0, allocator=fa)
    run = _host_build_and_count if how == "host" else _device_build_and_count
    try:
        ctx.stream.synchronize()
        baseline = dict(fa.live)
        refused_calls = 0
        for k in range(1, 200):
            fa.arm(k)
            say(f"[faults] {how} build, allocation {k} refused")
            try:
                got = run(eh, ctx, torch)
                failed = False
            except eh.EHError as e:
                assert e.status == eh.EH_ENOMEM, (k, e)
                failed = True
            fa.disarm()
            ctx.stream.synchronize()
            assert fa.bad_frees == 0, k
            assert fa.live == baseline, (k, len(fa.live), len(baseline))
            if failed:
                refused_calls += 1
            else:
                assert got == truth
                if fa.refused == 0:
                    break  # the sequence makes fewer than k allocations
        assert refused_calls >= 5
        # the context still builds and counts
        assert run(eh, ctx, torch) == truth
        assert fa.live == baseline
    finally:
        ctx.close()
    assert fa.bad_frees == 0


def test_set_store_allocation_failures(eh):
    import torch
    fa = FailingAllocator(torch)
    ctx = eh.Context(0, allocator=fa)
    sp = inputs.dense_region_sets(32, 500, 0.5, domain=1 << 16, seed=5)
    want, _ = oracle.pair_intersections(sp.off, sp.members, sp.pairs)
    d_pairs = torch.from_numpy(np.ascontiguousarray(sp.pairs).view(np.int32)).cuda()
    ctx.stream.wait_stream(torch.cuda.current_stream())
    try:
        ctx.stream.synchronize()
        baseline = dict(fa.live)
        for k in range(1, 10):
            fa.arm(k)
            try:
                st = ctx.build_sets(sp.off, sp.members)
            except eh.EHError as e:
                assert e.status == eh.EH_ENOMEM
                st = None
            fa.disarm()
            if st is not None:
                assert ctx.intersect_pairs(st, d_pairs) == want
                st.free()
            ctx.stream.synchronize()
            assert fa.bad_frees == 0 and fa.live == baseline, k
    finally:
        ctx.close()
