"""Allocator failure injection: a caller's allocator that refuses its k-th
request, for every k a build or workspace makes, must make the call return
OUT_OF_MEMORY with every earlier allocation handed back (no leak), and a
later call with a working allocator must succeed."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import lib, torch_cuda

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """dsbfs_allocator over PyTorch's caching allocator that counts live
    allocations and returns NULL on request number `fail_at` (0-based)."""

    def __init__(self, fail_at=None):
        d = lib()
        torch = torch_cuda()
        self.fail_at = fail_at
        self.requests = 0
        self.live = {}

        def _alloc(ctx, nbytes, stream):
            k = self.requests
            self.requests += 1
            if self.fail_at is not None and k == self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                   stream or 0)
            self.live[p] = nbytes
            return p

        def _free(ctx, ptr, stream):
            if ptr:
                self.live.pop(ptr)
                torch.cuda.caching_allocator_delete(ptr)

        self._a = d.ALLOC_FN(_alloc)
        self._f = d.FREE_FN(_free)
        self.struct = d.dsbfs_allocator(None, self._a, self._f)


def test_graph_and_workspace_survive_every_allocation_failure(inputs_mod, oracle_mod):
    d = lib()
    torch = torch_cuda()
    n = 1 << 10
    src, dst = inputs_mod.rmat_edges(10)
    # how many requests a build and a workspace make
    probe = CountingAllocator()
    g = d.Graph(src, dst, n, threshold=8, allocator=probe)
    build_requests = probe.requests
    ws = d.Workspace(g)
    ws_requests = probe.requests - build_requests
    ws.destroy()
    g.destroy()
    assert not probe.live and build_requests > 10 and ws_requests > 5
    for k in range(build_requests):
        a = CountingAllocator(fail_at=k)
        with pytest.raises(d.DsbfsError) as e:
            d.Graph(src, dst, n, threshold=8, allocator=a)
        assert e.value.status == d.ERR_OUT_OF_MEMORY, k
        assert not a.live, f"build leaked {len(a.live)} allocations after failing request {k}"
    for k in range(ws_requests):
        a = CountingAllocator(fail_at=build_requests + k)
        g = d.Graph(src, dst, n, threshold=8, allocator=a)
        with pytest.raises(d.DsbfsError) as e:
            d.Workspace(g)
        assert e.value.status == d.ERR_OUT_OF_MEMORY, k
        g.destroy()
        assert not a.live, f"workspace leaked after failing request {k}"
    # and everything still works afterwards
    a = CountingAllocator()
    g = d.Graph(src, dst, n, threshold=8, allocator=a)
    ws = d.Workspace(g)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    O = oracle_mod.Graph(src, dst, n)
    s = int(inputs_mod.pick_sources(src, dst, n, 1, seed=3)[0])
    d.bfs(g, ws, s, depth, None, opts=d.run_opts(want_parent=False))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(depth.cpu().numpy(), O.bfs(s, want_parent=False)[0])
    ws.destroy()
    g.destroy()
    assert not a.live
