"""Shared plumbing of the GPU tests: run the HIP path through the C-ABI binding
and bring results back to the host. Expected values always come from the
oracle or from closed forms, never from here."""
import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test started without a visible GPU")
    return torch


def lib():
    from paper_1803_03922_amd import dsbfs
    return dsbfs


# pytest's capture manager, set by conftest.py: log() suspends capture so that
# a long test's progress lines appear while it runs, also under -q
CAPTURE_MANAGER = None


def log(*a):
    cm = CAPTURE_MANAGER
    if cm is not None:
        with cm.global_and_fixture_disabled():
            print(*a, flush=True)
            sys.stdout.flush()
    else:
        print(*a, flush=True)
        sys.stdout.flush()


class GpuGraph:
    """A graph on the GPU plus a workspace and output buffers."""

    def __init__(self, src, dst, n, threshold=32, keep_plain=True, lanes=0, nn_copy=True):
        torch = torch_cuda()
        d = lib()
        self.torch = torch
        self.n = n
        self.g = d.Graph(src, dst, n, threshold=threshold, keep_plain_csr=keep_plain,
                         nn_copy=nn_copy)
        self.ws = d.Workspace(self.g, max_lanes=lanes)
        self.depth = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        self.parent = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")

    @property
    def stats(self):
        return self.g.stats

    def bfs(self, s, mode=1, forced=0, seed=0, want_parent=True, want_stats=False,
            factor0=None, factor1=None, profile=False, nn_do=False, factor_nn=None):
        d = lib()
        o = d.run_opts(mode=mode, want_parent=want_parent, forced=forced, forced_seed=seed,
                       factor0=factor0, factor1=factor1, profile=profile, nn_do=nn_do,
                       factor_nn=factor_nn)
        st = d.bfs(self.g, self.ws, s, self.depth, self.parent if want_parent else None, opts=o,
                   want_stats=want_stats)
        self.torch.cuda.synchronize()
        depth = self.depth[:self.n].cpu().numpy()
        parent = self.parent[:self.n].cpu().numpy() if want_parent else None
        return depth, parent, st

    def close(self):
        self.ws.destroy()
        self.g.destroy()
