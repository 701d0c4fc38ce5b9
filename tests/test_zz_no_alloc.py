"""The allocation-free single-source search (dsbfs_bfs_noalloc) against the
workspace search (dsbfs_bfs) through the C-ABI: two calls in a row, the second
on a smaller graph, in both modes; depths bit-exact against the workspace
search and the oracle, parents through the oracle's invariant checker."""
import numpy as np
import pytest

from gpu_helpers import lib, log, torch_cuda

pytestmark = pytest.mark.gpu


def _run_both(d, torch, G, O, s, mode):
    n = G.n
    dev = torch.device("cuda")
    a_d = torch.empty(n, dtype=torch.int32, device=dev)
    a_p = torch.empty(n, dtype=torch.int32, device=dev)
    b_d = torch.full((n,), 7, dtype=torch.int32, device=dev)
    b_p = torch.full((n,), 7, dtype=torch.int32, device=dev)
    ws = d.Workspace(G)
    o = d.run_opts(mode=mode, want_parent=True)
    st_ws = d.bfs(G, ws, s, a_d, a_p, opts=o, want_stats=True)
    d.bfs_noalloc(G, s, b_d, b_p, opts=o)
    torch.cuda.synchronize()
    ws.destroy()
    want, _ = O.bfs(s, want_parent=False)
    got_ws, got = a_d.cpu().numpy(), b_d.cpu().numpy()
    np.testing.assert_array_equal(got, got_ws, err_msg=f"noalloc vs workspace, s={s} mode={mode}")
    np.testing.assert_array_equal(got, want, err_msg=f"noalloc vs oracle, s={s} mode={mode}")
    code, bad = O.check(s, got, b_p.cpu().numpy())
    assert code == 0, f"parent invariant {code} fails at {bad}, s={s} mode={mode}"
    return st_ws


def test_noalloc_matches_workspace_search_two_calls(inputs_mod, oracle_mod):
    d = lib()
    torch = torch_cuda()
    for scale, TH, k in ((16, 32, 6), (12, 8, 6)):   # second call: a smaller graph
        n = 1 << scale
        src, dst = inputs_mod.rmat_edges(scale)
        G = d.Graph(src, dst, n, threshold=TH, keep_plain_csr=True)
        O = oracle_mod.Graph(src, dst, n)
        for s in inputs_mod.pick_sources(src, dst, n, k, seed=300 + scale).tolist():
            for mode in (1, 0):
                log(f"noalloc scale={scale} TH={TH} s={s} mode={mode}")
                _run_both(d, torch, G, O, s, mode)
        G.destroy()


def test_noalloc_stats_and_errors(inputs_mod, oracle_mod):
    d = lib()
    torch = torch_cuda()
    scale = 14
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    G = d.Graph(src, dst, n, threshold=16, keep_plain_csr=False)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(d.DsbfsError) as e:
        d.bfs_noalloc(G, n, depth, None, opts=d.run_opts(want_parent=False))
    assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        d.bfs_noalloc(G, 0, depth, None, opts=d.run_opts(want_parent=False, profile=True))
    assert e.value.status == d.ERR_INVALID_ARG
    # a good call after the refused ones
    O = oracle_mod.Graph(src, dst, n)
    s = int(inputs_mod.pick_sources(src, dst, n, 1, seed=3)[0])
    d.bfs_noalloc(G, s, depth, None, opts=d.run_opts(want_parent=False))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(depth.cpu().numpy(), O.bfs(s, want_parent=False)[0])
    G.destroy()
    # a graph whose search scratch exceeds the static array is refused before any work
    big = 22
    nb = 1 << big
    src, dst = inputs_mod.rmat_edges(big)
    G = d.Graph(src, dst, nb, threshold=32, keep_plain_csr=False)
    dbig = torch.full((nb,), 5, dtype=torch.int32, device="cuda")
    with pytest.raises(d.DsbfsError) as e:
        d.bfs_noalloc(G, 0, dbig, None, opts=d.run_opts(want_parent=False))
    assert e.value.status == d.ERR_RANGE
    torch.cuda.synchronize()
    assert int((dbig != 5).sum()) == 0
    G.destroy()
