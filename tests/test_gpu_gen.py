"""Device-side RMAT generation and the builder fed by it, through the C-ABI:
the device edge list equals the seeded host generator's bit for bit; a graph
built from generated keys equals the graph built from the host edge list,
array for array; at RMAT scale 28 (4.3 billion generated pairs, beyond the
host path's reach in this test) sampled depth rows equal the oracle's
digests."""
import os

import numpy as np
import pytest

from gpu_helpers import lib, log, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scale,ef,permute,abc", [
    (8, 16, True, (0.57, 0.19, 0.19)), (12, 16, False, (0.57, 0.19, 0.19)),
    (16, 16, True, (0.57, 0.19, 0.19)), (20, 16, True, (0.57, 0.19, 0.19)),
    (14, 4, True, (0.45, 0.15, 0.15)), (13, 8, True, (0.25, 0.25, 0.25))])
def test_rmat_generate_equals_host_generator(inputs_mod, scale, ef, permute, abc):
    d = lib()
    torch_cuda()
    a, b, c = abc
    sp = d.rmat_spec(scale, edge_factor=ef, permute=permute, a=a, b=b, c=c)
    src, dst = d.rmat_generate(sp)
    hs, hd = inputs_mod.rmat_edges(scale, edge_factor=ef, permute=permute, a=a, b=b, c=c)
    np.testing.assert_array_equal(src.cpu().numpy(), hs)
    np.testing.assert_array_equal(dst.cpu().numpy(), hd)


def test_graph_from_generated_keys_equals_edge_list_build(inputs_mod, oracle_mod):
    d = lib()
    torch = torch_cuda()
    scale = 14
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    A = d.Graph(src, dst, n, threshold=16)
    B = d.Graph(None, None, 0, threshold=16, rmat=d.rmat_spec(scale))
    assert A.stats == B.stats
    for which, dt in ((0, np.int32), (1, np.int32), (3, np.uint64), (4, np.int32),
                      (5, np.uint64), (6, np.int32), (7, np.int32), (10, np.int64),
                      (11, np.int32), (12, np.int64), (13, np.int32), (16, np.uint16),
                      (17, np.int32)):
        np.testing.assert_array_equal(A.export(which, dt), B.export(which, dt), err_msg=str(which))
    O = oracle_mod.Graph(src, dst, n)
    ws = d.Workspace(B)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    for s in inputs_mod.pick_sources(src, dst, n, 4, seed=44).tolist():
        d.bfs(B, ws, s, depth, None, opts=d.run_opts(want_parent=False))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(depth.cpu().numpy(), O.bfs(s, want_parent=False)[0])
    ws.destroy()
    A.destroy()
    B.destroy()


def test_rmat28_built_on_device_sampled_rows_match_digests():
    """RMAT scale 28, TH 32, generated and built on the device (no edge list
    on the host or in HBM), single-source DOBFS from the digest file's
    sources: each depth row's SHA-256 equals the oracle's, and the
    component sizes match."""
    from digests import GOLD, load, row_digest, sources_of
    if not os.path.exists(os.path.join(GOLD, "depth_digests_rmat28.txt")):
        pytest.skip("oracle digests of RMAT scale 28 not written")
    d = lib()
    torch = torch_cuda()
    want = load("rmat28")
    n = 1 << 28
    G = d.Graph(None, None, 0, threshold=32, keep_plain_csr=False, rmat=d.rmat_spec(28))
    log(f"scale 28 graph: m_dir={G.stats['m_dir']} d={G.stats['d']}")
    ws = d.Workspace(G)
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    for s in sources_of("rmat28"):
        st = d.bfs(G, ws, s, depth, parent, opts=d.run_opts(want_parent=True), want_stats=True)
        torch.cuda.synchronize()
        row = depth.cpu().numpy()
        assert st["reached"] == want[s]["reached"] and st["edges_cc"] == want[s]["edges_cc"], s
        assert row_digest(row) == want[s]["sha256"], f"source {s}: depth row differs"
        # parents: one level shallower than their child, for a sample
        par = parent.cpu().numpy()
        rng = np.random.default_rng(s)
        vs = rng.choice(np.nonzero(row > 0)[0], size=4096, replace=False)
        assert np.all(row[par[vs]] == row[vs] - 1)
        log(f"scale 28 source {s}: {st['num_levels']} levels, row equals the oracle's")
    ws.destroy()
    G.destroy()
