"""GPU parity of bit-parallel multi-source BFS: every lane's depths equal the
oracle's single-source depths, for partial batches, duplicate sources, forced
top-down-only / bottom-up-only schedules, captured-graph and cooperative
launches, and at full size (RMAT scale 24, 1024 sources: every row against
the oracle's digest)."""
import os
import tempfile

import numpy as np
import pytest

from closed_forms import disjoint_paths, grid, hypercube, path, star, two_cliques_path
from gpu_helpers import lib, log, torch_cuda

pytestmark = pytest.mark.gpu


def _opts(block=256, per_cu=4, permille=2, graph=1, lanes=0):
    d = lib()
    return d.dsbfs_ms_opts(block, per_cu, permille, graph, lanes)


def _setup(src, dst, n):
    torch_cuda()
    d = lib()
    g = d.Graph(src, dst, n, threshold=32, keep_plain_csr=True)
    ws = d.Workspace(g, max_lanes=64)
    return g, ws


def _run(g, ws, n, sources, opts):
    torch = torch_cuda()
    d = lib()
    depth = torch.full((len(sources), n), -7, dtype=torch.int32, device="cuda")
    d.msbfs(g, ws, sources, depth, opts)
    torch.cuda.synchronize()
    return depth


@pytest.mark.parametrize("permille", [0, 2, 1000])
@pytest.mark.parametrize("graph", [0, 1])
def test_msbfs_rmat12_all_lanes(inputs_mod, oracle_mod, permille, graph):
    scale = 12
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    O = oracle_mod.Graph(src, dst, n)
    g, ws = _setup(src, dst, n)
    sources = inputs_mod.pick_sources(src, dst, n, 100, seed=404)   # 2 batches, 64 + 36
    depth = _run(g, ws, n, sources, _opts(permille=permille, graph=graph)).cpu().numpy()
    for i, s in enumerate(sources.tolist()):
        want, _ = O.bfs(s, want_parent=False)
        np.testing.assert_array_equal(depth[i], want, err_msg=f"lane {i} source {s}")


@pytest.mark.parametrize("lanes", [64, 128, 256, 0])
def test_msbfs_lane_widths_rmat12(inputs_mod, oracle_mod, lanes):
    """300 sources: full and partial batches at every lane width (64: 5
    batches, 128: 3, 256: 2; 0 picks 256)."""
    scale = 12
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    O = oracle_mod.Graph(src, dst, n)
    g, ws = _setup(src, dst, n)
    sources = inputs_mod.pick_sources(src, dst, n, 300, seed=77)
    for permille in (0, 2, 1000):
        depth = _run(g, ws, n, sources, _opts(block=1024, per_cu=1, permille=permille,
                                              lanes=lanes)).cpu().numpy()
        for i, s in enumerate(sources.tolist()):
            want, _ = O.bfs(s, want_parent=False)
            np.testing.assert_array_equal(depth[i], want,
                                          err_msg=f"lanes {lanes} permille {permille} row {i}")


def test_msbfs_hubs_and_long_searches(oracle_mod):
    """Two 70-cliques joined by a 30-vertex path: clique vertices are hubs
    (degree 69 > 64: whole-wave scans and the hub frontier cache) and
    searches run past the ring of level masks; every vertex as a source."""
    n, src, dst, _ = two_cliques_path(70, 30)
    O = oracle_mod.Graph(src, dst, n)
    g, ws = _setup(src, dst, n)
    sources = np.arange(n, dtype=np.int32)
    wants = [O.bfs(int(s), want_parent=False)[0] for s in sources.tolist()]
    for lanes in (64, 0):
        for permille in (0, 2, 1000):
            depth = _run(g, ws, n, sources, _opts(block=1024, per_cu=1, permille=permille,
                                                  lanes=lanes)).cpu().numpy()
            for i in range(n):
                np.testing.assert_array_equal(depth[i], wants[i],
                                              err_msg=f"lanes {lanes} permille {permille} row {i}")


def test_msbfs_closed_forms_and_duplicates(oracle_mod):
    # the paths run far more levels than the kernel's ring of level masks
    # holds, so their depths are written in several passes, and the disjoint
    # pair leaves lanes unreached after such passes
    for n, src, dst, dist in (grid(13, 11), hypercube(8), star(70), path(150),
                              disjoint_paths(40, 33)):
        g, ws = _setup(src, dst, n)
        sources = np.array([0, 1, 0, n - 1, 5, 5, 5], dtype=np.int32)   # repeated sources
        for permille in (0, 1000):
            for lanes in (0, 256):
                depth = _run(g, ws, n, sources, _opts(permille=permille, lanes=lanes)).cpu().numpy()
                for i, s in enumerate(sources.tolist()):
                    np.testing.assert_array_equal(depth[i], dist(s),
                                                  err_msg=f"n={n} lanes {lanes} lane {i}")


def test_msbfs_launch_shapes(inputs_mod, oracle_mod):
    scale = 11
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    O = oracle_mod.Graph(src, dst, n)
    g, ws = _setup(src, dst, n)
    sources = inputs_mod.pick_sources(src, dst, n, 64, seed=5)
    wants = [O.bfs(s, want_parent=False)[0] for s in sources.tolist()]
    for block, per_cu in ((64, 1), (256, 2), (512, 4), (1024, 2)):
        depth = _run(g, ws, n, sources, _opts(block=block, per_cu=per_cu)).cpu().numpy()
        for i in range(len(sources)):
            np.testing.assert_array_equal(depth[i], wants[i], err_msg=f"{block}x{per_cu} lane {i}")
    # the same captured graph replayed several times, with other work in between
    torch = torch_cuda()
    depth = torch.empty((len(sources), n), dtype=torch.int32, device="cuda")
    for rep in range(3):
        depth.fill_(-9)
        lib().msbfs(g, ws, sources, depth, _opts(graph=1))
        torch.cuda.synchronize()
        got = depth.cpu().numpy()
        for i in range(len(sources)):
            np.testing.assert_array_equal(got[i], wants[i], err_msg=f"replay {rep} lane {i}")


@pytest.mark.parametrize("shape", ["64x16", "tuned"])
def test_msbfs_rmat24_1024_sources_all_rows(inputs_mod, oracle_mod, shape):
    """RMAT scale 24, 1024 seeded sources in one persistent launch, every one
    of the 1024 depth rows bit-exact against the oracle's digest: as 16
    batches of 64 lanes (one 64-bit lane mask per vertex), and with the
    tuner's launch configuration as the benchmark uses it."""
    from digests import RowChecker, first_difference, load, sources_of
    torch = torch_cuda()
    want = load("rmat24")
    sources = np.array(sources_of("rmat24"), dtype=np.int32)
    assert len(sources) == 1024
    scale = 24
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    assert sources.tolist() == inputs_mod.pick_sources(src, dst, n, 1024, seed=1004).tolist()
    g, ws = _setup(src, dst, n)
    if shape == "64x16":
        opts = _opts(block=1024, per_cu=1, permille=1, graph=1, lanes=64)
    else:
        opts = lib().msbfs_tune(g, ws, sources)
    log(f"scale 24 multi-source BFS, {shape}: {opts.as_dict()}")
    depth = _run(g, ws, n, sources, opts)
    log("scale 24 multi-source BFS done")
    chk = RowChecker({i: want[int(s)] for i, s in enumerate(sources.tolist())}, pending=64)
    for c0 in range(0, 1024, 64):
        block = depth[c0:c0 + 64].cpu().numpy()
        for i in range(block.shape[0]):
            chk.submit(c0 + i, block[i])
        log(f"rows {c0}..{c0 + 63} copied")
    bad = chk.mismatches()
    if bad:
        O = oracle_mod.Graph(src, dst, n)
        msgs = []
        for i, _, _ in bad[:3]:
            ref, _ = O.bfs(int(sources[i]), want_parent=False)
            msgs.append(f"row {i} (source {int(sources[i])}): "
                        f"{first_difference(depth[i].cpu().numpy(), ref)}")
        raise AssertionError(f"{len(bad)} of 1024 rows differ: " + "; ".join(msgs))
    assert chk.checked == 1024
    del depth
    torch.cuda.empty_cache()


def test_msbfs_tuner_cache(inputs_mod, oracle_mod):
    d = lib()
    scale = 12
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    g, ws = _setup(src, dst, n)
    sources = inputs_mod.pick_sources(src, dst, n, 64, seed=6)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "tune.json")
        best = d.msbfs_tune(g, ws, sources, path)
        assert best.block in (256, 512, 1024) and best.use_graph == 1
        assert os.path.exists(path)
        again = d.msbfs_tune(g, ws, sources, path)     # served from the cache
        assert again.as_dict() == best.as_dict()
        with open(path) as f:
            assert len(f.read().strip().splitlines()) == 1
    O = oracle_mod.Graph(src, dst, n)
    depth = _run(g, ws, n, sources, best).cpu().numpy()
    for i, s in enumerate(sources.tolist()[:8]):
        np.testing.assert_array_equal(depth[i], O.bfs(s, want_parent=False)[0])


def test_msbfs_errors(inputs_mod):
    torch = torch_cuda()
    d = lib()
    src, dst = inputs_mod.rmat_edges(8)
    n = 256
    g = d.Graph(src, dst, n, threshold=8, keep_plain_csr=True)
    ws0 = d.Workspace(g, max_lanes=0)
    depth = torch.empty((2, n), dtype=torch.int32, device="cuda")
    with pytest.raises(d.DsbfsError) as e:
        d.msbfs(g, ws0, np.array([1, 2], np.int32), depth)
    assert e.value.status == d.ERR_INVALID_ARG
    ws = d.Workspace(g, max_lanes=64)
    with pytest.raises(d.DsbfsError) as e:
        d.msbfs(g, ws, np.array([1, n], np.int32), depth)
    assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        d.msbfs(g, ws, np.array([1, 2], np.int32), depth, _opts(block=96))
    assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        d.msbfs(g, ws, np.array([1, 2], np.int32), depth, _opts(lanes=96))
    assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        d.Workspace(g, max_lanes=32)
    assert e.value.status == d.ERR_INVALID_ARG
    g2 = d.Graph(src, dst, n, threshold=8, keep_plain_csr=False)
    ws2 = d.Workspace(g2, max_lanes=64)
    with pytest.raises(d.DsbfsError) as e:
        d.msbfs(g2, ws2, np.array([1, 2], np.int32), depth)
    assert e.value.status == d.ERR_INVALID_ARG
