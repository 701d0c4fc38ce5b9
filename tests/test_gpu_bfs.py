"""GPU parity of single-source BFS (plain top-down and degree-separated DOBFS)
against the CPU oracle and closed forms, through the C-ABI library.

Depths must match bit-exactly; parents are checked by the oracle's invariant
checker (several trees are correct)."""
import numpy as np
import pytest

from closed_forms import all_closed_forms
from gpu_helpers import GpuGraph, lib, log

pytestmark = pytest.mark.gpu

TH_CLOSED = (0, 1, 2, 3, 8, 10**6)


@pytest.mark.parametrize("case", all_closed_forms(), ids=lambda c: c[0])
def test_closed_forms_all_modes(oracle_mod, case):
    name, n, src, dst, dist, sources = case
    O = oracle_mod.Graph(src, dst, n)
    label = O.components()
    for TH in TH_CLOSED:
        log(f"closed form {name} n={n} TH={TH}")
        G = GpuGraph(src, dst, n, threshold=TH)
        for s in sources:
            want = dist(s)
            for mode, forced, seed in ((0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 2, 0), (1, 3, 7),
                                       (1, 3, 8)):
                depth, parent, _ = G.bfs(s, mode=mode, forced=forced, seed=seed)
                np.testing.assert_array_equal(depth, want,
                                              err_msg=f"{name} TH={TH} s={s} mode={mode} f={forced}")
                assert O.check(s, depth, parent, label)[0] == 0, (name, TH, s, mode, forced)
        G.close()


def _rmat(inputs_mod, oracle_mod, scale):
    src, dst = inputs_mod.rmat_edges(scale)
    n = 1 << scale
    return n, src, dst, oracle_mod.Graph(src, dst, n)


@pytest.mark.parametrize("scale,TH", [(10, 8), (12, 16), (14, 32), (16, 32), (16, 64)])
def test_rmat_parity(inputs_mod, oracle_mod, scale, TH):
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, scale)
    label = O.components()
    deg = O.degrees()
    G = GpuGraph(src, dst, n, threshold=TH)
    sources = inputs_mod.pick_sources(src, dst, n, 24, seed=2000 + scale)
    for s in sources.tolist():
        want, _ = O.bfs(s, want_parent=False)
        for mode in (0, 1):
            depth, parent, st = G.bfs(s, mode=mode, want_stats=True)
            log(f"rmat scale={scale} TH={TH} s={s} mode={mode} levels={st['num_levels']}")
            np.testing.assert_array_equal(depth, want)
            assert O.check(s, depth, parent, label)[0] == 0
            reached = want >= 0
            assert st["reached"] == int(reached.sum())
            assert st["edges_cc"] == int(deg[reached].sum() // 2)
    G.close()


def test_profiled_and_captured_levels_agree(inputs_mod, oracle_mod):
    """The search runs its levels as captured graphs, or (profile = 1) as
    direct launches timed kernel by kernel; both give the oracle's depths, the
    same level records and the same counts of kernels that had work."""
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, 14)
    label = O.components()
    G = GpuGraph(src, dst, n, threshold=16)
    for s in inputs_mod.pick_sources(src, dst, n, 8, seed=77).tolist():
        want, _ = O.bfs(s, want_parent=False)
        runs = []
        for prof in (False, True, False):
            depth, parent, st = G.bfs(s, want_stats=True, profile=prof)
            np.testing.assert_array_equal(depth, want)
            assert O.check(s, depth, parent, label)[0] == 0
            runs.append(st)
        a, b = runs[0], runs[1]
        log(f"profiled vs captured s={s} levels={a['num_levels']}")
        assert a["num_levels"] == b["num_levels"]
        assert a["levels"] == b["levels"]
        assert (a["reached"], a["edges_cc"]) == (b["reached"], b["edges_cc"])
        for k in a["kernels"]:
            assert a["kernels"][k]["launches"] == b["kernels"][k]["launches"], k
            assert a["kernels"][k]["bytes"] == b["kernels"][k]["bytes"], k
        assert b["kernels"]["prev_normal"]["ms"] > 0
        assert runs[2]["levels"] == a["levels"]
    G.close()


def test_level_graph_replays_and_recapture(inputs_mod, oracle_mod):
    """Captured level graphs replayed over many searches with eager work in
    between, then re-captured for other output buffers: every search matches
    the oracle."""
    d = lib()
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, 12)
    G = GpuGraph(src, dst, n, threshold=8)
    torch = G.torch
    srcs = inputs_mod.pick_sources(src, dst, n, 4, seed=91).tolist()
    want = {s: O.bfs(s, want_parent=False)[0] for s in srcs}
    bufs = [(G.depth, G.parent),
            (torch.empty(n, dtype=torch.int32, device="cuda"),
             torch.empty(n, dtype=torch.int32, device="cuda"))]
    junk = torch.zeros(1 << 20, device="cuda")
    for rnd in range(3):
        for depth_t, parent_t in bufs:
            for s in srcs:
                junk.add_(1.0)                      # eager work between replays
                d.bfs(G.g, G.ws, s, depth_t, parent_t if rnd != 1 else None,
                      opts=d.run_opts(want_parent=rnd != 1))
                torch.cuda.synchronize()
                np.testing.assert_array_equal(depth_t.cpu().numpy(), want[s],
                                              err_msg=f"round {rnd} source {s}")
    assert float(junk[0]) == 3 * 2 * len(srcs)
    G.close()


def test_plain_rmat16_64_sources(inputs_mod, oracle_mod):
    """Plain top-down BFS, RMAT scale 16, 64 seeded sources with degree >= 1."""
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, 16)
    label = O.components()
    G = GpuGraph(src, dst, n, threshold=32)
    sources = inputs_mod.pick_sources(src, dst, n, 64, seed=1001)
    assert len(sources) == 64
    for s in sources.tolist():
        want, _ = O.bfs(s, want_parent=False)
        depth, parent, _ = G.bfs(s, mode=0)
        np.testing.assert_array_equal(depth, want)
        assert O.check(s, depth, parent, label)[0] == 0
    G.close()


def _oracle_row_report(inputs_mod, oracle_mod, scale, bad, rows):
    """Message for digest mismatches: recomputes the oracle row of each bad
    source (at most 3) and names the first differing vertex."""
    from digests import first_difference
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    O = oracle_mod.Graph(src, dst, n)
    msgs = []
    for key, got, want in bad[:3]:
        s = key[-1] if isinstance(key, tuple) else key
        ref, _ = O.bfs(int(s), want_parent=False)
        msgs.append(f"{key}: {first_difference(rows[key], ref)}")
    return f"{len(bad)} rows differ from the oracle: " + "; ".join(msgs)


def test_do_rmat22_all_64_sources(inputs_mod, oracle_mod):
    """Degree-separated DOBFS, TH = 32, RMAT scale 22, all 64 seeded sources:
    every depth row bit-exact against the oracle's digest, every parent array
    through the oracle's invariant checker, and the component's size and edge
    count per source."""
    import concurrent.futures as cf
    from digests import RowChecker, load, sources_of, threads
    want = load("rmat22")
    sources = sources_of("rmat22")
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, 22)
    assert sources == inputs_mod.pick_sources(src, dst, n, 64, seed=1002).tolist()
    log("scale 22 oracle graph built")
    G = GpuGraph(src, dst, n, threshold=32)
    st = O.split_stats(32)
    for k in ("d", "e_nn", "e_nd", "e_dn", "e_dd", "n_ndsrc", "n_ddsrc", "n_dnsrc"):
        assert G.stats[k] == st[k], k
    assert G.stats["m_dir"] == O.m
    chk = RowChecker(want)
    pool = cf.ThreadPoolExecutor(max_workers=threads())
    checks, rows = [], {}
    for i, s in enumerate(sources):
        depth, parent, rs = G.bfs(s, mode=1, want_stats=True)
        assert rs["reached"] == want[s]["reached"] and rs["edges_cc"] == want[s]["edges_cc"], s
        assert rs["num_levels"] == want[s]["max_depth"] + 1, s
        rows[s] = depth
        chk.submit(s, depth)
        checks.append((s, pool.submit(O.check, s, depth, parent, None)))
        if i % 16 == 15:
            log(f"scale 22: {i + 1} of 64 sources searched")
    bad = chk.mismatches()
    assert not bad, _oracle_row_report(inputs_mod, oracle_mod, 22, bad, rows)
    for s, f in checks:
        assert f.result()[0] == 0, f"parent invariants fail from source {s}: {f.result()}"
    pool.shutdown()
    log(f"scale 22: {chk.checked} rows equal the oracle's")
    G.close()


def test_do_rmat26_64_sources_each_threshold(inputs_mod, oracle_mod):
    """RMAT scale 26 (2.1e9 directed edges, within 2% of 2^31), the bench's
    configuration (captured level graphs, parents on): at TH 16, 32, 64 and
    128, all 64 seeded sources, every depth row bit-exact against the oracle's
    digest and the component size and edge count per source; at TH 32 every
    parent array also passes the oracle's invariant checker."""
    import concurrent.futures as cf
    from digests import RowChecker, load, sources_of, threads
    want = load("rmat26")
    sources = sources_of("rmat26")
    scale = 26
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    assert sources == inputs_mod.pick_sources(src, dst, n, 64, seed=1003).tolist()
    O = oracle_mod.Graph(src, dst, n)
    log("scale 26 oracle graph built")
    for TH in (32, 16, 64, 128):
        G = GpuGraph(src, dst, n, threshold=TH, keep_plain=False)
        assert G.stats["m_dir"] == O.m and O.m > 2 * 10 ** 9
        chk = RowChecker(want, pending=8)
        pool = cf.ThreadPoolExecutor(max_workers=threads()) if TH == 32 else None
        checks, rows = [], {}
        for i, s in enumerate(sources):
            depth, parent, rs = G.bfs(s, want_stats=True, want_parent=TH == 32)
            assert rs["reached"] == want[s]["reached"], (TH, s)
            assert rs["edges_cc"] == want[s]["edges_cc"], (TH, s)
            chk.submit(s, depth)
            if pool is not None:
                checks.append((s, pool.submit(O.check, s, depth, parent, None)))
                if len(checks) >= 16:   # bound the rows held for checking
                    s0, f0 = checks.pop(0)
                    assert f0.result()[0] == 0, f"parent invariants fail from {s0}: {f0.result()}"
            if i % 16 == 15:
                log(f"scale 26 TH {TH}: {i + 1} of 64 sources searched")
        bad = chk.mismatches()
        if bad:
            rows = {k: G.bfs(k, want_parent=False)[0] for k, _, _ in bad[:3]}
            G.close()
            del src, dst
            raise AssertionError(f"TH {TH}: " +
                                 _oracle_row_report(inputs_mod, oracle_mod, 26, bad, rows))
        for s, f in checks:
            assert f.result()[0] == 0, f"parent invariants fail from source {s}: {f.result()}"
        if pool is not None:
            pool.shutdown()
        log(f"scale 26 TH {TH}: {chk.checked} rows equal the oracle's")
        G.close()


def test_schedule_and_threshold_invariance(inputs_mod, oracle_mod):
    """Direction never changes depths (Section IV-B), nor does TH."""
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, 14)
    maxdeg = int(O.degrees().max())
    sources = inputs_mod.pick_sources(src, dst, n, 6, seed=77)
    wants = {s: O.bfs(s, want_parent=False)[0] for s in sources.tolist()}
    for TH in (0, 16, 32, 64, 128, maxdeg):
        G = GpuGraph(src, dst, n, threshold=TH)
        for s, want in wants.items():
            for forced, seed in [(0, 0), (1, 0), (2, 0)] + [(3, k) for k in range(8)]:
                depth, parent, _ = G.bfs(s, forced=forced, seed=seed)
                np.testing.assert_array_equal(depth, want, err_msg=f"TH={TH} f={forced}/{seed}")
                assert O.check(s, depth, parent, None)[0] == 0
        G.close()


@pytest.mark.parametrize("TH", [2, 32, 10**6])
def test_without_compact_nn_copy(inputs_mod, oracle_mod, TH):
    """skip_nn_copy = 1: the forward nn visits read the packed offsets and the
    full rows (the path a graph with e_nn >= 2^32 takes). Depths equal the
    oracle's and parents pass its invariants under the heuristic schedule,
    all forward, and with nn under the decision; arrays 18 and 19 are empty."""
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, 13)
    G = GpuGraph(src, dst, n, threshold=TH, nn_copy=False)
    assert len(G.g.export(18, np.uint32)) == 0 and len(G.g.export(19, np.int32)) == 0
    for s in inputs_mod.pick_sources(src, dst, n, 4, seed=91).tolist():
        want, _ = O.bfs(s, want_parent=False)
        for kw in ({}, {"forced": 1}, {"nn_do": True, "factor_nn": (1e-3, 0.0)}):
            depth, parent, _ = G.bfs(s, **kw)
            np.testing.assert_array_equal(depth, want, err_msg=f"TH={TH} {kw}")
            assert O.check(s, depth, parent, None)[0] == 0
    G.close()


@pytest.mark.parametrize("scale,TH", [(12, 8), (14, 16), (16, 32)])
def test_direction_schedule_matches_oracle_replay(inputs_mod, oracle_mod, scale, TH):
    """Per-level q, s, |U|, FV, BV and the chosen directions equal the oracle's
    replay of Section IV-B from its own level sets."""
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, scale)
    G = GpuGraph(src, dst, n, threshold=TH)
    for f0 in ((0.5, 0.05, 1e-7), (10.0, 10.0, 10.0), (1e-3, 1e-3, 1e-3)):
        for f1 in ((0.0, 0.0, 0.0), (0.2, 0.5, 2.0)):
            for s in inputs_mod.pick_sources(src, dst, n, 4, seed=31 + scale).tolist():
                want, _ = O.bfs(s, want_parent=False)
                depth, _, st = G.bfs(s, want_stats=True, factor0=f0, factor1=f1)
                np.testing.assert_array_equal(depth, want)
                rep = O.do_replay(TH, want, f0, f1)
                assert st["num_levels"] == len(rep)
                for L, (a, b) in enumerate(zip(st["levels"], rep)):
                    for k in ("q", "s", "U", "FV", "dir"):
                        assert a[k] == b[k], (L, k, a[k], b[k])
                    assert a["BV"] == b["BV"], (L, a["BV"], b["BV"])
                    assert a["FV_nn"] == b["FV_nn"] and a["q_nn"] == b["q_nn"]
                    assert a["frontier_normal"] == b["frontier_normal"]
                    assert a["frontier_delegate"] == b["frontier_delegate"]
    G.close()


def _deg_bucket(x):
    """Log-scale degree bucket: 8 per power of two (floor(log2) and the next
    three bits), capped at 255."""
    if x <= 1:
        return 0
    lg = x.bit_length() - 1
    frac = (x >> (lg - 3)) & 7 if lg >= 3 else (x << (3 - lg)) & 7
    return min(lg * 8 + frac, 255)


def _buckets(deg):
    """Vectorized _deg_bucket."""
    deg = np.asarray(deg, dtype=np.int64)
    out = np.zeros(deg.shape, dtype=np.int64)
    m = deg > 1
    lg = np.zeros(deg.shape, dtype=np.int64)
    lg[m] = np.floor(np.log2(deg[m])).astype(np.int64)
    hi = m & (lg >= 3)
    lo = m & (lg < 3)
    frac = np.zeros(deg.shape, dtype=np.int64)
    frac[hi] = (deg[hi] >> (lg[hi] - 3)) & 7
    frac[lo] = (deg[lo] << (3 - lg[lo])) & 7
    out[m] = np.minimum(lg[m] * 8 + frac[m], 255)
    return out


def _check_degree_ordered_rows(off, col, want_col, deg):
    """Every row holds the oracle's neighbours, ordered by neighbour degree
    bucket (highest first), ties by ascending ID."""
    off = np.asarray(off, dtype=np.int64)
    n = len(off) - 1
    row = np.repeat(np.arange(n), np.diff(off))
    order = np.lexsort((col, row))
    np.testing.assert_array_equal(col[order], want_col)
    b = 255 - _buckets(deg[col])
    same = row[1:] == row[:-1]
    ok = (b[1:] > b[:-1]) | ((b[1:] == b[:-1]) & (col[1:] > col[:-1]))
    assert np.all(ok | ~same)


def _decode(off):
    off = off.astype(np.uint64)
    start = (off & np.uint64((1 << 40) - 1)).astype(np.int64)
    first = (off >> np.uint64(40)).astype(np.int64)
    return start, first


@pytest.mark.parametrize("scale,TH", [(8, 0), (10, 2), (10, 8), (12, 32), (12, 10**6)])
def test_builder_layout_matches_oracle_split(inputs_mod, oracle_mod, scale, TH):
    n, src, dst, O = _rmat(inputs_mod, oracle_mod, scale)
    G = GpuGraph(src, dst, n, threshold=TH)
    g = G.g
    st = O.split_stats(TH)
    for k in ("d", "e_nn", "e_nd", "e_dn", "e_dd", "n_ndsrc", "n_ddsrc", "n_dnsrc"):
        assert G.stats[k] == st[k], k
    assert G.stats["m_dir"] == O.m and G.stats["max_degree"] == st["max_deg"]
    assert G.stats["bytes_layout"] == 8 * (n + 1) + 8 * (st["d"] + 1) + 4 * O.m
    r = O.split_rows(TH)
    d = st["d"]
    np.testing.assert_array_equal(g.export(0, np.int32), O.degrees())
    np.testing.assert_array_equal(g.export(1, np.int32), r["did"])
    np.testing.assert_array_equal(g.export(2, np.int32), np.nonzero(r["did"] >= 0)[0])
    np.testing.assert_array_equal(g.export(10, np.int64), O.off)
    _check_degree_ordered_rows(O.off, g.export(11, np.int32), O.col, O.degrees())
    ns, nf = _decode(g.export(3, np.uint64))
    ncol = g.export(4, np.int32)
    nn_len = np.diff(r["nn_off"])
    nd_len = np.diff(r["nd_off"])
    np.testing.assert_array_equal(nf[:n], nn_len)
    lens = g.export(16, np.uint16).astype(np.int64)
    fits = (nn_len < 255) & (nd_len < 255)
    np.testing.assert_array_equal(lens[fits], (nn_len | (nd_len << 8))[fits])
    assert np.all(lens[~fits] == 0xFFFF)
    np.testing.assert_array_equal(np.diff(ns), nn_len + nd_len)
    deg = O.degrees()
    vid = np.nonzero(r["did"] >= 0)[0]
    for v in range(n):
        row = ncol[ns[v]:ns[v + 1]]
        assert row[:nf[v]].tolist() == r["nn_col"][r["nn_off"][v]:r["nn_off"][v + 1]].tolist()
        nd_part = row[nf[v]:]
        want = r["nd_col"][r["nd_off"][v]:r["nd_off"][v + 1]]
        assert sorted(nd_part.tolist()) == want.tolist()
        if len(nd_part) <= 64:   # degree descending, ties by ascending delegate ID
            keys = [(-int(deg[vid[x]]), int(x)) for x in nd_part]
            assert keys == sorted(keys), v
    ds, df = _decode(g.export(5, np.uint64))
    dcol = g.export(6, np.int32)
    assert len(ds) == d + 1
    for k in range(d):
        row = dcol[ds[k]:ds[k + 1]]
        dd_part = row[:df[k]]
        assert sorted(dd_part.tolist()) == \
            r["dd_col"][r["dd_off"][k]:r["dd_off"][k + 1]].tolist()
        keys = [(-_deg_bucket(int(deg[vid[x]])), int(x)) for x in dd_part]
        assert keys == sorted(keys), k
        assert row[df[k]:].tolist() == r["dn_col"][r["dn_off"][k]:r["dn_off"][k + 1]].tolist()
    nd_src = np.nonzero(nd_len > 0)[0]
    np.testing.assert_array_equal(g.export(7, np.int32), nd_src)
    nn_src = np.nonzero(nn_len > 0)[0]
    np.testing.assert_array_equal(g.export(17, np.int32), nn_src)
    assert G.stats["n_nnsrc"] == len(nn_src)
    # the compact nn copy is the oracle's nn subgraph in CSR form: part starts
    # (32-bit) and the parts concatenated in vertex order
    np.testing.assert_array_equal(g.export(18, np.uint32).astype(np.int64), r["nn_off"][:n])
    np.testing.assert_array_equal(g.export(19, np.int32), r["nn_col"])
    nds_off = g.export(12, np.int64)
    nds_col = g.export(13, np.int32)
    np.testing.assert_array_equal(np.diff(nds_off), nd_len[nd_src])
    for i, v in enumerate(nd_src.tolist()):   # the row's own nd part, in the same order
        assert nds_col[nds_off[i]:nds_off[i + 1]].tolist() == \
            ncol[ns[v] + nf[v]:ns[v + 1]].tolist()
    ddf = g.export(15, np.int32).reshape(-1, 2)
    assert len(ddf) == d
    for k in range(d):
        if df[k] > 0:
            assert ddf[k, 0] == dcol[ds[k]] and ddf[k, 1] == vid[ddf[k, 0]]
        else:
            assert ddf[k].tolist() == [-1, -1]
    first = g.export(14, np.int32).reshape(-1, 2)
    assert len(first) == len(nd_src)
    if len(nd_src):
        np.testing.assert_array_equal(first[:, 0], nds_col[nds_off[:-1]])
        np.testing.assert_array_equal(first[:, 1], vid[first[:, 0]])
    words = (d + 31) // 32
    for which, lens in ((8, np.diff(r["dd_off"])), (9, np.diff(r["dn_off"]))):
        m = g.export(which, np.uint32)
        assert len(m) == words
        bits = np.unpackbits(m.view(np.uint8), bitorder="little")[:d]
        np.testing.assert_array_equal(bits, (lens > 0).astype(np.uint8))
    G.close()


def test_degenerate_inputs(oracle_mod):
    # isolated source: depth 0 there, -1 elsewhere
    src = np.array([1, 2, 3], np.int32)
    dst = np.array([2, 3, 1], np.int32)
    G = GpuGraph(src, dst, 6, threshold=1)
    for mode in (0, 1):
        depth, parent, st = G.bfs(0, mode=mode, want_stats=True)
        assert depth.tolist() == [0, -1, -1, -1, -1, -1]
        assert parent.tolist() == [0, -1, -1, -1, -1, -1]
        assert st["reached"] == 1 and st["edges_cc"] == 0
    G.close()
    # no edges at all; one vertex; only self-loops and duplicates
    for src, dst, n in ((np.zeros(0, np.int32), np.zeros(0, np.int32), 4),
                        (np.zeros(0, np.int32), np.zeros(0, np.int32), 1),
                        (np.array([0, 1, 1, 1, 2], np.int32), np.array([0, 1, 2, 2, 1], np.int32), 3)):
        G = GpuGraph(src, dst, n, threshold=0)
        O = oracle_mod.Graph(src, dst, n)
        for s in range(n):
            want, _ = O.bfs(s)
            for mode in (0, 1):
                depth, parent, _ = G.bfs(s, mode=mode)
                np.testing.assert_array_equal(depth, want)
                assert O.check(s, depth, parent, None)[0] == 0
        G.close()


def test_error_paths():
    d = lib()
    import torch
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 2], np.int32)
    G = GpuGraph(src, dst, 3, threshold=1)
    for bad in (-1, 3, 1 << 30):
        with pytest.raises(d.DsbfsError) as e:
            G.bfs(bad)
        assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        d.bfs(G.g, G.ws, 0, G.depth, None, opts=d.run_opts(want_parent=True))
    assert e.value.status == d.ERR_INVALID_ARG
    G.close()
    with pytest.raises(d.DsbfsError) as e:
        d.Graph(np.array([0, 5], np.int32), np.array([1, 1], np.int32), 5)
    assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        d.Graph(np.array([0, -2], np.int32), np.array([1, 1], np.int32), 5)
    assert e.value.status == d.ERR_INVALID_ARG
    G2 = GpuGraph(src, dst, 3, threshold=1, keep_plain=False)
    with pytest.raises(d.DsbfsError) as e:
        G2.bfs(0, mode=0)
    assert e.value.status == d.ERR_INVALID_ARG
    depth, parent, _ = G2.bfs(0, mode=1)
    assert depth.tolist() == [0, 1, 2]
    G2.close()
    torch.cuda.synchronize()
