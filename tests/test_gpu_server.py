"""GPU tests of the query server: every served result equals the oracle, the
same query gives the same result alone and in a mix (continuous batching),
plain, batched and adaptive modes agree, admission follows the HBM budget, and errors
are reported as status codes."""
import time

import numpy as np
import pytest

from closed_forms import disjoint_paths, path
from gpu_helpers import lib, log, torch_cuda

pytestmark = pytest.mark.gpu

BIG = 1 << 40


def _graphs(inputs_mod, oracle_mod):
    """Three small resident graphs: RMAT 10, RMAT 12, ER n=3000 (avg degree ~16)."""
    specs = []
    for scale in (10, 12):
        src, dst = inputs_mod.rmat_edges(scale)
        specs.append((1 << scale, src, dst))
    src, dst = inputs_mod.er_edges(3000, 8 * 3000, seed=0x22)
    specs.append((3000, src, dst))
    return [(n, s, d, oracle_mod.Graph(s, d, n)) for n, s, d in specs]


def _server(specs, batched, budget=BIG, lanes=64):
    torch_cuda()
    d = lib()
    S = d.Server(budget, max_lanes=lanes, batched=batched)
    gids = []
    for n, s, t, _ in specs:
        g = d.Graph(s, t, n, threshold=16, keep_plain_csr=True)
        gids.append(S.add_graph(g))
    return S, gids


def _fetch(S, ticket, n):
    d = lib()
    ptr, st = S.wait(ticket)
    row = d.device_row(ptr, n).cpu().numpy().copy()
    S.release(ticket)
    return row, st


@pytest.mark.parametrize("batched", [1, 0, 2])
def test_server_mix_matches_oracle(inputs_mod, oracle_mod, batched):
    specs = _graphs(inputs_mod, oracle_mod)
    S, gids = _server(specs, batched)
    rng = np.random.default_rng(7)
    jobs = []
    for i in range(300):
        k = int(rng.integers(0, len(specs)))
        n, src, dst, _ = specs[k]
        s = int(inputs_mod.pick_sources(src, dst, n, 1, seed=5000 + i)[0])
        jobs.append((k, s, S.submit(gids[k], s)))
        if i % 50 == 49:
            time.sleep(0.002)   # arrivals in bursts, while earlier ones run
    for k, s, t in jobs:
        n, _, _, O = specs[k]
        row, st = _fetch(S, t, n)
        want, _ = O.bfs(s, want_parent=False)
        np.testing.assert_array_equal(row, want, err_msg=f"graph {k} source {s}")
        assert st["done_ns"] >= st["start_ns"] >= st["admit_ns"] >= st["arrival_ns"] > 0
        assert st["batched"] == int(batched) or (batched == 2 and st["batched"] in (0, 1))
    S.destroy()


def test_server_long_paths(oracle_mod):
    """Searches far longer than the kernel's ring of level masks (a path of
    150 vertices, and two disjoint paths so that rows also hold -1), with
    queries joining at different levels: rows are written in several passes
    per lane, each lane from its own start level."""
    forms = [path(150), disjoint_paths(60, 50)]
    specs = [(n, s, t, None) for n, s, t, _ in forms]
    S, gids = _server(specs, 1)
    rng = np.random.default_rng(11)
    jobs = []
    for i in range(60):
        k = i % 2
        n = forms[k][0]
        src = int(rng.integers(0, n))
        jobs.append((k, src, S.submit(gids[k], src)))
        if i % 6 == 5:
            time.sleep(0.003)
    for k, src, t in jobs:
        n, _, _, dist = forms[k]
        row, st = _fetch(S, t, n)
        np.testing.assert_array_equal(row, dist(src), err_msg=f"graph {k} source {src}")
        assert st["batched"] == 1
    S.destroy()


def test_server_adaptive_uses_both_forms(inputs_mod, oracle_mod):
    """Adaptive mode: a lone query runs as a single-source search; a burst of
    48 queries on one graph opens a batch. Every row equals the oracle's."""
    specs = _graphs(inputs_mod, oracle_mod)
    S, gids = _server(specs, 2)
    n, src, dst, O = specs[1]
    srcs = inputs_mod.pick_sources(src, dst, n, 49, seed=31).tolist()
    row, st = _fetch(S, S.submit(gids[1], int(srcs[0])), n)
    assert st["batched"] == 0
    np.testing.assert_array_equal(row, O.bfs(int(srcs[0]), want_parent=False)[0])
    tickets = [S.submit(gids[1], int(s)) for s in srcs[1:]]
    forms = []
    for s, t in zip(srcs[1:], tickets):
        row, st = _fetch(S, t, n)
        forms.append(st["batched"])
        np.testing.assert_array_equal(row, O.bfs(int(s), want_parent=False)[0],
                                      err_msg=f"source {s}")
    log(f"adaptive burst: {sum(forms)} of {len(forms)} queries ran as lanes")
    assert sum(forms) > 0
    S.destroy()


def test_server_rejects_unknown_mode():
    d = lib()
    torch_cuda()
    with pytest.raises(d.DsbfsError) as e:
        d.Server(BIG, batched=3)
    assert e.value.status == d.ERR_INVALID_ARG


def test_server_alone_equals_in_mix(inputs_mod, oracle_mod):
    """A query served alone and the same query served among 100 others that
    keep arriving while it runs give identical depth rows."""
    specs = _graphs(inputs_mod, oracle_mod)
    n, src, dst, O = specs[1]
    probe = int(inputs_mod.pick_sources(src, dst, n, 1, seed=99)[0])
    S, gids = _server(specs, True)
    alone, _ = _fetch(S, S.submit(gids[1], probe), n)
    tickets = [S.submit(gids[i % 3], int(inputs_mod.pick_sources(
        specs[i % 3][1], specs[i % 3][2], specs[i % 3][0], 1, seed=700 + i)[0]))
        for i in range(50)]
    mid = S.submit(gids[1], probe)
    tickets += [S.submit(gids[i % 3], int(inputs_mod.pick_sources(
        specs[i % 3][1], specs[i % 3][2], specs[i % 3][0], 1, seed=800 + i)[0]))
        for i in range(50)]
    mixed, st = _fetch(S, mid, n)
    for t in tickets:
        S.wait(t)
        S.release(t)
    np.testing.assert_array_equal(alone, mixed)
    np.testing.assert_array_equal(alone, O.bfs(probe, want_parent=False)[0])
    S.destroy()


def test_server_budget_admission(inputs_mod, oracle_mod):
    d = lib()
    specs = _graphs(inputs_mod, oracle_mod)[:1]       # RMAT 10, n = 1024
    n, src, dst, O = specs[0]
    torch_cuda()
    # a budget too small for the graph itself
    S = d.Server(1024, batched=True)
    g = d.Graph(src, dst, n, threshold=16, keep_plain_csr=True)
    with pytest.raises(d.DsbfsError) as e:
        S.add_graph(g)
    assert e.value.status == d.ERR_BUDGET
    g.destroy()
    S.destroy()
    # find the smallest budget that admits the graph (its resident footprint
    # plus one result row, by bisection), then allow exactly two result rows
    def admits(budget):
        S = d.Server(budget, batched=True)
        g = d.Graph(src, dst, n, threshold=16, keep_plain_csr=True)
        try:
            S.add_graph(g)
            return True
        except d.DsbfsError as err:
            assert err.status == d.ERR_BUDGET
            g.destroy()
            return False
        finally:
            S.destroy()

    lo, hi = 0, 1 << 30
    assert admits(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if admits(mid):
            hi = mid
        else:
            lo = mid
    foot = hi   # footprint + one row of 4n bytes
    S = d.Server(foot + 2 * 4 * n - 1, batched=True)
    gid = S.add_graph(d.Graph(src, dst, n, threshold=16, keep_plain_csr=True))
    sources = inputs_mod.pick_sources(src, dst, n, 5, seed=3)
    ts = [S.submit(gid, int(s)) for s in sources]
    S.wait(ts[0])
    S.wait(ts[1])
    with pytest.raises(d.DsbfsError) as e:
        S.wait(ts[2], timeout_ns=200_000_000)        # no row free: still waiting
    assert e.value.status == d.ERR_NOT_READY
    S.release(ts[0])
    row, _ = _fetch(S, ts[2], n)
    np.testing.assert_array_equal(row, O.bfs(int(sources[2]), want_parent=False)[0])
    S.release(ts[1])
    for t, s in ((ts[3], sources[3]), (ts[4], sources[4])):
        row, _ = _fetch(S, t, n)
        np.testing.assert_array_equal(row, O.bfs(int(s), want_parent=False)[0])
    S.destroy()
    # the footprint is what the server charges for the resident graph
    S = d.Server(foot, batched=True)
    S.add_graph(d.Graph(src, dst, n, threshold=16, keep_plain_csr=True))
    st = S.stats()
    assert st["used_bytes"] == foot - 4 * n and st["resident_graphs"] == 1
    S.destroy()


def test_server_errors(inputs_mod, oracle_mod):
    d = lib()
    specs = _graphs(inputs_mod, oracle_mod)[:1]
    S, gids = _server(specs, True)
    n = specs[0][0]
    for gid, s in ((5, 0), (-1, 0), (gids[0], n), (gids[0], -3)):
        with pytest.raises(d.DsbfsError) as e:
            S.submit(gid, s)
        assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        S.wait(12345)
    assert e.value.status == d.ERR_INVALID_ARG
    t = S.submit(gids[0], 1)
    S.wait(t)
    S.release(t)
    with pytest.raises(d.DsbfsError) as e:
        S.release(t)
    assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DsbfsError) as e:
        d.Server(1 << 30, max_lanes=65)
    assert e.value.status == d.ERR_INVALID_ARG
    S.destroy()


@pytest.mark.parametrize("batched", [1, 2])
def test_server_real_mix_rows_match_digests(inputs_mod, batched):
    """The served mix at its real sizes: RMAT scales 18, 20, 22, 24 and an
    Erdos-Renyi graph with 2^22 vertices and 8n pairs, TH 32, all resident.
    The 320 digest queries (64 sources per graph) arrive shuffled as a
    Poisson stream at 1500 queries/s; every returned row must equal the
    oracle's depth row (SHA-256 digest), for continuous batching (1) and the
    adaptive mode (2)."""
    import threading
    from digests import load, row_digest
    d = lib()
    torch_cuda()
    want = load("served")
    specs = [("rmat", 18), ("rmat", 20), ("rmat", 22), ("rmat", 24), ("er", 22)]
    S = d.Server(BIG, max_lanes=64, batched=batched)
    gids, ns = [], []
    for kind, sc in specs:
        n = 1 << sc
        if kind == "rmat":
            src, dst = inputs_mod.rmat_edges(sc)
        else:
            src, dst = inputs_mod.er_edges(n, 8 * n, seed=0x22)
        gi = len(gids)
        picked = inputs_mod.pick_sources(src, dst, n, 64, seed=6000 + gi).tolist()
        assert sorted(picked) == sorted(s for g, s in want if g == gi)
        gids.append(S.add_graph(d.Graph(src, dst, n, threshold=32, keep_plain_csr=True)))
        ns.append(n)
        log(f"served graph {gi} ({kind} {sc}) resident")
    keys = sorted(want)
    rng = np.random.default_rng(5100 + batched)
    order = rng.permutation(len(keys))
    gaps = rng.exponential(1.0 / 1500.0, size=len(keys))
    tickets = [None] * len(keys)
    ready = threading.Semaphore(0)
    bad, done = [], []

    def collect():
        for j in range(len(keys)):
            ready.acquire()
            gi, s = keys[order[j]]
            ptr, st = S.wait(tickets[j])
            row = d.device_row(ptr, ns[gi]).cpu().numpy()
            S.release(tickets[j])
            if row_digest(row) != want[(gi, s)]["sha256"]:
                bad.append((gi, s))
            done.append(st["batched"])

    th = threading.Thread(target=collect)
    th.start()
    at = d.now_ns() + 1_000_000
    for j in range(len(keys)):
        at += int(gaps[j] * 1e9)
        while d.now_ns() < at:
            time.sleep(50e-6)
        gi, s = keys[order[j]]
        tickets[j] = S.submit(gids[gi], s, at)
        ready.release()
    th.join()
    S.destroy()
    log(f"served {len(done)} queries, {sum(done)} as lanes, {len(bad)} rows differ")
    assert len(done) == len(keys)
    assert not bad, f"served rows differ from the oracle for (graph, source) {bad[:5]}"
    if batched == 1:
        assert sum(done) == len(keys)


def _footprints(specs, batched):
    """Resident bytes the server charges for each graph of specs."""
    d = lib()
    out = []
    for n, src, dst, _ in specs:
        S = d.Server(BIG, batched=batched)
        S.add_graph(d.Graph(src, dst, n, threshold=16, keep_plain_csr=True))
        out.append(S.stats()["used_bytes"])
        S.destroy()
    return out


@pytest.mark.parametrize("batched", [1, 0, 2])
def test_server_evicts_and_loads_graphs(inputs_mod, oracle_mod, batched):
    """A budget that holds one graph (plus a few rows) at a time: graphs added
    beyond it wait in host memory, idle graphs are evicted to make room, and
    every query of every graph still gets the oracle's depths."""
    d = lib()
    torch_cuda()
    # three RMAT scale-12 graphs of similar size (different seeds)
    specs = []
    for i in range(3):
        src, dst = inputs_mod.rmat_edges(12, seed=inputs_mod.graph_seed(12) + 100 + i)
        specs.append((1 << 12, src, dst, oracle_mod.Graph(src, dst, 1 << 12)))
    fp = _footprints(specs, batched)
    nmax = max(n for n, _, _, _ in specs)
    budget = max(fp) + 6 * 4 * nmax
    assert sorted(fp)[0] + sorted(fp)[1] > budget   # two graphs never fit together
    S = d.Server(budget, batched=batched)
    gids = [S.add_graph(d.Graph(s, t, n, threshold=16, keep_plain_csr=True))
            for n, s, t, _ in specs]
    st = S.stats()
    assert st["graphs"] == 3 and st["resident_graphs"] == 1, st
    rng = np.random.default_rng(11)
    for rnd in range(3):
        # one graph at a time: its queries are submitted, then collected (a
        # client that held results while waiting for another graph's query
        # could keep that graph from ever fitting)
        for k in rng.permutation(3).tolist():
            n, src, dst, O = specs[k]
            srcs = inputs_mod.pick_sources(src, dst, n, 3, seed=700 + 10 * rnd + k).tolist()
            ts = [S.submit(gids[k], s) for s in srcs]
            for s, t in zip(srcs, ts):
                row, qs = _fetch(S, t, n)
                np.testing.assert_array_equal(row, O.bfs(s, want_parent=False)[0],
                                              err_msg=f"round {rnd} graph {k} source {s}")
                assert qs["graph_id"] == gids[k]
        log(f"evict/load batched={batched} round {rnd}: {S.stats()}")
    st = S.stats()
    assert st["loads"] >= 4 and st["evictions"] >= 4, st
    assert st["resident_graphs"] == 1 and st["used_bytes"] <= budget, st
    assert st["queries_done"] == 3 * 3 * 3
    S.destroy()


def test_server_add_graph_while_serving(inputs_mod, oracle_mod):
    """Graphs added from another thread while queries of the first one run."""
    import threading
    d = lib()
    torch_cuda()
    specs = _graphs(inputs_mod, oracle_mod)
    S = d.Server(BIG, batched=2)
    gids = [S.add_graph(d.Graph(specs[0][1], specs[0][2], specs[0][0], threshold=16,
                                keep_plain_csr=True))]
    n0, src0, dst0, O0 = specs[0]
    stream_src = inputs_mod.pick_sources(src0, dst0, n0, 60, seed=41).tolist()
    tickets = []

    def client():
        for i, s in enumerate(stream_src):
            tickets.append((s, S.submit(gids[0], s)))
            if i % 10 == 9:
                time.sleep(0.001)

    th = threading.Thread(target=client)
    th.start()
    for n, s, t, _ in specs[1:]:   # added while the client's queries are being served
        gids.append(S.add_graph(d.Graph(s, t, n, threshold=16, keep_plain_csr=True)))
    late = []
    for k in (1, 2):
        n, src, dst, _ = specs[k]
        for s in inputs_mod.pick_sources(src, dst, n, 8, seed=50 + k).tolist():
            late.append((k, s, S.submit(gids[k], s)))
    th.join()
    for s, t in tickets:
        row, _ = _fetch(S, t, n0)
        np.testing.assert_array_equal(row, O0.bfs(s, want_parent=False)[0])
    for k, s, t in late:
        n, _, _, O = specs[k]
        row, _ = _fetch(S, t, n)
        np.testing.assert_array_equal(row, O.bfs(s, want_parent=False)[0])
    assert S.stats()["graphs"] == 3
    S.destroy()


def test_server_rows_from_allocator_and_budget_waits(inputs_mod, oracle_mod):
    """Result rows from PyTorch's caching allocator (called on the scheduler
    thread); with room for two rows, later queries wait for budget and are
    counted."""
    d = lib()
    torch = torch_cuda()
    specs = _graphs(inputs_mod, oracle_mod)[:1]
    n, src, dst, O = specs[0]
    fp = _footprints(specs, True)[0]
    alloc = d.default_allocator()
    S = d.Server(fp + 2 * 4 * n, batched=True, allocator=alloc)
    gid = S.add_graph(d.Graph(src, dst, n, threshold=16, keep_plain_csr=True))
    before = torch.cuda.memory_allocated()
    sources = inputs_mod.pick_sources(src, dst, n, 6, seed=8).tolist()
    ts = [S.submit(gid, s) for s in sources]
    p0, _ = S.wait(ts[0])
    p1, _ = S.wait(ts[1])
    assert torch.cuda.memory_allocated() >= before + 2 * 4 * n   # rows came from torch
    with pytest.raises(d.DsbfsError) as e:
        S.wait(ts[2], timeout_ns=100_000_000)
    assert e.value.status == d.ERR_NOT_READY
    waited = []
    for s, t in zip(sources, ts):
        row, qs = _fetch(S, t, n)
        np.testing.assert_array_equal(row, O.bfs(s, want_parent=False)[0])
        waited.append(qs["waited_budget"])
    assert waited[:2] == [0, 0] and sum(waited) >= 1
    st = S.stats()
    assert st["budget_waits"] == sum(waited) and st["queries_done"] == 6
    S.destroy()


@pytest.mark.parametrize("batched", [1, 2])
def test_server_budget_serves_oldest_first(inputs_mod, oracle_mod, batched):
    """When the budget binds, a waiting query keeps its place: with two large
    results held, a large-graph query X waits for room, and later queries on
    a small graph, whose rows would fit the room left, are not admitted
    before X (they would otherwise take every release and starve it). All
    rows equal the oracle's."""
    d = lib()
    specs = _graphs(inputs_mod, oracle_mod)
    small, large = specs[0], specs[1]            # RMAT 10 and RMAT 12
    fps = _footprints([small, large], batched)
    nl, ns = large[0], small[0]
    S = d.Server(sum(fps) + 2 * 4 * nl + 2 * 4 * ns, batched=batched)
    gs = S.add_graph(d.Graph(small[1], small[2], ns, threshold=16, keep_plain_csr=True))
    gl = S.add_graph(d.Graph(large[1], large[2], nl, threshold=16, keep_plain_csr=True))
    srcl = inputs_mod.pick_sources(large[1], large[2], nl, 3, seed=12).tolist()
    srcs = inputs_mod.pick_sources(small[1], small[2], ns, 4, seed=13).tolist()
    held = [S.submit(gl, s) for s in srcl[:2]]
    for t in held:
        S.wait(t)                                # done, rows still held
    x = S.submit(gl, srcl[2])
    ys = [S.submit(gs, s) for s in srcs]
    time.sleep(0.05)                             # room for the small rows, none for X's
    with pytest.raises(d.DsbfsError) as e:
        S.wait(x, timeout_ns=1_000_000)
    assert e.value.status == d.ERR_NOT_READY
    for t, s in zip(held, srcl[:2]):
        row, _ = _fetch(S, t, nl)
        np.testing.assert_array_equal(row, large[3].bfs(s, want_parent=False)[0])
    row, qx = _fetch(S, x, nl)
    np.testing.assert_array_equal(row, large[3].bfs(srcl[2], want_parent=False)[0])
    assert qx["waited_budget"] == 1
    for t, s in zip(ys, srcs):
        row, qy = _fetch(S, t, ns)
        np.testing.assert_array_equal(row, small[3].bfs(s, want_parent=False)[0])
        assert qy["admit_ns"] >= qx["admit_ns"], "a later query was admitted before the waiting one"
    S.destroy()
