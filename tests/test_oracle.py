"""Pins of the CPU oracle against things other than itself: closed forms,
brute-force all-pairs shortest paths, hand-derived values from the paper's
definitions, and a textbook identity. None of these needs a GPU."""
import os

import numpy as np
import pytest

from closed_forms import all_closed_forms, complete, cycle, grid, path, star

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _graph(oracle_mod, n, src, dst):
    return oracle_mod.Graph(src, dst, n)


@pytest.mark.parametrize("case", all_closed_forms(), ids=lambda c: c[0])
def test_closed_form_depths(oracle_mod, case):
    name, n, src, dst, dist, sources = case
    G = _graph(oracle_mod, n, src, dst)
    label = G.components()
    for s in sources:
        depth, parent = G.bfs(s)
        np.testing.assert_array_equal(depth, dist(s), err_msg=f"{name} s={s}")
        assert G.check(s, depth, parent, label) == (0, -1)


def test_apsp_matches_closed_forms(oracle_mod):
    for n, src, dst, dist in (path(30), cycle(31), grid(5, 7), complete(9)):
        D = oracle_mod.apsp(n, src, dst)
        for s in range(n):
            np.testing.assert_array_equal(D[s], dist(s))


def _random_pairs(rng, n, k, loops=True):
    src = rng.integers(0, n, size=k).astype(np.int32)
    dst = rng.integers(0, n, size=k).astype(np.int32)
    if loops:
        src[: k // 20] = dst[: k // 20]          # some self-loops
    dup = rng.integers(0, k, size=k // 10)
    src = np.concatenate([src, dst[dup]])      # some reversed duplicates
    dst = np.concatenate([dst, src[dup]])
    return src, dst


@pytest.mark.parametrize("n,k,seed", [(60, 40, 1), (100, 150, 2), (128, 400, 3), (90, 900, 4)])
def test_bfs_equals_brute_force_random(oracle_mod, n, k, seed):
    rng = np.random.default_rng(seed)
    src, dst = _random_pairs(rng, n, k)
    D = oracle_mod.apsp(n, src, dst)
    G = _graph(oracle_mod, n, src, dst)
    label = G.components()
    for s in range(n):
        depth, parent = G.bfs(s)
        np.testing.assert_array_equal(depth, D[s])
        assert G.check(s, depth, parent, label)[0] == 0


@pytest.mark.parametrize("scale", [5, 6, 7])
def test_bfs_equals_brute_force_tiny_rmat(oracle_mod, inputs_mod, scale):
    src, dst = inputs_mod.rmat_edges(scale)
    n = 1 << scale
    D = oracle_mod.apsp(n, src, dst)
    G = _graph(oracle_mod, n, src, dst)
    for s in range(0, n, 3):
        depth, _ = G.bfs(s, want_parent=False)
        np.testing.assert_array_equal(depth, D[s])


def test_csr_is_the_simple_symmetric_graph(oracle_mod):
    rng = np.random.default_rng(7)
    n = 70
    src, dst = _random_pairs(rng, n, 500)
    G = _graph(oracle_mod, n, src, dst)
    adj = [set() for _ in range(n)]
    for u, v in zip(src.tolist(), dst.tolist()):
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    off, col = G.off, G.col
    assert G.m == sum(len(a) for a in adj)
    for v in range(n):
        assert col[off[v]:off[v + 1]].tolist() == sorted(adj[v])


def test_csr_rejects_out_of_range(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.Graph(np.array([0, 5], np.int32), np.array([1, 1], np.int32), 5)


def test_components_closed_form(oracle_mod):
    from closed_forms import disjoint_paths
    n, src, dst, _ = disjoint_paths(6, 4)
    lab = _graph(oracle_mod, n, src, dst).components()
    assert lab.tolist() == [0] * 6 + [6] * 4


def test_checker_flags_planted_mistakes(oracle_mod):
    """Every invariant fires on a result broken in the way it guards against."""
    n, src, dst, dist = grid(6, 6)
    G = _graph(oracle_mod, n, src, dst)
    label = G.components()
    depth, parent = G.bfs(0)
    assert G.check(0, depth, parent, label)[0] == 0

    d, p = depth.copy(), parent.copy()
    p[0] = 1                                     # source is not its own parent
    assert G.check(0, d, p, label)[0] == 1

    d, p = depth.copy(), parent.copy()
    p[35] = 0                                    # parent that is not a neighbour
    assert G.check(0, d, p, label) == (2, 35)

    d, p = depth.copy(), parent.copy()
    d[35] += 2                                   # depth off by two: parent level wrong
    assert G.check(0, d, p, label)[0] == 2

    d = depth.copy()
    d[35] += 2                                   # same, without parents: edge rule fires
    assert G.check(0, d, None, label)[0] == 3

    n2, s2, t2, _ = path(5)
    src2 = np.concatenate([s2, [5]]).astype(np.int32)   # edge 5-6: a second component
    dst2 = np.concatenate([t2, [6]]).astype(np.int32)
    G2 = _graph(oracle_mod, 7, src2, dst2)
    lab2 = G2.components()
    d2, p2 = G2.bfs(0)
    assert G2.check(0, d2, p2, lab2)[0] == 0
    d2b = d2.copy()
    d2b[5], d2b[6] = 9, 10                      # reached outside the component
    assert G2.check(0, d2b, None, lab2)[0] == 4
    d2c = d2.copy()
    d2c[6] = -3
    assert G2.check(0, d2c, None, None)[0] == 5


def test_split_star(oracle_mod):
    k = 20
    n, src, dst, _ = star(k)
    G = _graph(oracle_mod, n, src, dst)
    for TH in (1, 5, 19):
        st = G.split_stats(TH)
        assert st["d"] == 1
        assert (st["e_nn"], st["e_nd"], st["e_dn"], st["e_dd"]) == (0, k, k, 0)
        assert (st["n_ndsrc"], st["n_ddsrc"], st["n_dnsrc"]) == (k, 0, 1)
    st = G.split_stats(k)                       # strict '>': degree == TH stays normal
    assert st["d"] == 0 and st["e_nn"] == 2 * k


def test_split_threshold_edge_cases(oracle_mod, inputs_mod):
    src, dst = inputs_mod.rmat_edges(9)
    G = _graph(oracle_mod, 512, src, dst)
    deg = G.degrees()
    st = G.split_stats(int(deg.max()))
    assert st["d"] == 0 and st["e_nn"] == G.m and st["e_nd"] == st["e_dn"] == st["e_dd"] == 0
    st = G.split_stats(0)                       # every non-isolated vertex is a delegate
    assert st["d"] == int((deg > 0).sum())
    assert st["e_nn"] == st["e_nd"] == st["e_dn"] == 0 and st["e_dd"] == G.m
    n, s, t, _ = complete(8)
    st = _graph(oracle_mod, n, s, t).split_stats(6)
    assert st["d"] == 8 and st["e_dd"] == 56


def test_split_path_th1(oracle_mod):
    # path 0-1-2-3-4: interior vertices have degree 2 > 1 -> delegates 0,1,2
    n, src, dst, _ = path(5)
    G = _graph(oracle_mod, n, src, dst)
    r = G.split_rows(1)
    assert r["did"].tolist() == [-1, 0, 1, 2, -1]
    assert r["nd_col"].tolist() == [0, 2]       # 0->1 (delegate 0), 4->3 (delegate 2)
    assert r["nd_off"].tolist() == [0, 1, 1, 1, 1, 2]
    assert r["dn_off"].tolist() == [0, 1, 1, 2] and r["dn_col"].tolist() == [0, 4]
    assert r["dd_off"].tolist() == [0, 1, 3, 4] and r["dd_col"].tolist() == [1, 0, 2, 1]
    assert r["nn_col"].size == 0


def _csr_to_pairs(off, col):
    rows = np.repeat(np.arange(len(off) - 1), np.diff(off))
    return set(zip(rows.tolist(), col.tolist()))


@pytest.mark.parametrize("TH", [0, 2, 8, 16, 32, 10**6])
def test_split_identities_rmat(oracle_mod, inputs_mod, TH):
    src, dst = inputs_mod.rmat_edges(10)
    G = _graph(oracle_mod, 1024, src, dst)
    st = G.split_stats(TH)
    r = G.split_rows(TH)
    assert st["e_nn"] + st["e_nd"] + st["e_dn"] + st["e_dd"] == G.m
    assert st["e_nd"] == st["e_dn"]
    assert st["d"] == int((G.degrees() > TH).sum())
    dd = _csr_to_pairs(r["dd_off"], r["dd_col"])
    assert dd == {(b, a) for a, b in dd}                     # dd symmetric
    nd = _csr_to_pairs(r["nd_off"], r["nd_col"])             # (normal, delegate id)
    dn = _csr_to_pairs(r["dn_off"], r["dn_col"])             # (delegate id, normal)
    assert nd == {(b, a) for a, b in dn}                     # nd is dn reversed
    nn = _csr_to_pairs(r["nn_off"], r["nn_col"])
    assert nn == {(b, a) for a, b in nn}                     # nn symmetric at one GPU


def test_fig2_renumbering(oracle_mod):
    """Fig. 2 caption: TH = 5, vertices 7 and 8 become delegates 0 and 1."""
    fix = {}
    with open(os.path.join(GOLD, "fig2_renumbering.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            if t[0] == "threshold":
                TH = int(t[1])
            else:
                fix[int(t[1])] = int(t[2])
    # a graph on 0..12 in which only 7 and 8 have degree > 5 (7: 6, 8: 7)
    pairs = [(7, x) for x in (0, 1, 2, 3, 4, 8)] + [(8, x) for x in (5, 6, 9, 10, 11, 12)]
    pairs += [(0, 1), (2, 3)]
    src = np.array([a for a, _ in pairs], np.int32)
    dst = np.array([b for _, b in pairs], np.int32)
    G = _graph(oracle_mod, 13, src, dst)
    assert (G.degrees() > TH).sum() == len(fix)
    did = G.delegate_ids(TH)
    for v, want in fix.items():
        assert did[v] == want
    assert (did[[v for v in range(13) if v not in fix]] == -1).all()


def test_bv_closed_form_is_geometric_sum(oracle_mod):
    for a in (1e-3, 0.01, 0.1, 0.37, 0.5, 0.9, 1.0):
        for k in (1, 2, 3, 7, 16, 33, 64):
            direct = sum((1 - a) ** i for i in range(k))
            assert oracle_mod.bv_term(a, k) == pytest.approx(direct, rel=1e-12)
            # the first line of the printed equation sums to exactly 1 for every
            # od, which is why it is read as garbled (see the reading list)
            printed = (1 - a) ** k + sum(a * (1 - a) ** i for i in range(k))
            assert printed == pytest.approx(1.0, rel=1e-12)
    # large od: the term tends to 1/a, so sum over U tends to |U|/a = |U|(q+s)/q
    assert oracle_mod.bv_term(0.25, 10**6) == pytest.approx(4.0)
    assert oracle_mod.bv_approx(10, 2, 6) == pytest.approx(10 * 8 / 2)
    assert oracle_mod.bv_approx(0, 2, 6) == 0.0 and oracle_mod.bv_approx(5, 0, 6) == 0.0


def _factors():
    f0, f1 = {}, {}
    with open(os.path.join(GOLD, "do_factors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, k, v = line.split()
            (f0 if kind == "factor0" else f1)[k] = float(v)
    order = ("dd", "dn", "nd")
    return tuple(f0[k] for k in order), tuple(f1[k] for k in order)


def test_do_replay_star_hand_derived(oracle_mod):
    """Star with hub 0 (the only delegate) and k leaves, searched from leaf 1.
    Level 0: frontier {1}: nd has q=1, FV=1, U = {hub}, s = k-1 unvisited
    leaves, BV = 1*(1+k-1)/1 = k; FV = 1 > 1e-7*k so nd goes backward.
    Level 1: frontier {hub}: dn has q=1, FV=k, U = k-1 leaves, s = 0, BV = k-1;
    k > 0.05(k-1) so dn goes backward. nd has no frontier and stays backward.
    Level 2: frontier = k-1 leaves: nd q=k-1, FV=k-1, U = {}, BV = 0."""
    k = 12
    n, src, dst, _ = star(k)
    G = _graph(oracle_mod, n, src, dst)
    f0, f1 = _factors()
    depth, _ = G.bfs(1)
    L = G.do_replay(2, depth, f0, f1)
    assert len(L) == 3
    assert L[0]["q"] == [0, 0, 1] and L[0]["FV"] == [0, 0, 1]
    assert L[0]["U"] == [0, k - 1, 1] and L[0]["s"] == [0, 1, k - 1]
    assert L[0]["BV"][2] == pytest.approx(k) and L[0]["dir"] == [0, 0, 1]
    assert L[1]["q"] == [0, 1, 0] and L[1]["FV"] == [0, k, 0]
    assert L[1]["U"] == [0, k - 1, 0] and L[1]["s"] == [0, 0, k - 1]
    assert L[1]["BV"][1] == pytest.approx(k - 1) and L[1]["dir"] == [0, 1, 1]
    assert L[2]["q"] == [0, 0, k - 1] and L[2]["FV"] == [0, 0, k - 1]
    assert L[2]["U"] == [0, 0, 0] and L[2]["BV"] == [0.0, 0.0, 0.0]
    assert L[2]["dir"] == [0, 1, 1]
    assert [x["frontier_normal"] for x in L] == [1, 0, k - 1]
    assert [x["frontier_delegate"] for x in L] == [0, 1, 0]


def test_do_replay_two_hubs_strict_comparison(oracle_mod):
    """Hubs A=0 and B=1 joined, each with k leaves; TH=2, source A.
    Level 0: dd: q=1, FV=1, U={B}, s=1 -> BV = 1*(1+1)/1 = 2 and
    FV = 1 is not > 0.5*2 = 1, so dd stays forward (strict comparison).
    dn: q=1, FV=k, U = all 2k leaves, s = |{B}| = 1 -> BV = 2k*(1+1)/1 = 4k,
    and FV = k > 0.05*4k = 0.2k, so dn goes backward."""
    k = 10
    pairs = [(0, 1)] + [(0, 2 + i) for i in range(k)] + [(1, 2 + k + i) for i in range(k)]
    src = np.array([a for a, _ in pairs], np.int32)
    dst = np.array([b for _, b in pairs], np.int32)
    G = _graph(oracle_mod, 2 + 2 * k, src, dst)
    f0, f1 = _factors()
    depth, _ = G.bfs(0)
    L = G.do_replay(2, depth, f0, f1)
    assert L[0]["q"][:2] == [1, 1] and L[0]["FV"][:2] == [1, k]
    assert L[0]["U"][:2] == [1, 2 * k] and L[0]["s"][:2] == [1, 1]
    assert L[0]["BV"][0] == pytest.approx(2.0) and L[0]["BV"][1] == pytest.approx(4 * k)
    assert L[0]["dir"] == [0, 1, 0]
    # factor1 > FV/BV at a backward kernel switches it back to forward
    L2 = G.do_replay(2, depth, f0, (0.0, 10.0, 0.0))
    assert L2[0]["dir"][1] == 1
    assert L2[1]["dir"][1] == (0 if L2[1]["q"][1] > 0 else 1)


def _table1_total(p, n, d, e_nn, e_nd, e_dn, e_dd):
    """Sum of Table I's per-subgraph rows over p GPUs: offsets n/p*4 (nn),
    n/p*4 (nd), d*4 (dn), d*4 (dd); columns |E_nn|/p*8, |E_nd|/p*4,
    |E_dn|/p*4, |E_dd|/p*4."""
    per_gpu = (n / p * 4 + e_nn / p * 8) + (n / p * 4 + e_nd / p * 4) \
        + (d * 4 + e_dn / p * 4) + (d * 4 + e_dd / p * 4)
    return per_gpu * p


def test_table1_memory_of_split_graphs(oracle_mod):
    """Table I at p = 1 applied to the oracle's split of small graphs whose
    four edge classes are counted by hand (fixture table1_graphs.txt)."""
    k = 12
    graphs = {}
    n, s, t, _ = star(k)
    graphs["star12"] = (n, s, t)
    pairs = [(0, 1)] + [(0, 2 + i) for i in range(10)] + [(1, 12 + i) for i in range(10)]
    graphs["two_hubs10"] = (22, np.array([a for a, _ in pairs], np.int32),
                            np.array([b for _, b in pairs], np.int32))
    n, s, t, _ = complete(4)
    graphs["k4"] = (n, s, t)
    n, s, t, _ = path(5)
    graphs["path5"] = (n, s, t)
    with open(os.path.join(GOLD, "table1_graphs.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 4
    for name, TH, d, e_nn, e_nd, e_dn, e_dd, want in rows:
        n, s, t = graphs[name]
        st = _graph(oracle_mod, n, s, t).split_stats(int(TH))
        got = (st["d"], st["e_nn"], st["e_nd"], st["e_dn"], st["e_dd"])
        assert got == tuple(int(x) for x in (d, e_nn, e_nd, e_dn, e_dd)), name
        assert _table1_total(1, n, st["d"], st["e_nn"], st["e_nd"], st["e_dn"],
                             st["e_dd"]) == int(want), name


def _expected_checks_brute(a, od):
    """Expected number of potential parents a bottom-up scan checks, stopping
    at the first one in the frontier, when each of od potential parents is in
    the frontier independently with probability a: enumerates every frontier
    subset (no closed form)."""
    total = 0.0
    for mask in range(1 << od):
        pr = 1.0
        for i in range(od):
            pr *= a if (mask >> i) & 1 else (1 - a)
        checks = od
        for i in range(od):
            if (mask >> i) & 1:
                checks = i + 1
                break
        total += pr * checks
    return total


def test_do_replay_exact_bv_star_brute_force(oracle_mod):
    """Exact BV (Section IV-B's expected checks summed over U) on the star of
    test_do_replay_star_hand_derived: level 0, nd kernel, U = {hub}, whose
    reversed-subgraph degree is k (its dn edges) and a = q/(q+s) = 1/k; level
    1, dn kernel, U = the k-1 unvisited leaves, each with one delegate
    neighbour, a = 1/(1+0) = 1. Each term is checked against the brute-force
    expectation over frontier subsets."""
    k = 12
    n, src, dst, _ = star(k)
    G = _graph(oracle_mod, n, src, dst)
    f0, f1 = _factors()
    depth, _ = G.bfs(1)
    L = G.do_replay(2, depth, f0, f1, bv_exact=True)
    assert len(L) == 3
    assert L[0]["BV"][2] == pytest.approx(_expected_checks_brute(1.0 / k, k), rel=1e-12)
    assert L[0]["BV"][0] == 0.0 and L[0]["BV"][1] == 0.0      # q = 0: not evaluated
    assert L[1]["BV"][1] == pytest.approx((k - 1) * _expected_checks_brute(1.0, 1), rel=1e-12)
    assert L[2]["BV"] == [0.0, 0.0, 0.0]                     # U empty
    assert [x["dir"] for x in L] == [[0, 0, 1], [0, 1, 1], [0, 1, 1]]


def test_do_replay_exact_bv_changes_the_decision(oracle_mod):
    """Two hubs A=0, B=1 joined, each with k leaves, TH=2, source A. With the
    exact sum, level 0's dd term is U = {B} with one dd edge and a = 1/2: one
    check, BV_dd = 1, so FV_dd = 1 > 0.5*1 and dd goes backward, where the
    paper's approximation (BV_dd = 2) keeps it forward. dn: U = the 2k
    leaves, one delegate each: BV_dn = 2k (approximation 4k)."""
    k = 10
    pairs = [(0, 1)] + [(0, 2 + i) for i in range(k)] + [(1, 2 + k + i) for i in range(k)]
    src = np.array([a for a, _ in pairs], np.int32)
    dst = np.array([b for _, b in pairs], np.int32)
    G = _graph(oracle_mod, 2 + 2 * k, src, dst)
    f0, f1 = _factors()
    depth, _ = G.bfs(0)
    ex = G.do_replay(2, depth, f0, f1, bv_exact=True)
    ap = G.do_replay(2, depth, f0, f1, bv_exact=False)
    assert ex[0]["BV"][0] == pytest.approx(_expected_checks_brute(0.5, 1))
    assert ex[0]["BV"][1] == pytest.approx(2 * k * _expected_checks_brute(0.5, 1))
    assert ap[0]["BV"][:2] == [pytest.approx(2.0), pytest.approx(4.0 * k)]
    assert ex[0]["dir"][0] == 1 and ap[0]["dir"][0] == 0
    # level 1: nd frontier = A's k leaves, a = k/(k+k); U = unvisited delegates
    # with dn edges = {} (B is visited) -> 0
    assert ex[1]["q"][2] == k and ex[1]["s"][2] == k and ex[1]["BV"][2] == 0.0


def test_do_replay_exact_bv_two_delegate_neighbours(oracle_mod):
    """Hubs 0, 1, 2 (degree > TH = 2); normals 3..8 adjacent to hubs 0 and 1,
    normals 9..11 to hub 2, and the dd edge 0-2; source hub 0. Level 0, dn:
    q = 1, s = |{1, 2}| = 2 (delegates with dn edges, unvisited), a = 1/3;
    U = normals 3..11: six with two delegate neighbours, three with one.
    BV_dn = 6 E(1/3, 2) + 3 E(1/3, 1). dd: q = 1, s = |{2}| = 1, a = 1/2,
    U = {2} with one dd edge: BV_dd = E(1/2, 1)."""
    pairs = [(h, v) for v in range(3, 9) for h in (0, 1)] + [(2, v) for v in (9, 10, 11)]
    pairs += [(0, 2)]
    src = np.array([a for a, _ in pairs], np.int32)
    dst = np.array([b for _, b in pairs], np.int32)
    G = _graph(oracle_mod, 12, src, dst)
    assert G.split_stats(2)["d"] == 3
    depth, _ = G.bfs(0)
    L = G.do_replay(2, depth, (10.0, 10.0, 10.0), (0.0, 0.0, 0.0), bv_exact=True)
    want_dn = 6 * _expected_checks_brute(1 / 3, 2) + 3 * _expected_checks_brute(1 / 3, 1)
    assert L[0]["q"][:2] == [1, 1] and L[0]["s"][:2] == [1, 2]
    assert L[0]["BV"][1] == pytest.approx(want_dn, rel=1e-12)
    assert L[0]["BV"][0] == pytest.approx(_expected_checks_brute(0.5, 1), rel=1e-12)


# ---------------------------------------------------------------------------
# Work model (algorithmic bytes of a search)
# ---------------------------------------------------------------------------

def _pairs(n, pairs):
    return (n, np.array([a for a, _ in pairs], np.int32), np.array([b for _, b in pairs], np.int32))


def test_work_model_star_hand_derived(oracle_mod):
    """Star, hub 0 (the only delegate at TH = 2) and k = 12 leaves, from leaf
    1, the paper's factors (schedule as in test_do_replay_star_hand_derived).
    Level 0: nd backward: one candidate (the hub), whose dn part is its
    leaves ascending, so the scan stops at leaf 1, the first entry; mask bytes
    2 * ceil(1/8). Level 1: dn backward: the other 11 leaves, one entry each,
    all reached; candidate-set bytes 4 * 12 + ceil(13/8). Bytes: frontier
    normals 16 * (1 + 11); delegate previsit 16; dn backward
    16*11 + 4*11 + 50 + 8*11; delegate backward 16 + 4 + 2 + 8."""
    k = 12
    n, src, dst, _ = star(k)
    G = _graph(oracle_mod, n, src, dst)
    f0, f1 = _factors()
    depth, _ = G.bfs(1)
    L, B, runs = oracle_mod.WorkModel(G, 2).run(depth, f0, f1)
    assert len(L) == 3
    assert (L[0]["c_deleg"], L[0]["c_nd"], L[0]["e_bu_nd"], L[0]["s_nd"], L[0]["cl_bu_deleg"]) == \
        (1, 1, 1, 2, 1)
    assert (L[1]["c_dn"], L[1]["e_bu_dn"], L[1]["s_dn"], L[1]["cl_bu_dn"]) == (11, 11, 50, 11)
    assert L[2]["runs"] == [0, 0, 0, 0, 0] and L[2]["f_norm"] == 11
    assert B == {"init": 8.0, "normal_frontier": 192.0, "delegate_previsit": 16.0,
                 "nd_forward": 0.0, "deleg_forward": 0.0, "dn_backward": 358.0,
                 "deleg_backward": 30.0}
    assert runs["dn_backward"] == 1 and runs["deleg_backward"] == 1
    # without parents the output costs 4 bytes per vertex
    _, B4, _ = oracle_mod.WorkModel(G, 2).run(depth, f0, f1, want_parent=False)
    assert B4["dn_backward"] == 358.0 - 4 * 11 and B4["deleg_backward"] == 30.0 - 4


def test_work_model_stored_order_hand_derived(oracle_mod):
    """Delegates A=0, B=1, C=2 (degrees 4, 5, 6 > TH = 3) share the normal
    neighbour x=3 (degree 3); A has leaves 4..6, B 7..10, C 11..15. From A
    with the paper's factors:
    level 0: dn: q=1, FV=4, U = 13 normals with a delegate neighbour, s = 2
    (B, C): BV = 39 and 4 > 0.05*39, backward. The candidates are the 13
    normals. x's nd part is stored by decreasing degree (C, B, A), so its scan
    reads 3 entries before it finds A (1 in ascending order); A's leaves read
    1 entry each and are reached, B's and C's leaves read 1 each and miss:
    15 entries, 4 reached, 4*13 + 2 candidate-set bytes.
    level 1: frontier x and A's leaves (normals): nd: q=4, FV=6, U={B, C},
    s=9: BV = 6.5, backward: B's and C's dn parts are ascending and start
    with x: 1 entry each, both reached.
    level 2: frontier B, C: dn stays backward: the 9 leaves of B and C, one
    entry each, all reached. level 3: nd has no unvisited candidate."""
    pairs = [(0, 3), (1, 3), (2, 3)] + [(0, v) for v in (4, 5, 6)] + \
        [(1, v) for v in (7, 8, 9, 10)] + [(2, v) for v in (11, 12, 13, 14, 15)]
    n, src, dst = _pairs(16, pairs)
    G = _graph(oracle_mod, n, src, dst)
    assert G.split_stats(3)["d"] == 3
    f0, f1 = _factors()
    depth, _ = G.bfs(0)
    L, B, _ = oracle_mod.WorkModel(G, 3).run(depth, f0, f1)
    assert len(L) == 4
    assert L[0]["dir"][1] == 1 and L[0]["BV"][1] == pytest.approx(39.0)
    assert (L[0]["c_dn"], L[0]["e_bu_dn"], L[0]["cl_bu_dn"], L[0]["s_dn"]) == (13, 15, 4, 54)
    assert L[1]["dir"][2] == 1 and L[1]["BV"][2] == pytest.approx(6.5)
    assert (L[1]["c_deleg"], L[1]["c_nd"], L[1]["e_bu_nd"], L[1]["cl_bu_deleg"]) == (2, 2, 2, 2)
    assert (L[2]["c_dn"], L[2]["e_bu_dn"], L[2]["cl_bu_dn"]) == (9, 9, 9)
    assert L[3]["runs"] == [0, 0, 0, 0, 0]
    assert B["dn_backward"] == 16 * 13 + 4 * 15 + 54 + 8 * 4 + 16 * 9 + 4 * 9 + 54 + 8 * 9
    assert B["deleg_backward"] == 16 * 2 + 4 * 2 + 2 + 8 * 2


def _reach_invariants(L, depth):
    """Every vertex at depth l + 1 is first reached exactly once, at level l."""
    for lv, r in enumerate(L):
        got = r["cl_nn"] + r["cl_nd"] + r["cl_dd"] + r["cl_dn"] + r["cl_bu_dn"] + r["cl_bu_deleg"]
        assert got == int((depth == lv + 1).sum()), lv


@pytest.mark.parametrize("TH", [0, 2, 8, 32, 10 ** 6])
def test_work_model_all_forward_closed_form(oracle_mod, inputs_mod, TH):
    """With factor0 = inf no kernel leaves the forward direction: every
    reached vertex's row is expanded once, so the forward edges sum to the
    component's directed edge count (sum of its degrees), the frontier
    vertices with an edge are the reached vertices of positive degree, and
    no backward work is done."""
    src, dst = inputs_mod.rmat_edges(10)
    n = 1 << 10
    G = _graph(oracle_mod, n, src, dst)
    deg = G.degrees()
    W = oracle_mod.WorkModel(G, TH)
    inf = float("inf")
    for s in inputs_mod.pick_sources(src, dst, n, 4, seed=5).tolist():
        depth, _ = G.bfs(s)
        L, B, _ = W.run(depth, (inf, inf, inf), (0.0, 0.0, 0.0))
        reached = depth >= 0
        assert sum(r["e_nn"] + r["e_nd"] + r["e_dd"] + r["e_dn"] for r in L) == deg[reached].sum()
        assert sum(r["f_norm"] + r["f_deleg"] for r in L) == int((reached & (deg > 0)).sum())
        for r in L:
            assert r["c_dn"] == r["c_deleg"] == r["e_bu_dn"] == r["e_bu_dd"] == r["e_bu_nd"] == 0
            assert r["s_dn"] == r["s_dd"] == r["s_nd"] == 0
        _reach_invariants(L, depth)
        assert B["init"] == 8 * (int((~reached).sum()) + 1)   # unreached + the source
        total = sum(B.values())
        assert total == 16 * int((reached & (deg > 0)).sum()) + 4 * deg[reached].sum() + 8 * n


@pytest.mark.parametrize("scale,TH", [(10, 4), (12, 16), (12, 64)])
def test_work_model_schedule_equals_replay(oracle_mod, inputs_mod, scale, TH):
    """The work model's schedule (summed from per-depth histograms) equals the
    level-by-level replay of Section IV-B (pinned above by hand-derived
    cases) under several factor pairs; every vertex is reached once; a
    backward scan never reads more entries than its candidates' rows hold
    and at least one per candidate."""
    src, dst = inputs_mod.rmat_edges(scale)
    n = 1 << scale
    G = _graph(oracle_mod, n, src, dst)
    W = oracle_mod.WorkModel(G, TH)
    r = G.split_rows(TH)
    nd_len = np.diff(r["nd_off"])
    for f0, f1 in (((0.5, 0.05, 1e-7), (0.0, 0.0, 0.0)), ((0.02, 0.001, 1e-6), (0.0, 0.0, 0.0)),
                   ((1e-3, 1e-3, 1e-3), (0.2, 0.5, 2.0)), ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))):
        for s in inputs_mod.pick_sources(src, dst, n, 3, seed=40 + scale).tolist():
            depth, _ = G.bfs(s)
            L, _, _ = W.run(depth, f0, f1)
            rep = G.do_replay(TH, depth, f0, f1)
            assert len(L) == len(rep)
            for a, b in zip(L, rep):
                for k in ("q", "s", "U", "FV", "BV", "dir"):
                    assert a[k] == b[k], (k, a[k], b[k])
            _reach_invariants(L, depth)
            for lv, a in enumerate(L):
                if a["c_dn"]:
                    unvis = (depth < 0) | (depth > lv)
                    cap = int(nd_len[unvis].sum())
                    assert a["c_dn"] <= a["e_bu_dn"] <= cap


# ---------------------------------------------------------------------------
# Work model of bit-parallel multi-source BFS
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k,permille", [(5, 0), (64, 2), (100, 50), (256, 1000), (200, 10)])
def test_ms_work_lanes_equal_single_source(oracle_mod, inputs_mod, k, permille):
    """Every lane of the simulated batch (1, 2 or 4 words of lanes) has the
    depths of a single-source search from its source, whatever the mix of
    top-down and bottom-up levels."""
    src, dst = inputs_mod.rmat_edges(10)
    n = 1 << 10
    G = _graph(oracle_mod, n, src, dst)
    rng = np.random.default_rng(k)
    sources = rng.integers(0, n, size=k).astype(np.int32)   # repeats allowed
    levels, _, depth = G.ms_work(sources, permille, want_depth=True)
    for i, s in enumerate(sources.tolist()):
        np.testing.assert_array_equal(depth[i], G.bfs(s, want_parent=False)[0], err_msg=str(i))
    assert len(levels) == int(depth.max()) + 1


def test_ms_work_top_down_closed_form(oracle_mod, inputs_mod):
    """All levels top-down (permille 1000): vertex v is active once per
    distinct depth it has over the lanes, and each time its whole row is
    read, so E = sum over v of deg(v) * #distinct depths and V = sum of
    #distinct depths; bytes = 4 k n + 4 E + 8 W E + 24 W V + 16 V."""
    src, dst = inputs_mod.rmat_edges(9)
    n = 1 << 9
    G = _graph(oracle_mod, n, src, dst)
    deg = G.degrees()
    for k in (3, 64, 130):
        sources = inputs_mod.pick_sources(src, dst, n, k, seed=k)
        D = np.stack([G.bfs(int(s), want_parent=False)[0] for s in sources])
        distinct = np.array([len(set(D[:, v][D[:, v] >= 0].tolist())) for v in range(n)])
        levels, b, _ = G.ms_work(sources, 1000)
        E = sum(x["e"] for x in levels)
        V = sum(x["v"] for x in levels)
        assert not any(x["bottom_up"] for x in levels)
        assert E == int((deg * distinct).sum()) and V == int(distinct.sum())
        W = (k + 63) // 64
        assert b == 4 * k * n + 4 * E + 8 * W * E + 24 * W * V + 16 * V


def test_ms_work_bottom_up_path_hand_derived(oracle_mod):
    """Path 0-1-...-(n-1), one lane from 0, every level bottom-up
    (permille 0). Rows are stored by decreasing degree bucket, so vertex 1
    reads 2 (degree 2) before 0 (degree 1). Level 0: vertex 1 reads 2
    entries and finds 0; 2..n-2 read both entries and miss; n-1 reads its
    one entry: E = 2n - 3, V = n - 1. Level L in 1..n-3: L+1 finds L at once,
    L+2..n-2 read 2 each, n-1 reads 1: E = 2n - 4 - 2L, V = n - 1 - L.
    Level n-2: only n-1 is unseen and finds n-2: E = V = 1. Level n-1: the
    frontier is n-1 and nothing is unseen: E = V = 0."""
    n = 12
    _, src, dst, _ = path(n)
    G = _graph(oracle_mod, n, src, dst)
    levels, b, depth = G.ms_work(np.array([0], np.int32), 0, want_depth=True)
    assert depth[0].tolist() == list(range(n))
    want = [(2 * n - 3, n - 1)] + [(2 * n - 4 - 2 * L, n - 1 - L) for L in range(1, n - 2)] + \
        [(1, 1), (0, 0)]
    assert [(x["e"], x["v"]) for x in levels] == want
    assert all(x["bottom_up"] == 1 for x in levels) and [x["active"] for x in levels] == [1] * n
    E = sum(e for e, _ in want)
    V = sum(v for _, v in want)
    assert b == 4 * n + 4 * E + 8 * E + 24 * V + 16 * V


# ---------------------------------------------------------------------------
# Direction decision with nn included (the DO-on-nn variant)
# ---------------------------------------------------------------------------

def test_do_replay4_path_nn_hand_derived(oracle_mod):
    """Path 0-1-...-9 at TH = 5 (every vertex normal, every edge nn), from 0,
    nn factors 0.02 forward->backward and 0.5 backward->forward.
    Level 0: q=1, FV=1, U = the 9 unvisited vertices (all have nn edges),
    s = 9: BV = 9*(1+9)/1 = 90; 1 > 0.02*90 = 1.8 is false: forward.
    Level 1: frontier {1}: FV=2, U = s = 8: BV = 72; 2 > 1.44: backward.
    Level 2: frontier {2}: FV=2, U = s = 7: BV = 56; 2 < 0.5*56: forward
    again. The other kernels have no frontier (q = 0) and stay forward."""
    n, src, dst, _ = path(10)
    G = _graph(oracle_mod, n, src, dst)
    depth, _ = G.bfs(0)
    inf = float("inf")
    L = G.do_replay4(5, depth, (inf, inf, inf, 0.02), (0.0, 0.0, 0.0, 0.5))
    assert len(L) == 10
    assert [x["q"][3] for x in L] == [1] * 10
    assert [x["FV"][3] for x in L] == [1] + [2] * 8 + [1]
    assert [x["U"][3] for x in L[:3]] == [9, 8, 7] and [x["s"][3] for x in L[:3]] == [9, 8, 7]
    assert [x["BV"][3] for x in L[:3]] == [pytest.approx(90.0), pytest.approx(72.0),
                                             pytest.approx(56.0)]
    assert [x["dir"][3] for x in L[:3]] == [0, 1, 0]
    assert all(x["q"][:3] == [0, 0, 0] and x["dir"][:3] == [0, 0, 0] for x in L)


def test_do_replay4_reduces_to_replay_when_nn_forward(oracle_mod, inputs_mod):
    """With nn's factor0 at +infinity the four-kernel schedule is the
    three-kernel one of Section IV-B (nn columns: FV_nn and q_nn)."""
    src, dst = inputs_mod.rmat_edges(11)
    n = 1 << 11
    G = _graph(oracle_mod, n, src, dst)
    for s in inputs_mod.pick_sources(src, dst, n, 3, seed=17).tolist():
        depth, _ = G.bfs(s)
        for f0 in ((0.5, 0.05, 1e-7), (1e-3, 1e-3, 1e-3)):
            a = G.do_replay(16, depth, f0, (0.0, 0.1, 0.0))
            b = G.do_replay4(16, depth, f0 + (float("inf"),), (0.0, 0.1, 0.0, 0.0))
            assert len(a) == len(b)
            for x, y in zip(a, b):
                for k in ("q", "s", "U", "FV", "BV", "dir"):
                    assert x[k] == y[k][:3]
                assert (x["FV_nn"], x["q_nn"]) == (y["FV"][3], y["q"][3])
                assert y["dir"][3] == 0


# ---------------------------------------------------------------------------
# PageRank
# ---------------------------------------------------------------------------

def test_pagerank_regular_graphs_stay_uniform(oracle_mod):
    """On a regular graph every vertex receives exactly what it gives: the
    uniform vector is fixed at every step."""
    from closed_forms import hypercube
    for n, src, dst, _ in (cycle(17), complete(9), hypercube(6)):
        G = _graph(oracle_mod, n, src, dst)
        for it in (1, 5, 40):
            r = G.pagerank(0.85, it)
            np.testing.assert_allclose(r, 1.0 / n, rtol=1e-13, atol=0)


def test_pagerank_star_closed_form(oracle_mod):
    """Star, hub 0 with k leaves (n = k + 1), no dangling vertex. The fixed
    point solves h = (1-a)/n + a k l and l = (1-a)/n + a h / k, so
    h = (1 + a k) / (n (1 + a)) and l = (1-a)/n + a h / k; the iteration
    contracts by a per step."""
    a = 0.85
    for k in (1, 5, 40):
        n, src, dst, _ = star(k)
        r = _graph(oracle_mod, n, src, dst).pagerank(a, 400)
        h = (1 + a * k) / (n * (1 + a))
        l = (1 - a) / n + a * h / k
        np.testing.assert_allclose(r[0], h, rtol=1e-12)
        np.testing.assert_allclose(r[1:], l, rtol=1e-12)


@pytest.mark.parametrize("n,k,seed", [(40, 60, 1), (90, 200, 2), (120, 90, 3)])
def test_pagerank_matches_dense_solve(oracle_mod, n, k, seed):
    """Random graphs with isolated vertices (dangling): the iteration's limit
    equals the solution of (I - a M) r = (1 - a)/n, M[v, u] = 1/deg(u) for
    each edge {u, v} and 1/n in the column of a degree-0 vertex, solved by
    numpy's dense LU; every step keeps the ranks summing to 1."""
    rng = np.random.default_rng(seed)
    src, dst = _random_pairs(rng, n, k)
    G = _graph(oracle_mod, n, src, dst)
    a = 0.85
    deg = G.degrees()
    M = np.zeros((n, n))
    off, col = G.off, G.col
    for u in range(n):
        if deg[u] == 0:
            M[:, u] = 1.0 / n
        for i in range(off[u], off[u + 1]):
            M[col[i], u] = 1.0 / deg[u]
    want = np.linalg.solve(np.eye(n) - a * M, np.full(n, (1 - a) / n))
    np.testing.assert_allclose(G.pagerank(a, 400), want, rtol=1e-11, atol=1e-15)
    for it in (1, 2, 7):
        assert abs(G.pagerank(a, it).sum() - 1.0) < 1e-13
