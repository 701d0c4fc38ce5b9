"""GPU parity of the DO-on-nn variant (nn_do = 1): nn, which Section IV-B
keeps forward because across GPUs it is not symmetric, goes under the
direction decision too, with its own bottom-up visit. Depths must equal the
oracle's whatever the schedule; the per-level schedule must equal the
oracle's four-kernel replay (or_do_replay4)."""
import numpy as np
import pytest

from closed_forms import all_closed_forms
from gpu_helpers import GpuGraph, log

pytestmark = pytest.mark.gpu

FACTORS = ((0.02, 0.001, 1e-6), (0.0, 0.0, 0.0))


@pytest.mark.parametrize("case", all_closed_forms(), ids=lambda c: c[0])
def test_nn_do_closed_forms(oracle_mod, case):
    name, n, src, dst, dist, sources = case
    O = oracle_mod.Graph(src, dst, n)
    label = O.components()
    for TH in (0, 2, 8, 10 ** 6):
        G = GpuGraph(src, dst, n, threshold=TH)
        for s in sources:
            want = dist(s)
            for forced, seed, fnn in ((0, 0, (1e-3, 0.0)), (0, 0, (0.0, 0.0)), (1, 0, None),
                                      (2, 0, None), (3, 5, None), (3, 6, None)):
                depth, parent, _ = G.bfs(s, forced=forced, seed=seed, nn_do=True, factor_nn=fnn)
                np.testing.assert_array_equal(depth, want,
                                              err_msg=f"{name} TH={TH} s={s} f={forced}/{seed}")
                assert O.check(s, depth, parent, label)[0] == 0, (name, TH, s, forced)
        G.close()


@pytest.mark.parametrize("scale,TH", [(10, 8), (12, 32), (14, 64), (14, 512)])
def test_nn_do_rmat_parity_and_schedule(inputs_mod, oracle_mod, scale, TH):
    """Depths equal the oracle's for several nn factors, and every level's q,
    s, U, FV, BV and direction (dd, dn, nd, nn) equal the oracle's replay."""
    n = 1 << scale
    src, dst = inputs_mod.rmat_edges(scale)
    O = oracle_mod.Graph(src, dst, n)
    G = GpuGraph(src, dst, n, threshold=TH)
    f0, f1 = FACTORS
    for fnn in ((1e-3, 0.0), (1e-6, 0.0), (10.0, 0.0), (1e-3, 0.5), (0.0, 0.0)):
        for s in inputs_mod.pick_sources(src, dst, n, 6, seed=900 + scale).tolist():
            want, _ = O.bfs(s, want_parent=False)
            depth, parent, st = G.bfs(s, want_stats=True, factor0=f0, factor1=f1, nn_do=True,
                                      factor_nn=fnn)
            np.testing.assert_array_equal(depth, want, err_msg=f"s={s} fnn={fnn}")
            assert O.check(s, depth, parent, None)[0] == 0
            rep = O.do_replay4(TH, want, f0 + (fnn[0],), f1 + (fnn[1],))
            assert st["num_levels"] == len(rep)
            for L, (a, b) in enumerate(zip(st["levels"], rep)):
                for k in ("q", "s", "U", "FV", "dir"):
                    assert a[k] == b[k][:3], (L, k, a[k], b[k])
                assert a["BV"] == b["BV"][:3], (L, a["BV"], b["BV"])
                assert (a["q_nn"], a["FV_nn"], a["U_nn"], a["s_nn"], a["dir_nn"]) == \
                    (b["q"][3], b["FV"][3], b["U"][3], b["s"][3], b["dir"][3]), (L, a, b)
                assert a["BV_nn"] == b["BV"][3]
            if scale >= 12 and fnn == (1e-6, 0.0):
                assert any(lv["dir_nn"] == 1 for lv in st["levels"]) or TH < 8
        log(f"nn_do scale={scale} TH={TH} fnn={fnn} ok")
    G.close()


def test_nn_do_profiled_captured_and_default_agree(inputs_mod, oracle_mod):
    """nn_do searches as captured level graphs and as profiled direct
    launches give the same levels; switching between nn_do and the default
    path on one workspace re-captures the level graphs correctly."""
    n = 1 << 14
    src, dst = inputs_mod.rmat_edges(14)
    O = oracle_mod.Graph(src, dst, n)
    G = GpuGraph(src, dst, n, threshold=64)
    for s in inputs_mod.pick_sources(src, dst, n, 4, seed=61).tolist():
        want, _ = O.bfs(s, want_parent=False)
        runs = []
        for nn_do, prof in ((True, False), (False, False), (True, True), (True, False)):
            depth, parent, st = G.bfs(s, want_stats=True, profile=prof, nn_do=nn_do,
                                      factor_nn=(1e-6, 0.0))
            np.testing.assert_array_equal(depth, want)
            assert O.check(s, depth, parent, None)[0] == 0
            runs.append(st)
        assert runs[0]["levels"] == runs[2]["levels"] == runs[3]["levels"]
        for k in runs[0]["kernels"]:
            assert runs[0]["kernels"][k]["launches"] == runs[2]["kernels"][k]["launches"], k
        assert runs[0]["reached"] == runs[1]["reached"] == int((want >= 0).sum())
    G.close()


def test_nn_do_rmat22_all_64_sources(inputs_mod):
    """DO-on-nn at RMAT scale 22, TH 64 (more nn edges than at TH 32), all 64
    seeded sources: every depth row equal to the oracle's digest."""
    from digests import RowChecker, load, sources_of
    want = load("rmat22")
    sources = sources_of("rmat22")
    n = 1 << 22
    src, dst = inputs_mod.rmat_edges(22)
    G = GpuGraph(src, dst, n, threshold=64)
    del src, dst
    for fnn in ((1e-3, 0.0), (1e-7, 0.0)):
        chk = RowChecker(want)
        levels_bwd = 0
        for s in sources:
            depth, _, st = G.bfs(s, want_parent=False, want_stats=True, nn_do=True,
                                 factor_nn=fnn)
            assert st["reached"] == want[s]["reached"], s
            levels_bwd += sum(lv["dir_nn"] for lv in st["levels"])
            chk.submit(s, depth)
        bad = chk.mismatches()
        assert not bad, f"fnn={fnn}: {len(bad)} rows differ from the oracle's digests: {bad[:2]}"
        log(f"nn_do scale 22 fnn={fnn}: {chk.checked} rows equal, {levels_bwd} levels nn backward")
    G.close()
