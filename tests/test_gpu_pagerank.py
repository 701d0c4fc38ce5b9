"""PageRank on the degree-separated layout (dsbfs_pagerank) against the
oracle's FP64 power iteration, step for step.

Tolerance: both sides compute in FP64; they differ only in the order of the
additions (a delegate row is summed by 64 strided partial sums, the dangling
mass by atomics). One reordered sum of k terms of magnitude at most x moves
by at most about k * 2^-53 * k x; with rows up to 10^6 entries summed in 64
stripes and values near 1/n, the per-step difference stays below 1e-11
relative, and the iteration contracts by alpha per step, so 1e-10 relative
(plus 1e-18 absolute) bounds it after any number of steps."""
import numpy as np
import pytest

from closed_forms import all_closed_forms
from gpu_helpers import lib, log, torch_cuda

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-10, 1e-18


def _run(d, torch, G, n, alpha, iters, tol=0.0):
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    steps, delta = d.pagerank(G, r, alpha=alpha, iterations=iters, tolerance=tol)
    torch.cuda.synchronize()
    return r.cpu().numpy(), steps, delta


@pytest.mark.parametrize("case", all_closed_forms()[:6], ids=lambda c: c[0])
def test_pagerank_closed_forms(oracle_mod, case):
    d = lib()
    torch = torch_cuda()
    name, n, src, dst, _, _ = case
    O = oracle_mod.Graph(src, dst, n)
    for TH in (0, 2, 10 ** 6):
        G = d.Graph(src, dst, n, threshold=TH, keep_plain_csr=False)
        for iters in (0, 1, 7, 30):
            got, steps, _ = _run(d, torch, G, n, 0.85, iters)
            assert steps == iters
            np.testing.assert_allclose(got, O.pagerank(0.85, iters), rtol=RTOL, atol=ATOL,
                                       err_msg=f"{name} TH={TH} iters={iters}")
        G.destroy()


@pytest.mark.parametrize("kind,scale,TH", [("rmat", 12, 8), ("rmat", 16, 32), ("rmat", 16, 0),
                                           ("rmat", 14, 10 ** 6), ("er", 14, 16)])
def test_pagerank_matches_oracle(inputs_mod, oracle_mod, kind, scale, TH):
    """RMAT (hubs become delegates with long rows) and Erdos-Renyi with
    isolated vertices (dangling mass), several thresholds, several alphas."""
    d = lib()
    torch = torch_cuda()
    n = 1 << scale
    if kind == "rmat":
        src, dst = inputs_mod.rmat_edges(scale)
    else:
        src, dst = inputs_mod.er_edges(n, n // 2, seed=0x22)   # many isolated vertices
    O = oracle_mod.Graph(src, dst, n)
    G = d.Graph(src, dst, n, threshold=TH, keep_plain_csr=False)
    for alpha, iters in ((0.85, 20), (0.5, 5), (1.0, 3), (0.0, 2)):
        got, _, _ = _run(d, torch, G, n, alpha, iters)
        want = O.pagerank(alpha, iters)
        np.testing.assert_allclose(got, want, rtol=RTOL, atol=ATOL,
                                   err_msg=f"{kind} {scale} TH={TH} alpha={alpha}")
        assert abs(got.sum() - 1.0) < 1e-9
    log(f"pagerank {kind} {scale} TH={TH} ok, d={G.stats['d']}")
    G.destroy()


def test_pagerank_tolerance_stop_and_errors(inputs_mod, oracle_mod):
    d = lib()
    torch = torch_cuda()
    n = 1 << 12
    src, dst = inputs_mod.rmat_edges(12)
    O = oracle_mod.Graph(src, dst, n)
    G = d.Graph(src, dst, n, threshold=16, keep_plain_csr=False)
    got, steps, delta = _run(d, torch, G, n, 0.85, 500, tol=1e-9)
    assert 5 < steps < 500 and 0 < delta < 1e-9
    np.testing.assert_allclose(got, O.pagerank(0.85, steps), rtol=RTOL, atol=ATOL)
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    for bad in ((1.5, 3), (-0.1, 3), (0.85, -1)):
        with pytest.raises(d.DsbfsError) as e:
            d.pagerank(G, r, alpha=bad[0], iterations=bad[1])
        assert e.value.status == d.ERR_INVALID_ARG
    G.destroy()
