"""Boundary calls not exercised by the solver tests, through the C ABI:
lrc_ops_update_values (a new linearisation point on the same pattern: the
fused SpMM then multiplies by the new values, element by element against
SciPy, and a solve after it matches a problem built from the new operators
from scratch) and lrc_prob_spectrum (the ratio interval of the Sec. 4.2
centre preconditioner against the oracle's, on an asymmetric table)."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import chebyshev as och
from workloads import config

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "no GPU"
    return t


@pytest.fixture(scope="module")
def L():
    from paper_2008_10275_amd import lrcheb
    return lrcheb


def test_update_values_then_spmm_and_solve(torch, L):
    say("update_values")
    cfg = config("c1")
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    n, m = K[0].shape[0], d.shape[1]
    rng = np.random.default_rng(5)
    # K_0 at a new linearisation point on the same (symmetric) pattern: its
    # symmetric part added once more, which changes the upwind and the
    # symmetric entries differently and keeps K_0 + K_0^T positive definite
    K0n = sp.csr_matrix(K[0] + 0.5 * (K[0] + K[0].T))
    K0n.sort_indices()
    assert np.array_equal(K0n.indptr, K[0].indptr) and np.array_equal(K0n.indices, K[0].indices)
    ctx = L.Context(0)
    ops = L.Operators(ctx, K)
    ops.update_values(0, K0n.data)
    U = rng.standard_normal((n, 8))
    Ud = torch.from_numpy(U).cuda()
    W = torch.zeros((len(K) * n, 8), dtype=torch.float64, device="cuda")
    ops.spmm_dev(Ud, W, 8)
    torch.cuda.synchronize()
    Wh = W.cpu().numpy()
    for i, Ki in enumerate([K0n] + list(K[1:])):
        ref = Ki @ U
        scale = abs(Ki) @ np.abs(U) + 1e-300
        assert np.all(np.abs(Wh[i * n:(i + 1) * n] - ref) <= 1e-14 * scale), i
    # a solve on the updated operators equals one on operators built anew
    kw = dict(rank_cap=cfg["rank_cap"], trunc_tol=cfg["trunc_tol"], res_tol=1e-8,
              init=L.LRC_INIT_MEDIAN)
    p1 = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    p1.precondition()
    c1, i1 = p1.solve(**kw)
    ops2 = L.Operators(ctx, [K0n] + list(K[1:]))
    p2 = L.Problem(ops2, d, f[:, None], np.ones((m, 1)))
    p2.precondition()
    c2, i2 = p2.solve(**kw)
    say("iters", i1["iters"], i2["iters"], i1["relres"], i2["relres"])
    assert c1 == 0 and c2 == 0 and i1["iters"] == i2["iters"]
    U1, s1, V1 = p1.solution()
    U2, s2, V2 = p2.solution()
    X1, X2 = U1 @ np.diag(s1) @ V1.T, U2 @ np.diag(s2) @ V2.T
    assert np.linalg.norm(X1 - X2) <= 1e-12 * np.linalg.norm(X2)
    with pytest.raises(L.LrcError):
        ops.update_values(len(K), K0n.data)       # no such operator


def test_spectrum_matches_oracle_interval(torch, L):
    say("spectrum")
    cfg = config("c1")
    K, f = cfg["ops"].K, cfg["f"]
    n = K[0].shape[0]
    # asymmetric table: the mean differs from the midrange, and one column
    # lies below 1 in every ratio
    d = np.vstack([np.ones(5), [0.6e4, 1.0e4, 1.1e4, 1.9e4, 2.0e4],
                   [1.0e4, 1.2e4, 1.3e4, 3.9e4, 4.0e4]])
    ctx = L.Context(0)
    ops = L.Operators(ctx, K)
    p = L.Problem(ops, d, f[:, None], np.ones((5, 1)))
    c, dc = p.spectrum()
    co, do = och.chebyshev_interval(d, och.mean_parameters(d))
    say("gpu", c, dc, "oracle", co, do)
    assert abs(c - co) <= 1e-15 * do and abs(dc - do) <= 1e-15 * do
    # with an explicit centre the interval follows it
    p.precondition(dbar=np.array([1.0, 1.0e4, 1.0e4]))
    c2, d2 = p.spectrum()
    co2, do2 = och.chebyshev_interval(d, np.array([1.0, 1.0e4, 1.0e4]))
    assert abs(c2 - co2) <= 1e-15 * do2 and abs(d2 - do2) <= 1e-15 * do2
