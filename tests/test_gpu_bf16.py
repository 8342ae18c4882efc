"""The bf16 first CholeskyQR pass (LRC_MIXED_BF16GRAM and lrc_truncate_dev
with dtype 2): Gram products of fp32 factors rounded to bf16 on
v_mfma_f32_16x16x32_bf16 with fp32 accumulation, a preset shift on the first
Cholesky, the second pass in fp32.  Checked against the oracle's truncation
(Sec. 5 truncated SVD) at fp32-level tolerances, and in a full solve whose
fp64 residual and refinement reach relres 1e-6 (dense check on the host).

Tolerances: bf16 keeps 8 bits of mantissa, but only the first pass sees it:
the second pass re-orthogonalises in fp32, so products and orthogonality
are held to 1e-4 like the fp32 path, the leading singular values to 1e-4
relative."""
import sys

import numpy as np
import pytest

from oracle import lowrank as olr
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


def _dev(torch, a):
    a = np.asarray(a)
    ld = (a.shape[1] + 7) // 8 * 8
    t = torch.zeros((a.shape[0], ld), dtype=torch.float32, device="cuda")
    t[:, :a.shape[1]] = torch.from_numpy(np.ascontiguousarray(a)).float()
    return t


@pytest.mark.parametrize("n,m,k,cap,tol", [(3000, 400, 50, 20, 1e-6), (20000, 300, 123, 40, 1e-6),
                                           (5000, 80, 30, 30, 0.0), (513, 60, 1, 5, 1e-6)])
def test_bf16_first_pass_truncation_matches_oracle(torch, L, n, m, k, cap, tol):
    say("bf16 truncation", n, m, k, cap, tol)
    ctx = L.Context(0)
    rng = np.random.default_rng(k + n + 1)
    A = rng.standard_normal((n, k)) * rng.uniform(0.1, 10, k)
    B = rng.standard_normal((m, k))
    c = np.logspace(0, -5, k) * np.where(rng.uniform(size=k) < 0.5, -1, 1)
    Uo, so, Vo = olr.truncate(A, np.diag(c), B, cap, tol)
    ld = max(8, (cap + 7) // 8 * 8)
    Ud = torch.zeros((n, ld), dtype=torch.float32, device="cuda")
    Vd = torch.zeros((m, ld), dtype=torch.float32, device="cuda")
    s, r = L.truncate_dev(ctx, _dev(torch, A), c, _dev(torch, B), cap, tol, Ud, Vd, bf16=True)
    U = Ud.double().cpu().numpy()[:, :r]
    V = Vd.double().cpu().numpy()[:, :r]
    X = U @ np.diag(s) @ V.T
    Xo = Uo @ np.diag(so) @ Vo.T
    err = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    orth = max(np.abs(U.T @ U - np.eye(r)).max(), np.abs(V.T @ V - np.eye(r)).max())
    say("rank", r, so.size, "product error", err, "orthogonality", orth)
    assert abs(r - so.size) <= 1
    assert np.allclose(s[:3], so[:3], rtol=1e-4)
    assert err <= 1e-4
    assert orth <= 1e-4


def test_bf16gram_solve_reaches_1e6(torch, L):
    """The c2 structure on a 129 x 129 grid (n = 16,641, m = 200) with the
    bf16 form: fp32 inner ChebyshevT with bf16 first-pass Grams inside fp64
    refinement."""
    say("bf16gram solve")
    ctx = L.Context(0)
    cfg = config("c2", small=True)
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    ops = L.Operators(ctx, K)
    prob = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    prob.precondition()
    code, info = prob.solve(rank_cap=40, trunc_tol=1e-8, res_tol=1e-6,
                            precision=L.LRC_MIXED_BF16GRAM, init=L.LRC_INIT_MEDIAN)
    say("info", info["iters"], info["refinements"], info["relres"])
    assert code == 0 and info["relres"] <= 1e-6
    U, s, V = prob.solution()
    X = U @ np.diag(s) @ V.T
    assert olr.relres_dense(K, d, X, np.outer(f, np.ones(m))) <= 1.01e-6
