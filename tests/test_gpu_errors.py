"""Failure paths of the C ABI on the GPU (the status codes of include/lrcheb.h):
a singular centre operator (LRC_ESINGULAR from the factorisation), non-finite
right-hand sides (LRC_EINVAL before anything runs), a truncation whose
operands hold NaN (LRC_EBREAKDOWN: the Cholesky fails at every shift), and a
solve with a wrong spectrum interval that cannot converge within its
iteration limit (LRC_ENOTCONV, a warning: the call returns its best iterate
and its own residual).  Every case ends normally on the device: the kernels'
loops are bounded, NaN only fails their tests."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

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


def test_singular_centre_operator(torch, L):
    say("singular preconditioner")
    ctx = L.Context(0)
    K = config("c1")["ops"].K
    Z = [sp.csr_matrix((np.zeros_like(k.data), k.indices, k.indptr), shape=k.shape) for k in K]
    ops = L.Operators(ctx, Z)
    d = config("c1")["d"]
    n, m = K[0].shape[0], d.shape[1]
    p = L.Problem(ops, d, np.ones((n, 1)), np.ones((m, 1)))
    with pytest.raises(L.LrcError) as e:
        p.precondition()
    assert e.value.code == L.LRC_ESINGULAR


def test_non_finite_right_hand_side(torch, L):
    say("nan rhs")
    ctx = L.Context(0)
    cfg = config("c1")
    ops = L.Operators(ctx, cfg["ops"].K)
    f = cfg["f"].copy()
    f[7] = np.nan
    with pytest.raises(L.LrcError) as e:
        L.Problem(ops, cfg["d"], f[:, None], np.ones((cfg["d"].shape[1], 1)))
    assert e.value.code == L.LRC_EINVAL and "non-finite" in str(e.value)


def test_truncation_breakdown_on_nan(torch, L):
    say("nan truncation")
    ctx = L.Context(0)
    n, m, k = 500, 40, 6
    A = torch.randn((n, 8), dtype=torch.float64, device="cuda")
    A[3, 2] = float("nan")
    B = torch.randn((m, 8), dtype=torch.float64, device="cuda")
    U = torch.zeros((n, 8), dtype=torch.float64, device="cuda")
    V = torch.zeros((m, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(L.LrcError) as e:
        L.truncate_dev(ctx, A, np.ones(k), B, 4, 1e-8, U, V)
    assert e.value.code == L.LRC_EBREAKDOWN
    # the context stays usable: the same call on finite data succeeds
    A[3, 2] = 0.5
    s, r = L.truncate_dev(ctx, A, np.ones(k), B, 4, 1e-8, U, V)
    assert r == 4 and np.all(np.isfinite(s))


def test_wrong_interval_does_not_converge(torch, L):
    """The true preconditioned spectrum of c1 fills [0.4, 1.6]; an interval
    [0.95, 1.05] leaves its ends outside, where the Chebyshev polynomials grow:
    the solve stops at its iteration limit with LRC_ENOTCONV."""
    say("wrong interval")
    ctx = L.Context(0)
    cfg = config("c1")
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    ops = L.Operators(ctx, K)
    p = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    p.precondition()
    code, info = p.solve(rank_cap=20, trunc_tol=1e-8, res_tol=1e-8, init=L.LRC_INIT_MEDIAN,
                         cheb_c=0.05, cheb_d=1.0, max_iter=24)
    say("info", info["iters"], info["relres"], info["status"])
    assert code == L.LRC_ENOTCONV and info["status"] == L.LRC_ENOTCONV
    assert info["iters"] <= 24 and not info["relres"] <= 1e-8
    # the right interval converges on the same problem
    code, info = p.solve(rank_cap=20, trunc_tol=1e-8, res_tol=1e-8, init=L.LRC_INIT_MEDIAN)
    assert code == 0 and info["relres"] <= 1e-8


def test_truncation_capacity_exceeded(torch, L):
    """A random right-hand side of rank 8 (the least room the solver keeps
    for it) with rank_cap 64 and q = 3: once S passes rank 40 the residual
    B - L(S) concatenates more than 8 + 3 * 40 columns, beyond the
    truncation's 128.
    The device clamps the width (no access past the workspace), flags it, and
    the call fails with LRC_EINVAL naming the capacity, before the fp64
    residual check."""
    say("truncation capacity")
    ctx = L.Context(0)
    cfg = config("c1")
    K, d = cfg["ops"].K, cfg["d"]
    n, m = K[0].shape[0], d.shape[1]
    rng = np.random.default_rng(11)
    ops = L.Operators(ctx, K)
    p = L.Problem(ops, d, rng.standard_normal((n, 8)), rng.standard_normal((m, 8)))
    p.precondition()
    with pytest.raises(L.LrcError) as e:
        p.solve(rank_cap=64, trunc_tol=1e-14, res_tol=1e-12, init=L.LRC_INIT_ZERO, max_iter=12)
    say("error", e.value.code, str(e.value))
    assert e.value.code == L.LRC_EINVAL and "capacity" in str(e.value)
