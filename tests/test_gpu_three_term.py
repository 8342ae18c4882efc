"""The three-term form of the ChebyshevT recurrence on the GPU (one
truncation of [X_k | X_{k-1} | P^-1 R] per update, the iterate alternating
between two buffers) against the oracle's three-term form.

fp64: the same recurrence on the same data, so the iteration counts agree to
within one and the iterates to far below the residual bound, as for the
direction form.  Mixed forms: the dense residual of the result is checked with
the oracle's fp64 operator."""
import sys

import numpy as np
import pytest

from oracle import driver as odrv
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


@pytest.fixture(scope="module")
def ctx(torch, L):
    return L.Context(0)


@pytest.fixture(scope="module")
def c1(L, ctx):
    cfg = config("c1")
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    ops = L.Operators(ctx, K)
    prob = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    prob.precondition()
    return cfg, ops, prob


@pytest.mark.parametrize("restart", [6, 5, 1])
def test_c1_three_term_matches_oracle(torch, L, ctx, c1, restart):
    """restart 5 ends every full cycle in the second buffer (copied back on the
    device), restart 1 makes every update a first step."""
    cfg, _, prob = c1
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    say("solve c1 fp64 three-term restart", restart)
    code, info = prob.solve(rank_cap=20, trunc_tol=1e-8, res_tol=1e-8, init=L.LRC_INIT_MEDIAN,
                            restart=restart, recurrence=L.LRC_CHEB_THREE_TERM)
    say("info", info)
    ref = odrv.newton_subset(K, d, f, 20, 1e-8, 1e-8, restart=restart, form="three_term")
    say("oracle iters", ref["info"].iters, "converged", ref["info"].converged)
    assert ref["info"].converged
    assert code == 0 and info["relres"] <= 1e-8
    assert abs(info["iters"] - ref["info"].iters) <= 1
    assert info["prec_applies"] == info["iters"]
    U, s, V = prob.solution()
    X = U @ np.diag(s) @ V.T
    Xo = sum(olr.lr_dense(*t) for t in odrv.solution_terms(ref))
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) < 1e-9
    Fd = np.outer(f, np.ones(m))
    assert olr.relres_dense(K, d, X, Fd) <= 1.01e-8


def test_c1_three_term_tracks_direction_form(torch, L, ctx, c1):
    """Same polynomial iteration: the two forms stop after the same number of
    updates and their solutions agree to the truncation level."""
    _, _, prob = c1
    kw = dict(rank_cap=20, trunc_tol=1e-8, res_tol=1e-8, init=L.LRC_INIT_MEDIAN)
    say("solve c1 fp64 direction vs three-term")
    _, i2 = prob.solve(recurrence=L.LRC_CHEB_DIRECTION, **kw)
    U, s, V = prob.solution()
    X2 = U @ np.diag(s) @ V.T
    _, i3 = prob.solve(recurrence=L.LRC_CHEB_THREE_TERM, **kw)
    U, s, V = prob.solution()
    X3 = U @ np.diag(s) @ V.T
    say("iters", i2["iters"], i3["iters"])
    assert i3["iters"] == i2["iters"]
    assert np.linalg.norm(X3 - X2) <= 1e-6 * np.linalg.norm(X2)


@pytest.mark.parametrize("mode", ["dir", "refine", "fp64"])
def test_c2_small_three_term(torch, L, ctx, mode):
    cfg = config("c2", small=True)
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    say("solve c2-small three-term", mode)
    ops = L.Operators(ctx, K)
    prob = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    prob.precondition()
    prec = {"dir": L.LRC_MIXED_FP32_DIR, "refine": L.LRC_MIXED_FP32, "fp64": L.LRC_FP64}[mode]
    code, info = prob.solve(rank_cap=40, trunc_tol=1e-8, res_tol=1e-6, precision=prec,
                            init=L.LRC_INIT_MEDIAN, recurrence=L.LRC_CHEB_THREE_TERM)
    say("info", info)
    assert code == 0 and info["relres"] <= 1e-6
    U, s, V = prob.solution()
    X = U @ np.diag(s) @ V.T
    assert olr.relres_dense(K, d, X, np.outer(f, np.ones(m))) <= 1.01e-6
    if mode != "refine":
        ref = odrv.newton_subset(K, d, f, 40, 1e-8, 1e-6, form="three_term")
        say("oracle iters", ref["info"].iters)
        assert abs(info["iters"] - ref["info"].iters) <= 1


def test_three_term_rejects_wide_cap(torch, L, ctx, c1):
    """3 x rank_cap columns must fit the 128 of a truncation."""
    _, _, prob = c1
    with pytest.raises(L.LrcError) as e:
        prob.solve(rank_cap=48, trunc_tol=1e-8, res_tol=1e-8, recurrence=L.LRC_CHEB_THREE_TERM)
    assert e.value.code == L.LRC_EINVAL and "three-term" in str(e.value)
