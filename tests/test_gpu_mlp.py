"""The surrogate network's HIP kernels against the FP64 oracle (oracle/mlp.py),
and the gain of the learned initial guess over the median one.

Tolerances: weights and activations are bf16 (8-bit mantissa, relative
rounding 2^-9 ~ 2e-3 per operand), products accumulate in fp32; a few such
roundings per layer give per-tensor relative gradient errors of ~1e-2, so the
gradient check uses 3e-2.  The gain is measured, not pinned: the paper has no
network."""
import sys

import numpy as np
import pytest

from oracle import lowrank as olr
from oracle import mlp as omlp
from workloads import config, mlp_init, param_table

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


def _data(rng, B, r=30):
    X = rng.uniform(-1.0, 1.0, (B, 2))
    T = rng.standard_normal((B, r))
    return X, T


def test_mlp_gradients_match_oracle(torch, L, ctx):
    say("mlp gradients")
    params = mlp_init(11)
    X, T = _data(np.random.default_rng(0), 200)
    net = L.MLP(ctx, params)
    loss, g = net.grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    Y, cache = omlp.forward(params, X)
    ref = omlp.backward(params, cache, Y, T)
    assert abs(loss - omlp.loss(Y, T)) <= 1e-2 * omlp.loss(Y, T)
    for i, (a, b) in enumerate(zip(g, ref)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        say("tensor", i, "rel err", rel)
        assert rel < 3e-2, (i, rel)


def test_mlp_first_adam_step_is_signed_lr(torch, L, ctx):
    say("mlp first adam step")
    params = mlp_init(11)
    X, T = _data(np.random.default_rng(1), 128)
    net = L.MLP(ctx, params)
    net.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), 1, lr=1e-3)
    new = net.params()
    # bias-corrected first step: p - lr * g / (|g| + eps) = p - lr sign(g) where g != 0
    Y, cache = omlp.forward(params, X)
    ref = omlp.backward(params, cache, Y, T)
    mism = 0
    total = 0
    for p0, p1, gr in zip(params, new, ref):
        d = p1 - p0.astype(np.float32)
        big = np.abs(gr) > 1e-3 * np.max(np.abs(gr))
        total += int(big.sum())
        mism += int(np.sum(np.abs(d[big] + 1e-3 * np.sign(gr[big])) > 2e-5))
    assert mism <= 0.01 * total, (mism, total)


def test_mlp_training_tracks_oracle(torch, L, ctx):
    say("mlp training")
    params = mlp_init(11)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1.0, 1.0, (200, 2))
    # smooth, mostly low-order targets a small network fits quickly
    a = rng.standard_normal((3, 30))
    T = a[0] * X[:, :1] + a[1] * X[:, 1:] + 0.3 * a[2] * np.sin(X[:, :1] + X[:, 1:])
    T = (T - T.mean(0)) / T.std(0)
    net = L.MLP(ctx, params)
    hist = net.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), 300)
    _, ohist = omlp.train(params, X, T, 300)
    say("loss gpu", hist[0], hist[-1], "oracle", ohist[0], ohist[-1])
    assert abs(hist[0] - ohist[0]) <= 1e-2 * ohist[0]
    assert hist[-1] < 0.5 * hist[0]
    assert hist[-1] <= 1.25 * ohist[-1] + 1e-3


def test_mlp_predict_applies_fitted_scaling(torch, L, ctx):
    say("mlp predict")
    params = mlp_init(11)
    rng = np.random.default_rng(3)
    mu = rng.uniform(0.5e4, 2e4, 50)
    lam = rng.uniform(1e4, 4e4, 50)
    Xr = np.column_stack([mu, lam])
    Tr = rng.standard_normal((50, 30)) * 5.0 + 3.0
    net = L.MLP(ctx, params)
    net.fit_scaling(torch.from_numpy(Xr).cuda(), torch.from_numpy(Tr).cuda())
    Y = net.predict(torch.from_numpy(Xr).cuda()).cpu().numpy()
    Xn = omlp.normalise_inputs(mu, lam, (mu.min(), mu.max()), (lam.min(), lam.max()))
    _, mt, st = omlp.standardise(Tr)
    Yo, _ = omlp.forward(params, Xn)
    Yo = Yo * st + mt
    assert np.linalg.norm(Y - Yo) <= 2e-2 * np.linalg.norm(Yo)


def _solve(L, ops, d, f, **kw):
    m = d.shape[1]
    p = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    p.precondition()
    code, info = p.solve(rank_cap=30, trunc_tol=1e-8, res_tol=1e-6, **kw)
    return p, code, info


def test_learned_initial_guess_gain(torch, L, ctx):
    """Snapshots from the GPU solver on 40 training parameters, POD basis and
    coefficients from the GPU truncation, network trained on the GPU; on 60
    held-out parameters the learned X0 = U0 C^T is compared with the median
    guess by iterations to relres 1e-6 (both must reach it)."""
    say("surrogate gain")
    cfg = config("c4", small=True)
    K, f = cfg["ops"].K, cfg["f"]
    dtr, dte = cfg["d_train"], cfg["d_test"]
    ops = L.Operators(ctx, K)
    ptr, code, _ = _solve(L, ops, dtr, f, init=L.LRC_INIT_MEDIAN)
    assert code == 0
    U, s, V = ptr.solution()
    n, mtr = U.shape[0], V.shape[0]
    r = 30
    # POD of the snapshot matrix U diag(s) V^T by the GPU truncation (rank <= r,
    # tail cut at the solver's truncation tolerance)
    k = U.shape[1]
    ld = (k + 7) // 8 * 8
    Ud = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    Ud[:, :k] = torch.from_numpy(U).cuda()
    Vd = torch.zeros((mtr, ld), dtype=torch.float64, device="cuda")
    Vd[:, :k] = torch.from_numpy(V).cuda()
    U0 = torch.zeros((n, 32), dtype=torch.float64, device="cuda")
    V0 = torch.zeros((mtr, 32), dtype=torch.float64, device="cuda")
    s0, rr = L.truncate_dev(ctx, Ud, s, Vd, r, cfg["trunc_tol"], U0, V0)
    Ctr = V0[:, :rr] * torch.from_numpy(s0).cuda()          # training coefficients
    net = L.MLP(ctx, mlp_init(11, sizes=(2, 64, 64, rr)))
    Xtr = torch.from_numpy(np.ascontiguousarray(dtr[1:].T)).cuda()
    net.fit_scaling(Xtr, Ctr.contiguous())
    hist = net.train(Xtr, Ctr.contiguous(), 2000, lr=3e-3)
    say("train loss", hist[0], hist[-1])
    Xte = torch.from_numpy(np.ascontiguousarray(dte[1:].T)).cuda()
    Cte = net.predict(Xte).cpu().numpy()
    U0h = U0[:, :rr].cpu().numpy()
    pm, code_m, info_m = _solve(L, ops, dte, f, init=L.LRC_INIT_MEDIAN)
    pl, code_l, info_l = _solve(L, ops, dte, f, init=L.LRC_INIT_GIVEN, X0=(U0h, np.ones(rr), Cte))
    say("median", info_m["iters"], info_m["relres"], "learned", info_l["iters"], info_l["relres"])
    assert code_m == 0 and code_l == 0
    # the same guess passed as device factors (lrc_solve_x0_dev)
    code_d, info_d = pl.solve_x0_dev(U0[:, :rr].contiguous(), torch.from_numpy(Cte).cuda(),
                                     rank_cap=30, trunc_tol=1e-8, res_tol=1e-6)
    assert code_d == 0 and info_d["iters"] == info_l["iters"]
    assert abs(info_d["relres"] - info_l["relres"]) <= 1e-3 * info_l["relres"]
    Ul, sl, Vl = pl.solution()
    Xl = Ul @ np.diag(sl) @ Vl.T
    Fd = np.outer(f, np.ones(dte.shape[1]))
    assert olr.relres_dense(K, dte, Xl, Fd) <= 1.01e-6
    assert info_l["relres"] <= 1e-6
    # the learned guess starts closer: strictly fewer Chebyshev updates
    assert info_l["iters"] < info_m["iters"]
    # judged by the plain guess column by column (LRC_INIT_GIVEN_JUDGED): the
    # trained network keeps most columns and loses nothing against the median
    pj, code_j, info_j = _solve(L, ops, dte, f, init=L.LRC_INIT_GIVEN_JUDGED,
                                X0=(U0h, np.ones(rr), Cte))
    mte = dte.shape[1]
    say("judged", info_j["iters"], info_j["median_fallback_cols"], "of", mte)
    assert code_j == 0 and info_j["relres"] <= 1e-6
    assert info_j["median_fallback_cols"] < mte // 2
    assert info_j["iters"] <= info_l["iters"] + 1
    # a perturbed network (its output's sign flipped) loses in every column:
    # the fallback takes the median guess everywhere and the solve proceeds as
    # from the median guess alone
    pb, code_b, info_b = _solve(L, ops, dte, f, init=L.LRC_INIT_GIVEN_JUDGED,
                                X0=(U0h, np.ones(rr), -Cte))
    say("judged perturbed", info_b["iters"], info_b["median_fallback_cols"])
    assert code_b == 0 and info_b["relres"] <= 1e-6
    assert info_b["median_fallback_cols"] == mte
    assert abs(info_b["iters"] - info_m["iters"]) <= 1
    Ub, sb, Vb = pb.solution()
    assert olr.relres_dense(K, dte, Ub @ np.diag(sb) @ Vb.T, Fd) <= 1.01e-6
