"""Algorithm 1 (Sec. 4.1) through the C ABI's subset driver against the oracle.

The driver runs Newton on each subset's upper-median column (Sec. 3.3) from
the previous subset's solution, then one low-rank Newton step on the subset
(eq. newton_matrix1) with X^k = x~^k 1^T + S_k (eq. matrix_nextiterate1); the
oracle solves the median column directly and runs its own ChebyshevT.  Both
stop at the relative residual res_tol against ||b|| sqrt(m_k).  Parity is
judged through residuals, iteration counts (+-1) and the error against the
exact column-wise solution, never through factors.  The fixed-point variant
(Sec. 5.3, eq. picard_matrix1) truncates X itself; on these operators its
residual stalls far above the Newton variant's, which is the paper's
observation that Newton is at least ten times more accurate."""
import sys

import numpy as np
import pytest

from oracle import chebyshev as och
from oracle import driver as odrv
from oracle import lowrank as olr
from workloads import config, param_table, three_term_2d

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
def c1():
    cfg = config("c1")
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    Xstar = olr.solve_columns(K, d, np.outer(f, np.ones(d.shape[1])))
    return K, d, f, Xstar


def _dense(p):
    U, s, V = p.solution()
    return U @ np.diag(s) @ V.T


@pytest.mark.parametrize("sizes", [None, [10, 40, 20, 30]])
def test_algorithm1_matches_oracle(torch, L, ctx, c1, sizes):
    K, d, f, Xstar = c1
    say("algorithm1", sizes)
    ops = L.Operators(ctx, K)
    code, probs, infos, used = L.newton_subsets(ops, d, 4, f, sizes=sizes, rank_cap=20,
                                                trunc_tol=1e-8, res_tol=1e-8)
    ref = odrv.algorithm1(K, d, f, 4, 20, 1e-8, 1e-8, sizes=sizes)
    # subset sizes as the library used them: eq. clustering1 or the given list
    assert used == (odrv.subset_sizes(d.shape[1], 4) if sizes is None else sizes)
    assert code == 0
    for k, (p, inf, r) in enumerate(zip(probs, infos, ref)):
        J = r["cols"]
        say("subset", k, inf["iters"], r["info"].iters, inf["relres"], inf["newton_steps"])
        assert inf["newton_steps"] >= 1 and inf["relres"] <= 1e-8
        assert abs(inf["iters"] - r["info"].iters) <= 1
        X = _dense(p)
        Fk = np.outer(f, np.ones(J.size))
        assert olr.relres_dense(K, d[:, J], X, Fk) <= 1.01e-8
        Xo = sum(olr.lr_dense(*t) for t in odrv.solution_terms(r))
        Xs = Xstar[:, J]
        e_gpu = np.linalg.norm(X - Xs) / np.linalg.norm(Xs)
        e_orc = np.linalg.norm(Xo - Xs) / np.linalg.norm(Xs)
        say("error vs exact", e_gpu, e_orc)
        # the oracle solves the median column directly, the GPU iteratively to
        # eps_N = 1e-6 and lets S absorb the rest, so the GPU's error is not
        # the oracle's; both must stay far below what relres 1e-8 allows
        assert e_gpu <= 10 * e_orc + 1e-9


def test_algorithm1_callback_equals_linear_default(torch, L, ctx, c1):
    """A callback that returns the linear problem's J = K and B_k(x) =
    f 1^T - L(x 1^T) (computed here with SciPy) gives the library's own linear
    default, up to rounding."""
    K, d, f, _ = c1
    say("algorithm1 callback")
    ops = L.Operators(ctx, K)
    sizes = [30, 30, 40]
    starts = np.cumsum([0] + sizes)
    seen = []

    def lin(k, stage, x):
        seen.append((k, stage))
        dk = d[:, starts[k]:starts[k + 1]]
        if stage == 1:
            return None, f[:, None], np.ones((dk.shape[1], 1)), np.linalg.norm(f)
        BU = np.column_stack([f] + [-(Ki @ x) for Ki in K])
        BV = np.column_stack([np.ones(dk.shape[1])] + [dk[i] for i in range(len(K))])
        return None, BU, BV, np.linalg.norm(f)

    c_cb, p_cb, i_cb, _ = L.newton_subsets(ops, d, 3, sizes=sizes, linearize=lin,
                                           eps_newton=1e-5 * np.linalg.norm(f), rank_cap=20,
                                           trunc_tol=1e-8, res_tol=1e-8)
    c_df, p_df, i_df, _ = L.newton_subsets(ops, d, 3, f, sizes=sizes, rank_cap=20,
                                           trunc_tol=1e-8, res_tol=1e-8)
    assert c_cb == 0 and c_df == 0
    # two linearisations per subset: at x~^{k-1} and at x~^k (one Newton step)
    assert [s for s in seen if s[1] == 0] == [(k, 0) for k in range(3) for _ in range(2)]
    for a, b, ia, ib in zip(p_cb, p_df, i_cb, i_df):
        assert abs(ia["iters"] - ib["iters"]) <= 1
        Xa, Xb = _dense(a), _dense(b)
        assert np.linalg.norm(Xa - Xb) <= 1e-6 * np.linalg.norm(Xb)


def test_algorithm1_linearisation_points_per_subset(torch, L, ctx):
    """Each subset gets its own Jacobian through the callback (the batched
    workload's perturbed convection-diffusion operator); every subset's step
    must match the oracle's Newton step on that subset's operator."""
    say("algorithm1 per-subset operators")
    cfg = config("c3", small=True)
    subs = cfg["subsets"][:3]
    f = cfg["f"]
    d = np.concatenate([s["d"] for s in subs], axis=1)
    sizes = [s["d"].shape[1] for s in subs]
    starts = np.cumsum([0] + sizes)
    ops = L.Operators(ctx, cfg["base_ops"].K)

    def lin(k, stage, x):
        Kk = subs[k]["ops"].K
        dk = d[:, starts[k]:starts[k + 1]]
        vals = [Ki.data for Ki in Kk]
        if stage == 1:
            return vals, f[:, None], np.ones((dk.shape[1], 1)), np.linalg.norm(f)
        BU = np.column_stack([f] + [-(Ki @ x) for Ki in Kk])
        BV = np.column_stack([np.ones(dk.shape[1])] + [dk[i] for i in range(len(Kk))])
        return vals, BU, BV, np.linalg.norm(f)

    code, probs, infos, _ = L.newton_subsets(ops, d, 3, sizes=sizes, linearize=lin,
                                             eps_newton=1e-5 * np.linalg.norm(f), rank_cap=30,
                                             trunc_tol=1e-8, res_tol=1e-6)
    assert code == 0
    for k, (p, inf) in enumerate(zip(probs, infos)):
        Kk = subs[k]["ops"].K
        dk = subs[k]["d"]
        ref = odrv.newton_subset(Kk, dk, f, 30, 1e-8, 1e-6)
        say("subset", k, inf["iters"], ref["info"].iters, inf["relres"])
        assert abs(inf["iters"] - ref["info"].iters) <= 1
        X = _dense(p)
        assert olr.relres_dense(Kk, dk, X, np.outer(f, np.ones(dk.shape[1]))) <= 1.01e-6


def test_picard_variant_stalls_above_newton(torch, L, ctx, c1):
    """Fixed-point variant (eq. picard_matrix1): X itself is truncated, so its
    residual stalls near the oracle's fixed-point run (4.3e-3 on this
    problem), far above the Newton variant's (Sec. 5.3: at least 10x)."""
    K, d, f, _ = c1
    say("picard vs newton")
    ops = L.Operators(ctx, K)
    kw = dict(rank_cap=10, trunc_tol=1e-8, res_tol=1e-6, max_iter=40)
    c_n, p_n, i_n, _ = L.newton_subsets(ops, d, 1, f, **kw)
    c_p, p_p, i_p, _ = L.newton_subsets(ops, d, 1, f, picard=True, **kw)
    m = d.shape[1]
    dbar = och.mean_parameters(d)
    c, dc = och.chebyshev_interval(d, dbar)
    ref = np.linalg.norm(f) * np.sqrt(m)
    S, info = och.chebyshev_t(K, d, (f[:, None], np.eye(1), np.ones((m, 1))),
                              och.DirectPreconditioner(och.mean_preconditioner(K, dbar)), c, dc,
                              10, 1e-8, 1e-6, ref, max_iter=40)
    orc = info.history[-1] / ref
    say("newton", i_n[0]["relres"], "picard", i_p[0]["relres"], "oracle picard", orc)
    assert c_n == 0 and i_n[0]["relres"] <= 1e-6
    assert c_p == L.LRC_ENOTCONV and i_p[0]["iters"] == 40
    assert i_p[0]["relres"] >= 10 * i_n[0]["relres"]
    assert orc / 3 <= i_p[0]["relres"] <= 3 * orc
    Xp = _dense(p_p[0])
    assert abs(olr.relres_dense(K, d, Xp, np.outer(f, np.ones(m))) - i_p[0]["relres"]) <= \
        1e-3 * i_p[0]["relres"]
