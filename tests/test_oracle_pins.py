"""Pins of the FP64 oracle against facts fixed outside the oracle itself:
values printed in the paper, closed forms, library routines and brute force.
CPU only."""
import json
import os

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import chebyshev as ch
from oracle import driver
from oracle import lowrank as lr
from workloads import config, param_table, three_term_2d, grid_params_little_endian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ clustering (Sec. 3.3)
def test_paper_clustering_example():
    g = json.load(open(os.path.join(GOLDEN, "clustering_example.json")))
    m1, m2, K = g["m1"], g["m2"], g["K"]
    m = m1 * m2
    subs = driver.subsets(m, K)
    assert [len(s) for s in subs] == [len(s) for s in g["subsets"]]
    for J, members, med in zip(subs, g["subsets"], g["upper_median"]):
        got = [list(driver.multi_index(p + 1, m1)) for p in J]
        assert got == members
        assert list(driver.multi_index(J[driver.upper_median_offset(len(J))] + 1, m1)) == med


@pytest.mark.parametrize("m,K", [(20, 3), (5000, 50), (2000, 16), (7, 7), (101, 10)])
def test_subset_sizes_formula(m, K):
    s = driver.subset_sizes(m, K)
    assert len(s) == K and sum(s) == m
    assert all(x == m // K for x in s[:-1])


def test_little_endian_roundtrip():
    m1, m2 = 7, 5
    for i2 in range(1, m2 + 1):
        for i1 in range(1, m1 + 1):
            p = driver.little_endian_position(i1, i2, m1)
            assert driver.multi_index(p, m1) == (i1, i2)
    mu, lam = grid_params_little_endian(np.arange(1, m1 + 1), np.arange(1, m2 + 1) * 10)
    for p in range(1, m1 * m2 + 1):
        i1, i2 = driver.multi_index(p, m1)
        assert mu[p - 1] == i1 and lam[p - 1] == 10 * i2


def test_table1_storage():
    g = json.load(open(os.path.join(GOLDEN, "table1_storage.json")))
    mib = 2.0 ** 20
    assert round(lr.storage_bytes_lowrank(g["M"], g["m"], g["R"]) / mib, 2) == g["lowrank_mib"]
    assert round(lr.storage_bytes_full(g["M"], g["m"]) / mib, 2) == g["full_mib"]


# ------------------------------------------------------------------ plain definition
def _tiny(N=5, m=6, seed=0):
    ops = three_term_2d(N)
    rng = np.random.default_rng(seed)
    d = param_table(rng.uniform(0.5, 2, m), rng.uniform(1, 4, m))
    F = rng.standard_normal((ops.n, m))
    return ops.K, d, F


def test_kronecker_form_matches_matrix_form():
    K, d, F = _tiny()
    X = np.random.default_rng(1).standard_normal(F.shape)
    lhs = lr.kron_operator(K, d) @ lr.vec(X)
    rhs = lr.vec(lr.apply_L_dense(K, d, X))
    assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-12)
    # brute force: entry by entry from the definition sum_i K_i X D_i
    n, m = F.shape
    Kd = [Ki.toarray() for Ki in K]
    Y = np.zeros((n, m))
    for i in range(len(K)):
        for a in range(n):
            for j in range(m):
                Y[a, j] += sum(Kd[i][a, b] * X[b, j] for b in range(n)) * d[i, j]
    assert np.allclose(Y, lr.apply_L_dense(K, d, X), rtol=1e-13, atol=1e-12)


def test_kron_solve_equals_columnwise_solve():
    K, d, F = _tiny()
    X1 = lr.solve_kron(K, d, F)
    X2 = lr.solve_columns(K, d, F)
    assert np.allclose(X1, X2, rtol=1e-10, atol=1e-12)
    assert lr.relres_dense(K, d, X1, F) < 1e-13


def test_diagonal_operators_closed_form():
    rng = np.random.default_rng(3)
    n, m, q = 9, 5, 3
    diags = [rng.uniform(1, 2, n) for _ in range(q)]
    K = [sp.diags(a).tocsr() for a in diags]
    d = np.vstack([np.ones(m), rng.uniform(1, 3, (q - 1, m))])
    F = rng.standard_normal((n, m))
    X = F / sum(np.outer(diags[i], d[i]) for i in range(q))
    assert np.allclose(lr.solve_columns(K, d, F), X, rtol=1e-13)


def test_single_term_keeps_rank_of_rhs():
    K, d, _ = _tiny()
    m = d.shape[1]
    d_eq = np.repeat(d[:, :1], m, axis=1)          # all columns share one parameter
    rng = np.random.default_rng(5)
    F = rng.standard_normal((K[0].shape[0], 2)) @ rng.standard_normal((2, m))
    X = lr.solve_columns(K, d_eq, F)
    A0 = lr.column_operator(K, d_eq, 0).toarray()
    assert np.allclose(X, np.linalg.solve(A0, F), rtol=1e-10, atol=1e-12)
    assert np.linalg.matrix_rank(X, tol=1e-10 * np.linalg.norm(X)) == 2


def test_residual_lowrank_matches_dense():
    K, d, F = _tiny(N=6, m=9)
    rng = np.random.default_rng(7)
    U, V = rng.standard_normal((36, 3)), rng.standard_normal((9, 3))
    C = np.diag([2.0, 1.0, 0.5])
    FU, FV = rng.standard_normal((36, 2)), rng.standard_normal((9, 2))
    Fd = FU @ FV.T
    X = U @ C @ V.T
    nr, cols = lr.residual_lowrank(K, d, [(FU, np.eye(2), FV)], [(U, C, V)], block=4,
                                   per_column=True)
    R = Fd - lr.apply_L_dense(K, d, X)
    assert np.isclose(nr, np.linalg.norm(R), rtol=1e-12)
    assert np.allclose(cols, np.linalg.norm(R, axis=0), rtol=1e-12)


# ------------------------------------------------------------------ truncation
@pytest.mark.parametrize("cap,tol", [(4, 0.0), (50, 1e-3), (3, 1e-1)])
def test_truncation_is_eckart_young(cap, tol):
    rng = np.random.default_rng(11)
    n, m, k = 40, 25, 12
    A, B = rng.standard_normal((n, k)), rng.standard_normal((m, k))
    C = rng.standard_normal((k, k)) @ np.diag(np.logspace(0, -6, k))
    M = A @ C @ B.T
    sig = np.linalg.svd(M, compute_uv=False)
    U, s, V = lr.truncate(A, C, B, cap, tol)
    r = s.size
    # rank rule: smallest r with tail <= tol*||sig||, capped
    tails = [np.sqrt(np.sum(sig[j:] ** 2)) for j in range(sig.size + 1)]
    r_expect = min(cap, next(j for j, t in enumerate(tails) if t <= tol * np.linalg.norm(sig)))
    assert r == r_expect
    assert np.allclose(s, sig[:r], rtol=1e-10)
    assert np.allclose(U.T @ U, np.eye(r), atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(r), atol=1e-12)
    err = np.linalg.norm(M - U @ np.diag(s) @ V.T)
    assert np.isclose(err, tails[r], rtol=1e-6, atol=1e-12 * np.linalg.norm(sig))


def test_truncation_of_zero_is_rank_zero():
    U, s, V = lr.truncate(np.zeros((5, 2)), np.eye(2), np.zeros((4, 2)), 3, 1e-8)
    assert s.size == 0 and U.shape == (5, 0) and V.shape == (4, 0)


# ------------------------------------------------------------------ ChebyshevT
def _diag_problem(n=12, m=7, seed=2):
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(1, 2, n), rng.uniform(0.5, 1.5, n)
    K = [sp.diags(a).tocsr(), sp.diags(b).tocsr()]
    d = np.vstack([np.ones(m), rng.uniform(0.6, 1.4, m)])
    return K, d, rng


FORMS = {"direction": ch.chebyshev_t, "three_term": ch.chebyshev_t3}


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_chebyshev_residual_is_scaled_chebyshev_polynomial(k, form):
    """Without truncation the residual of every eigencomponent is
    T_k((d - lam)/c) / T_k(d/c) times the initial one (Chebyshev acceleration),
    in the direction form and in the three-term form alike."""
    K, d, rng = _diag_problem()
    n, m = K[0].shape[0], d.shape[1]
    dbar = d.mean(axis=1)
    P = ch.mean_preconditioner(K, dbar)
    lam = np.array([[(K[0][p, p] + d[1, j] * K[1][p, p]) / P[p, p] for j in range(m)]
                    for p in range(n)])
    c, dc = 0.5 * (lam.max() - lam.min()) * 1.05, 0.5 * (lam.max() + lam.min())
    B = (rng.standard_normal((n, 2)), np.eye(2), rng.standard_normal((m, 2)))
    S, info = FORMS[form](K, d, B, ch.DirectPreconditioner(P), c, dc, rank_cap=1000,
                          trunc_tol=0.0, res_tol=0.0, ref_norm=1.0, restart=0, max_iter=k)
    assert info.iters == k
    R0 = lr.lr_dense(*B)
    Rk = R0 - lr.apply_L_dense(K, d, lr.lr_dense(*lr.usv(*S)))
    e = np.zeros(k + 1)
    e[k] = 1.0
    poly = npcheb.chebval((dc - lam) / c, e) / npcheb.chebval(dc / c, e)
    assert np.allclose(Rk, poly * R0, rtol=1e-9, atol=1e-12 * np.abs(R0).max())


@pytest.mark.parametrize("form", sorted(FORMS))
def test_chebyshev_exact_preconditioner_converges_in_one_step(form):
    K, d, rng = _diag_problem()
    m = d.shape[1]
    d = np.repeat(d[:, :1], m, axis=1)                 # every column equals the mean
    P = ch.mean_preconditioner(K, d.mean(axis=1))
    B = (rng.standard_normal((K[0].shape[0], 2)), np.eye(2), rng.standard_normal((m, 2)))
    S, info = FORMS[form](K, d, B, ch.DirectPreconditioner(P), 0.5, 1.0, 100, 1e-14,
                          1e-12, 1.0, restart=0, max_iter=5)
    assert info.iters == 1 and info.converged


def test_chebyshev_interval_encloses_dense_spectrum():
    ops = three_term_2d(13)
    mu, lam = grid_params_little_endian(np.linspace(0.5, 2, 4) * 1e4, np.linspace(1, 4, 4) * 1e4)
    d = param_table(mu, lam)
    dbar = ch.mean_parameters(d)
    c, dc = ch.chebyshev_interval(d, dbar)
    P = ch.mean_preconditioner(ops.K, dbar).toarray()
    for j in range(d.shape[1]):
        A = lr.column_operator(ops.K, d, j).toarray()
        ev = sla.eigvals(A, P)
        assert np.all(ev.real >= dc - c - 1e-8) and np.all(ev.real <= dc + c + 1e-8)
        assert np.max(np.abs(ev.imag)) < 1e-3


def test_c1_interval_value():
    cfg = config("c1")
    c, dc = ch.chebyshev_interval(cfg["d"], ch.mean_parameters(cfg["d"]))
    assert np.isclose(c, 0.6) and np.isclose(dc, 1.0)


def test_planted_low_rank_solution_is_recovered():
    ops = three_term_2d(17)
    rng = np.random.default_rng(21)
    m, r = 30, 4
    d = param_table(rng.uniform(0.5, 2, m), rng.uniform(0.5, 2, m))   # O(1)-conditioned
    Us, _ = np.linalg.qr(rng.standard_normal((ops.n, r)))
    Vs, _ = np.linalg.qr(rng.standard_normal((m, r)))
    ss = np.array([3.0, 1.0, 0.3, 0.1])
    B = lr.lr_L(ops.K, d, Us, ss, Vs)
    dbar = ch.mean_parameters(d)
    c, dc = ch.chebyshev_interval(d, dbar)
    ref = lr.fro_lowrank(*B)
    S, info = ch.chebyshev_t(ops.K, d, B, ch.DirectPreconditioner(ch.mean_preconditioner(ops.K, dbar)),
                             c, dc, rank_cap=12, trunc_tol=1e-10, res_tol=1e-12, ref_norm=ref,
                             max_iter=200)
    assert info.converged
    X = lr.lr_dense(*lr.usv(*S))
    Xs = Us @ np.diag(ss) @ Vs.T
    assert np.linalg.norm(X - Xs) / np.linalg.norm(Xs) < 1e-9
    sv = np.linalg.svd(X, compute_uv=False)
    assert np.sum(sv > 1e-8 * sv[0]) == r


def test_mean_parameters_asymmetric_table():
    """On a skewed table the arithmetic mean (the configured centre) and the
    midrange (Sec. 4.2) differ; both are worked out by hand."""
    d = np.array([[1.0, 1.0, 1.0, 1.0], [1.0, 2.0, 3.0, 10.0], [4.0, 4.0, 5.0, 7.0]])
    assert np.allclose(ch.mean_parameters(d), [1.0, 4.0, 5.0], rtol=0, atol=1e-15)
    assert np.allclose(ch.mean_parameters(d, "midrange"), [1.0, 5.5, 5.5], rtol=0, atol=1e-15)


def test_chebyshev_interval_asymmetric_table_hand_values():
    """Interval from the ratios d_ij / dbar_i and 1 (hand-computed): with the
    means (1, 4, 5) the ratios span [1/4, 10/4], so c = 1.125, d = 1.375."""
    d = np.array([[1.0, 1.0, 1.0, 1.0], [1.0, 2.0, 3.0, 10.0], [4.0, 4.0, 5.0, 7.0]])
    c, dc = ch.chebyshev_interval(d, ch.mean_parameters(d))
    assert np.isclose(c, 1.125, rtol=1e-15) and np.isclose(dc, 1.375, rtol=1e-15)


def test_chebyshev_interval_skewed_grid_encloses_dense_spectrum():
    """A parameter grid clustered at one end (mean far from the midrange): the
    interval built from the mean preconditioner encloses every column's dense
    generalised spectrum, and its ends are attained to within 10%."""
    ops = three_term_2d(13)
    mu, lam = grid_params_little_endian(np.array([0.5, 0.55, 0.6, 2.0]) * 1e4,
                                        np.array([1.0, 1.1, 4.0]) * 1e4)
    d = param_table(mu, lam)
    dbar = ch.mean_parameters(d)
    assert not np.allclose(dbar, ch.mean_parameters(d, "midrange"))
    c, dc = ch.chebyshev_interval(d, dbar)
    P = ch.mean_preconditioner(ops.K, dbar).toarray()
    lo, hi = np.inf, -np.inf
    for j in range(d.shape[1]):
        ev = sla.eigvals(lr.column_operator(ops.K, d, j).toarray(), P)
        assert np.all(ev.real >= dc - c - 1e-8) and np.all(ev.real <= dc + c + 1e-8)
        lo, hi = min(lo, ev.real.min()), max(hi, ev.real.max())
    assert hi >= dc + c - 0.1 * 2 * c and lo <= dc - c + 0.1 * 2 * c


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("iters", [4, 5])
def test_chebyshev_restart_is_product_of_polynomials(iters, form):
    """Restarting every 2 updates without truncation: the recurrence starts
    again from the current iterate, so after cycles of lengths l_1, l_2, ...
    each eigencomponent's residual is the product of the scaled Chebyshev
    polynomials T_l((d - lam)/c) / T_l(d/c) of the cycles."""
    K, d, rng = _diag_problem(seed=4)
    n, m = K[0].shape[0], d.shape[1]
    dbar = d.mean(axis=1)
    P = ch.mean_preconditioner(K, dbar)
    lam = np.array([[(K[0][p, p] + d[1, j] * K[1][p, p]) / P[p, p] for j in range(m)]
                    for p in range(n)])
    c, dc = 0.5 * (lam.max() - lam.min()) * 1.1, 0.5 * (lam.max() + lam.min())
    B = (rng.standard_normal((n, 2)), np.eye(2), rng.standard_normal((m, 2)))
    S, info = FORMS[form](K, d, B, ch.DirectPreconditioner(P), c, dc, rank_cap=1000,
                          trunc_tol=0.0, res_tol=0.0, ref_norm=1.0, restart=2,
                          max_iter=iters)
    assert info.iters == iters
    R0 = lr.lr_dense(*B)
    Rk = R0 - lr.apply_L_dense(K, d, lr.lr_dense(*lr.usv(*S)))

    def p(l):
        e = np.zeros(l + 1)
        e[l] = 1.0
        return npcheb.chebval((dc - lam) / c, e) / npcheb.chebval(dc / c, e)

    poly = p(2) * p(2) * (p(1) if iters == 5 else 1.0)
    assert np.allclose(Rk, poly * R0, rtol=1e-9, atol=1e-12 * np.abs(R0).max())
    # a single unrestarted cycle of the same length gives a different residual
    assert not np.allclose(poly, p(iters), rtol=1e-3)


def test_three_term_form_truncates_once_per_update_and_tracks_direction_form():
    """With truncation the forms differ only by where the truncation errors
    enter: on c1 (tolerance 1e-8) both reach the target in the same number of
    updates with residual histories within a few per cent and nearly the
    same iterate, each applying the preconditioner once per update."""
    cfg = config("c1")
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    jmed = driver.upper_median_offset(m)
    xt = sla.lu_solve(sla.lu_factor(lr.column_operator(K, d, jmed).toarray()), f)
    B = driver.median_rhs(K, d, f, xt)
    dbar = ch.mean_parameters(d)
    c, dc = ch.chebyshev_interval(d, dbar)
    P = ch.DirectPreconditioner(ch.mean_preconditioner(K, dbar))
    ref = np.linalg.norm(f) * np.sqrt(m)
    args = (K, d, B, P, c, dc, cfg["rank_cap"], cfg["trunc_tol"], cfg["res_tol"], ref)
    S2, i2 = ch.chebyshev_t(*args)
    S3, i3 = ch.chebyshev_t3(*args)
    assert i2.converged and i3.converged
    assert i3.iters == i2.iters
    h2, h3 = np.array(i2.history), np.array(i3.history)
    assert np.all(np.abs(h3 - h2) <= 0.05 * h2)
    assert i3.prec_applies == i3.iters == i2.prec_applies
    X2, X3 = lr.lr_dense(*lr.usv(*S2)), lr.lr_dense(*lr.usv(*S3))
    assert np.linalg.norm(X3 - X2) <= 1e-6 * np.linalg.norm(X2)


# ------------------------------------------------------------------ Newton driver
def test_median_rhs_equals_dense_definition_and_rank():
    K, d, _ = _tiny(N=6, m=8)
    f = np.random.default_rng(4).standard_normal(K[0].shape[0])
    xt = np.random.default_rng(5).standard_normal(K[0].shape[0])
    B = driver.median_rhs(K, d, f, xt)
    F = np.outer(f, np.ones(d.shape[1]))
    dense = F - lr.apply_L_dense(K, d, np.outer(xt, np.ones(d.shape[1])))
    assert np.allclose(lr.lr_dense(*B), dense, rtol=1e-12, atol=1e-12)
    assert np.linalg.matrix_rank(dense, tol=1e-10 * np.linalg.norm(dense)) <= 3


def test_c1_newton_subset_reaches_tolerance():
    cfg = config("c1")
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    res = driver.newton_subset(K, d, f, cfg["rank_cap"], cfg["trunc_tol"], cfg["res_tol"])
    assert res["info"].converged
    assert res["jmed"] == 50          # upper median of 100 columns, 0-based
    m = d.shape[1]
    F = [(f[:, None], np.eye(1), np.ones((m, 1)))]
    nr = lr.residual_lowrank(K, d, F, driver.solution_terms(res))
    relres = nr / (np.linalg.norm(f) * np.sqrt(m))
    assert relres <= 1.2e-8
    assert 10 <= res["info"].iters <= 25
    # the low-rank result agrees with the exact column-wise solution
    Xs = lr.solve_columns(K, d, np.outer(f, np.ones(m)))
    X = sum(lr.lr_dense(*t) for t in driver.solution_terms(res))
    kappa_bound = 1e-8 * 1e9          # error <= cond * relres; cond(A_j) ~ 1e8 here
    assert np.linalg.norm(X - Xs) / np.linalg.norm(Xs) < kappa_bound


def test_algorithm1_tiny_matches_direct_solves():
    ops = three_term_2d(9)
    mu, lam = grid_params_little_endian(np.linspace(0.5, 2, 5) * 1e4, np.linspace(1, 4, 4) * 1e4)
    d = param_table(mu, lam)
    f = np.random.default_rng(0).standard_normal(ops.n)
    out = driver.algorithm1(ops.K, d, f, 3, rank_cap=40, trunc_tol=1e-13, res_tol=1e-11)
    X = np.hstack([sum(lr.lr_dense(*t) for t in driver.solution_terms(r)) for r in out])
    Xs = lr.solve_columns(ops.K, d, np.outer(f, np.ones(d.shape[1])))
    assert lr.relres_dense(ops.K, d, X, np.outer(f, np.ones(d.shape[1]))) < 2e-11
    assert [len(r["cols"]) for r in out] == [6, 6, 8]
