"""Pins of the theta-scheme oracle (oracle/timedep.py, paper Sec. 4.3), each
fixed by something other than the oracle's own formula: the textbook
amplification factor of the theta-scheme on a scalar decay equation, the
steady state reached by the implicit Euler limit (the stationary column-wise
solve), second-order accuracy of Crank-Nicolson, and the low-rank steps
against the column-wise definition on a small problem."""
import numpy as np
import scipy.sparse as sp

from oracle import lowrank as olr
from oracle import timedep as otd
from workloads import param_table, three_term_2d


def _diag_problem(n=5, m=4, seed=0):
    rng = np.random.default_rng(seed)
    K = [sp.diags(rng.uniform(1.0, 2.0, n)).tocsr() for _ in range(3)]
    d = param_table(rng.uniform(0.5, 2.0, m), rng.uniform(0.5, 2.0, m))
    M = sp.diags(rng.uniform(0.5, 1.5, n)).tocsr()
    return K, M, d


def test_amplification_factor_on_scalar_decay():
    """m x' + a x = 0: each step multiplies by (1 - (1 - theta) a dt / m) /
    (1 + theta a dt / m) (theta = 1: implicit Euler, 1/2: Crank-Nicolson)."""
    K, M, d = _diag_problem()
    n, m = K[0].shape[0], d.shape[1]
    X0 = np.random.default_rng(1).standard_normal((n, m))
    a = np.column_stack([sum(d[i, j] * K[i].diagonal() for i in range(3)) for j in range(m)])
    mm = M.diagonal()[:, None]
    for theta in (1.0, 0.5, 0.25):
        dt = 0.3
        Xs = otd.theta_exact(K, M, d, [np.zeros(n)] * 4, X0, theta, dt)
        R = (1 - (1 - theta) * a * dt / mm) / (1 + theta * a * dt / mm)
        for i, X in enumerate(Xs):
            assert np.allclose(X, R ** i * X0, rtol=1e-13, atol=0)


def test_implicit_euler_long_step_is_the_stationary_solve():
    """theta = 1 with dt -> infinity drops the mass term: one step solves
    A_j x = b column by column (the stationary problem of Sec. 3.4)."""
    ops = three_term_2d(9)
    K = ops.K
    d = param_table(np.array([0.6e4, 1.1e4, 1.9e4]), np.array([1.2e4, 3.5e4, 2.0e4]))
    M = sp.identity(ops.n, format="csr") * (1.0 / (10) ** 2)
    b = np.random.default_rng(2).standard_normal(ops.n)
    X1 = otd.theta_exact(K, M, d, [b, b], np.zeros((ops.n, 3)), 1.0, 1e14)[1]
    Xs = olr.solve_columns(K, d, np.outer(b, np.ones(3)))
    assert np.linalg.norm(X1 - Xs) <= 1e-9 * np.linalg.norm(Xs)


def test_crank_nicolson_is_second_order():
    """Against the exact exponential of the scalar decay equation, halving dt
    divides the theta = 1/2 error by 4 (and the implicit Euler error by 2)."""
    K, M, d = _diag_problem(n=3, m=2, seed=3)
    n, m = 3, 2
    X0 = np.ones((n, m))
    a = np.column_stack([sum(d[i, j] * K[i].diagonal() for i in range(3)) for j in range(m)])
    T = 0.5
    exact = np.exp(-a / M.diagonal()[:, None] * T) * X0
    for theta, order in ((0.5, 2), (1.0, 1)):
        errs = []
        for steps in (20, 40):
            X = otd.theta_exact(K, M, d, [np.zeros(n)] * (steps + 1), X0, theta, T / steps)[-1]
            errs.append(np.abs(X - exact).max())
        assert abs(errs[0] / errs[1] - 2 ** order) < 0.1 * 2 ** order


def test_lowrank_steps_match_columnwise_definition():
    """With the exact operator history and tight tolerances the low-rank steps
    reproduce the column-wise theta-scheme; with theta = 1 the rank-q median
    history is the same thing (its (1 - theta) term vanishes)."""
    ops = three_term_2d(17)
    K = ops.K
    mu = np.linspace(0.8, 1.6, 6) * 1e4
    lam = np.linspace(1.5, 3.0, 6) * 1e4
    d = param_table(mu, lam)
    h = 1.0 / 18
    M = sp.identity(ops.n, format="csr") * h * h
    f = np.random.default_rng(4).standard_normal(ops.n)
    b = [f * (1 + 0.5 * np.sin(2 * np.pi * 0.05 * i)) for i in range(4)]
    m = d.shape[1]
    X0 = np.zeros((ops.n, m))
    for theta in (0.5, 1.0):
        ex = otd.theta_exact(K, M, d, b, X0, theta, 0.05)
        lrs = otd.theta_lowrank(K, M, d, b, [(np.zeros((ops.n, 1)), np.eye(1), np.ones((m, 1)))],
                                theta, 0.05, 20, 1e-13, 1e-12, history="exact")
        for i, st in enumerate(lrs, 1):
            X = sum(olr.lr_dense(*t) for t in st["terms"])
            assert np.linalg.norm(X - ex[i]) <= 1e-8 * np.linalg.norm(ex[i]), (theta, i)
    lrm = otd.theta_lowrank(K, M, d, b, [(np.zeros((ops.n, 1)), np.eye(1), np.ones((m, 1)))],
                            1.0, 0.05, 20, 1e-13, 1e-12, history="median")
    for i, st in enumerate(lrm, 1):
        X = sum(olr.lr_dense(*t) for t in st["terms"])
        assert np.linalg.norm(X - ex[i]) <= 1e-8 * np.linalg.norm(ex[i])
