"""Pins of the GMREST oracle (oracle/gmrest.py): without truncation it is
GMRES, whose least-squares residual after j steps is the minimum of
||r0 - A_p z|| over the j-dimensional Krylov space of the preconditioned
Kronecker operator, computed here by brute force; a restart longer than the
problem's dimension solves it exactly; and the low-rank inner product is the
Frobenius inner product of the dense matrices."""
import numpy as np
import scipy.sparse as sp

from oracle import chebyshev as och
from oracle import gmrest as ogm
from oracle import lowrank as olr
from workloads import param_table, three_term_2d


def _tiny():
    ops = three_term_2d(4)
    K = ops.K
    d = param_table(np.array([0.6, 1.0, 1.4, 1.9, 0.8]) * 1e4, np.array([1.1, 2.0, 3.9, 1.5, 2.5]) * 1e4)
    f = np.random.default_rng(5).standard_normal(ops.n)
    return K, d, f


def test_inner_product_is_frobenius():
    rng = np.random.default_rng(1)
    X = (rng.standard_normal((30, 4)), rng.uniform(0.1, 2, 4), rng.standard_normal((9, 4)))
    Y = (rng.standard_normal((30, 6)), rng.uniform(0.1, 2, 6), rng.standard_normal((9, 6)))
    Xd = X[0] @ np.diag(X[1]) @ X[2].T
    Yd = Y[0] @ np.diag(Y[1]) @ Y[2].T
    assert np.isclose(ogm.inner(X, Y), np.sum(Xd * Yd), rtol=1e-13)


def test_untruncated_gmrest_is_minimal_residual_over_krylov_space():
    K, d, f = _tiny()
    n, m = K[0].shape[0], d.shape[1]
    P = och.mean_preconditioner(K, och.mean_parameters(d))
    Pi = np.linalg.inv(P.toarray())
    Ap = np.kron(np.eye(m), Pi) @ olr.kron_operator(K, d)
    B = (f[:, None], np.eye(1), np.ones((m, 1)))
    r0 = np.kron(np.ones(m), Pi @ f)
    _, info = ogm.gmrest(K, d, B, och.DirectPreconditioner(P), m, 0.0, 1e-30,
                         np.linalg.norm(f) * np.sqrt(m), restart=6, max_iter=6)
    Kr = [r0]
    for j in range(1, 7):
        basis = np.column_stack(Kr)
        z, *_ = np.linalg.lstsq(Ap @ basis, r0, rcond=None)
        best = np.linalg.norm(r0 - Ap @ basis @ z)
        assert np.isclose(info.estimates[j - 1], best, rtol=1e-6, atol=1e-12 * np.linalg.norm(r0))
        Kr.append(Ap @ Kr[-1])


def test_gmrest_reaches_tolerance_and_matches_direct_solve():
    ops = three_term_2d(17)
    K = ops.K
    d = param_table(np.linspace(0.8, 1.6, 12) * 1e4, np.linspace(1.5, 3.0, 12) * 1e4)
    f = np.random.default_rng(2).standard_normal(ops.n)
    m = d.shape[1]
    P = och.mean_preconditioner(K, och.mean_parameters(d))
    ref = np.linalg.norm(f) * np.sqrt(m)
    S, info = ogm.gmrest(K, d, (f[:, None], np.eye(1), np.ones((m, 1))),
                         och.DirectPreconditioner(P), 12, 1e-14, 1e-10, ref)
    assert info.converged
    X = olr.lr_dense(S[0], np.diag(S[1]), S[2])
    Xs = olr.solve_columns(K, d, np.outer(f, np.ones(m)))
    assert olr.relres_dense(K, d, X, np.outer(f, np.ones(m))) <= 1e-10
    assert np.linalg.norm(X - Xs) <= 1e-6 * np.linalg.norm(Xs)
