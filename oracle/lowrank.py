"""Plain definitions: the matrix-equation operator, exact solves, residual, truncation.

Notation (paper Sec. 3.4, eq. newton_matrix1 and eq. newtonstep_vectornot1):
the unknown X is n x m, one column per parameter; the operator is

    L(X) = sum_i K_i X D_i,   D_i = diag(d[i, :]),

and the equation is L(X) = F.  Because every D_i is diagonal, the vector
(Kronecker) form  (sum_i D_i (x) K_i) vec(X) = vec(F)  is block diagonal, so
column j solves the single system  A_j x_j = f_j  with  A_j = sum_i d[i, j] K_i.

Low-rank matrices are triples (A, C, B) meaning  A @ C @ B.T  (A: n x k,
C: k x k, B: m x k).  A truncated result is returned as (U, s, V) with
orthonormal U, V and non-increasing s >= 0, meaning U @ diag(s) @ V.T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# --------------------------------------------------------------------------- operator
def column_operator(K, d, j):
    """A_j = sum_i d[i, j] K_i  (the system matrix of parameter column j)."""
    A = d[0, j] * K[0]
    for i in range(1, len(K)):
        A = A + d[i, j] * K[i]
    return sp.csr_matrix(A)


def apply_L_dense(K, d, X):
    """L(X) = sum_i K_i X D_i for a dense X (n x m)."""
    Y = np.zeros_like(X, dtype=np.float64)
    for i, Ki in enumerate(K):
        Y += (Ki @ X) * d[i][None, :]
    return Y


def kron_operator(K, d):
    """The vector form  sum_i D_i (x) K_i  as a dense (n m) x (n m) array."""
    mats = [np.kron(np.diag(d[i]), Ki.toarray()) for i, Ki in enumerate(K)]
    return np.sum(mats, axis=0)


def vec(X):
    """Column stacking (paper Sec. 3.4, Definition 'Vectorization')."""
    return np.asarray(X).reshape(-1, order="F")


def unvec(x, n):
    return np.asarray(x).reshape(n, -1, order="F")


def solve_kron(K, d, F):
    """Exact solution from the dense vector form (tiny problems only)."""
    n = K[0].shape[0]
    return unvec(np.linalg.solve(kron_operator(K, d), vec(F)), n)


def solve_columns(K, d, F):
    """Exact solution column by column with sparse LU (SuperLU, partial pivoting)."""
    n, m = F.shape
    X = np.empty((n, m))
    for j in range(m):
        X[:, j] = spla.splu(sp.csc_matrix(column_operator(K, d, j))).solve(F[:, j])
    return X


# --------------------------------------------------------------------------- low rank
def lr_dense(A, C, B):
    return A @ C @ B.T


def lr_L(K, d, U, s, V):
    """L(U diag(s) V^T) in factored form:
    [K_0 U | ... | K_{q-1} U] blkdiag(diag(s), ...) [D_0 V | ... | D_{q-1} V]^T."""
    A = np.hstack([Ki @ U for Ki in K])
    C = sla.block_diag(*([np.diag(s)] * len(K)))
    B = np.hstack([d[i][:, None] * V for i in range(len(K))])
    return A, C, B


def lr_sum(*terms):
    """Sum of factored terms (A_t, C_t, B_t) by concatenation of the factors."""
    A = np.hstack([t[0] for t in terms])
    C = sla.block_diag(*[t[1] for t in terms])
    B = np.hstack([t[2] for t in terms])
    return A, C, B


def lr_scale(t, alpha):
    return t[0], alpha * t[1], t[2]


def usv(U, s, V):
    return U, np.diag(s), V


def truncate(A, C, B, rank_cap, tol):
    """Truncation T_{R,eps}(A C B^T): QR of both factors, SVD of the small core,
    then keep r' = min(R, smallest r whose discarded singular values have
    Frobenius norm <= eps * ||core||_F).  For a matrix (an order-2 tensor) this
    is the truncated SVD that Tucker truncation reduces to (paper Sec. 5, the
    truncation operator realised with the htucker toolbox).  Zero input gives
    rank 0.
    """
    n, m = A.shape[0], B.shape[0]
    if A.shape[1] == 0:
        return np.zeros((n, 0)), np.zeros(0), np.zeros((m, 0))
    QA, RA = np.linalg.qr(A)
    QB, RB = np.linalg.qr(B)
    core = RA @ C @ RB.T
    Uc, sig, Vct = np.linalg.svd(core)
    r = truncation_rank(sig, rank_cap, tol)
    return QA @ Uc[:, :r], sig[:r].copy(), QB @ Vct[:r].T


def truncation_rank(sig, rank_cap, tol):
    """Smallest r with sqrt(sum_{j >= r} sig_j^2) <= tol * ||sig||, capped."""
    total = np.sqrt(np.sum(sig ** 2))
    if total == 0.0:
        return 0
    tail = np.sqrt(np.maximum(np.cumsum((sig ** 2)[::-1])[::-1], 0.0))   # tail[r] = ||sig[r:]||
    tail = np.append(tail, 0.0)
    r = int(np.argmax(tail <= tol * total))
    return min(r, int(rank_cap))


# --------------------------------------------------------------------------- residual
def relres_dense(K, d, X, F):
    """||F - L(X)||_F / ||F||_F (paper Sec. 5.1 reports the same quotient per column)."""
    R = F - apply_L_dense(K, d, X)
    return np.linalg.norm(R) / np.linalg.norm(F)


def residual_lowrank(K, d, F_terms, X_terms, block=64, per_column=False):
    """Frobenius norm of F - L(X) computed entry by entry in column blocks.

    F and X are each a list of factored terms (A, C, B).  Column j of the
    residual is  F[:, j] - sum_i d[i, j] K_i X[:, j];  it is formed explicitly
    (no Gram-trace shortcut) so that no cancellation hides a small residual.
    Returns ||R||_F and, with ``per_column``, the vector of ||R[:, j]||_2.
    """
    m = d.shape[1]
    W = [[Ki @ t[0] for Ki in K] for t in X_terms]            # K_i A_t, n x k_t
    sq = np.zeros(m)
    for j0 in range(0, m, block):
        J = slice(j0, min(m, j0 + block))
        R = np.zeros((K[0].shape[0], J.stop - J.start))
        for (A, C, B) in F_terms:
            R += A @ (C @ B[J].T)
        for t, (A, C, B) in enumerate(X_terms):
            Y = C @ B[J].T                                     # k_t x |J|
            for i in range(len(K)):
                R -= (W[t][i] @ Y) * d[i, J][None, :]
        sq[J] = np.sum(R * R, axis=0)
    if per_column:
        return np.sqrt(np.sum(sq)), np.sqrt(sq)
    return np.sqrt(np.sum(sq))


def fro_lowrank(A, C, B):
    """||A C B^T||_F without forming the product (QR of both factors)."""
    if A.shape[1] == 0:
        return 0.0
    _, RA = np.linalg.qr(A)
    _, RB = np.linalg.qr(B)
    return np.linalg.norm(RA @ C @ RB.T)


def storage_bytes_lowrank(M, m, R, bytes_per=8):
    """Storage of a rank-R factorisation O((M + m + R) R) (paper Table 1)."""
    return (M + m + R) * R * bytes_per


def storage_bytes_full(M, m, bytes_per=8):
    return M * m * bytes_per
