"""GMREST: restarted GMRES with truncation for L(S) = B (paper Sec. 2.2 and
Sec. 4.1 name it next to ChebyshevT and cite the companion paper for it; it
is not printed here).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading: the classical restarted GMRES(l) (Saad, Iterative Methods for Sparse
Linear Systems, 2nd ed., Alg. 6.9 with restarts) on the left-preconditioned
operator Z -> P^-1 L(Z) (P acting on the left factor, I (x) P of Sec. 4.2) in
the Frobenius inner product, where every Krylov matrix is kept in low-rank
form and truncated after each operation:

    repeat:
      R  = T(B - L(S));  stop if ||R||_F <= tau ||F||_F        (explicit)
      V1 = T(P^-1 R);  beta = ||V1||_F;  V1 <- V1 / beta
      for j = 1..l:
        W = T(P^-1 T(L(V_j)))
        for i = 1..j:  h_ij = <V_i, W>_F;  W <- T(W - h_ij V_i)   (modified GS)
        h_{j+1,j} = ||W||_F;  V_{j+1} = W / h_{j+1,j}
        y_j = argmin_y || beta e_1 - H_j y ||  (Givens rotations; the small
              least-squares residual estimates ||P^-1 (B - L(S + V y))||)
        stop the cycle when that estimate <= beta tau ||F||_F / ||R||_F (the
        reduction the explicit residual still needs, carried over to the
        preconditioned one) or h_{j+1,j} = 0
      S <- T(S + sum_j y_j V_j)      (one truncation per term)

Inner products of low-rank matrices are formed from the factors,
<A1 C1 B1^T, A2 C2 B2^T>_F = sum over (A1^T A2) * (C1 (B1^T B2) C2^T).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import lowrank as lr
from .chebyshev import residual_factored


@dataclasses.dataclass
class GmresInfo:
    iters: int = 0               # Arnoldi steps (all cycles)
    cycles: int = 0
    converged: bool = False
    history: list = dataclasses.field(default_factory=list)   # ||B - L(S)||_F at each restart
    estimates: list = dataclasses.field(default_factory=list)  # preconditioned LS residuals
    prec_applies: int = 0


def inner(X, Y):
    """<X, Y>_F for X = (U1, s1, V1), Y = (U2, s2, V2) from the factors."""
    U1, s1, V1 = X
    U2, s2, V2 = Y
    if U1.shape[1] == 0 or U2.shape[1] == 0:
        return 0.0
    return float(np.sum((U1.T @ U2) * (np.diag(s1) @ (V1.T @ V2) @ np.diag(s2))))


def _axpy(a, X, Y, rank_cap, tol):
    """T(a X + Y) for truncated triples."""
    return lr.truncate(*lr.lr_sum(lr.lr_scale(lr.usv(*X), a), lr.usv(*Y)), rank_cap, tol)


def gmrest(K, d, B, prec, rank_cap, trunc_tol, res_tol, ref_norm, restart=6, max_iter=200,
           S0=None):
    """Solve L(S) = B approximately in low-rank form by GMREST.  Arguments as
    chebyshev.chebyshev_t (no spectrum interval is needed).  Returns
    ((U, s, V), GmresInfo)."""
    n, m = B[0].shape[0], B[2].shape[0]
    info = GmresInfo()
    S = (np.zeros((n, 0)), np.zeros(0), np.zeros((m, 0))) if S0 is None else S0

    def precond(X):
        info.prec_applies += 1
        U, s, V = X
        return lr.truncate(prec.solve(U), np.diag(s), V, rank_cap, trunc_tol)

    while True:
        R = lr.truncate(*residual_factored(K, d, B, S), rank_cap, trunc_tol)
        nr = float(np.linalg.norm(R[1]))
        info.history.append(nr)
        if nr <= res_tol * ref_norm or R[1].size == 0:
            info.converged = True
            return S, info
        if info.iters >= max_iter:
            return S, info
        info.cycles += 1
        Z = precond(R)
        beta = float(np.linalg.norm(Z[1]))
        if beta == 0.0:
            return S, info
        cyc_tol = beta * res_tol * ref_norm / nr
        Vs = [(Z[0], Z[1] / beta, Z[2])]
        H = np.zeros((restart + 1, restart))
        g = np.zeros(restart + 1)
        g[0] = beta
        cs, sn = np.zeros(restart), np.zeros(restart)
        y = np.zeros(0)
        for j in range(restart):
            Vj = Vs[j]
            LV = lr.truncate(*lr.lr_L(K, d, *Vj), rank_cap, trunc_tol)
            W = precond(LV)
            for i in range(j + 1):
                H[i, j] = inner(Vs[i], W)
                W = _axpy(-H[i, j], Vs[i], W, rank_cap, trunc_tol)
            H[j + 1, j] = float(np.linalg.norm(W[1]))
            info.iters += 1
            # Givens rotations keep the small least-squares problem triangular
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / rho, H[j + 1, j] / rho) if rho > 0 else (1.0, 0.0)
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1])
            info.estimates.append(est)
            y = np.linalg.solve(np.triu(H[:j + 1, :j + 1]), g[:j + 1]) if j + 1 else y
            hn = np.linalg.norm(W[1])
            if est <= cyc_tol or hn == 0.0 or info.iters >= max_iter or j == restart - 1:
                break
            Vs.append((W[0], W[1] / hn, W[2]))
        for jj, yj in enumerate(y):
            S = _axpy(yj, Vs[jj], S, rank_cap, trunc_tol)
