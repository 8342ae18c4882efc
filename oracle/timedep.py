"""The theta-scheme in time over a parameter subset (paper Sec. 4.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Linear stand-in of the time-dependent problem: for every parameter column j,

    M x_j'(t) + A_j x_j(t) = b(t),        A_j = sum_i d[i, j] K_i,

with a mass matrix M (the paper's rho_f A_t^f + rho_s A_t^s).  The theta-scheme
with step dt gives per column (the linear case of eq. time_indiv1)

    (M / dt + theta A_j) x_j^i = (M / dt - (1 - theta) A_j) x_j^{i-1}
                                 + theta b^i + (1 - theta) b^{i-1}.

``theta_exact`` is this definition solved column by column (SuperLU).

``theta_lowrank`` follows eq. timedep_matrix1: at step i the upper-median
column's theta step gives x~^i, and the update S^i of the subset solves

    L_theta(S) = F_i - L_theta(x~^i 1^T),
    L_theta(S) = (1/dt) M S + theta sum_k K_k S D_k,
    F_i = theta b^i 1^T + (1 - theta) b^{i-1} 1^T + (1/dt) M X^{i-1} - (1 - theta) G,

with X^i = x~^i 1^T + S^i.  G is the previous step's operator term: exactly
L(X^{i-1}) (``history="exact"``), or, as the paper's remark on the right-hand
side suggests, L(x~^{i-1} 1^T), which has rank <= q (``history="median"``).
Both coincide for theta = 1.  L_theta is the generic q-term operator with
K'_0 = M/dt + theta K_0 and K'_k = theta K_k, so the same ChebyshevT and
preconditioner (Sec. 4.2, centre parameters) apply unchanged.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import chebyshev as ch
from . import driver as dr
from . import lowrank as lr


def theta_operators(K, M, theta, dt):
    """K' of L_theta: [M/dt + theta K_0, theta K_1, ...]."""
    return [sp.csr_matrix(M / dt + theta * K[0])] + [sp.csr_matrix(theta * Ki) for Ki in K[1:]]


def theta_exact(K, M, d, b, X0, theta, dt):
    """Column-wise theta steps.  b: list of load vectors b^0..b^w (n each);
    X0: dense n x m initial value.  Returns [X^0, X^1, ..., X^w]."""
    m = d.shape[1]
    Xs = [np.array(X0, dtype=np.float64)]
    lus = []
    for j in range(m):
        A = lr.column_operator(K, d, j)
        lus.append((spla.splu(sp.csc_matrix(M / dt + theta * A)),
                    sp.csr_matrix(M / dt - (1.0 - theta) * A)))
    for i in range(1, len(b)):
        Xp = Xs[-1]
        Xn = np.empty_like(Xp)
        for j, (lu, B) in enumerate(lus):
            Xn[:, j] = lu.solve(B @ Xp[:, j] + theta * b[i] + (1.0 - theta) * b[i - 1])
        Xs.append(Xn)
    return Xs


def step_rhs(K, M, d, b_i, b_prev, X_terms, xt_prev, theta, dt, history):
    """F_i of eq. timedep_matrix1 as a list of factored terms (A, C, B)."""
    m = d.shape[1]
    ones = np.ones((m, 1))
    terms = [((theta * b_i + (1.0 - theta) * b_prev)[:, None], np.eye(1), ones)]
    for (A, C, B) in X_terms:                       # (1/dt) M X^{i-1}
        terms.append((M @ A / dt, C, B))
    if theta < 1.0:
        if history == "exact":
            for (A, C, B) in X_terms:                   # -(1 - theta) L(X^{i-1})
                for k, Kk in enumerate(K):
                    terms.append((Kk @ A, -(1.0 - theta) * C, d[k][:, None] * B))
        elif history == "median":
            for k, Kk in enumerate(K):                  # -(1 - theta) L(x~^{i-1} 1^T)
                terms.append(((Kk @ xt_prev)[:, None], -(1.0 - theta) * np.eye(1), d[k][:, None]))
        else:
            raise ValueError(history)
    return terms


def theta_lowrank(K, M, d, b, X0_terms, theta, dt, rank_cap, trunc_tol, res_tol,
                  history="exact", restart=6, max_iter=200):
    """Low-rank theta steps.  X0_terms: the initial value as factored terms;
    its median column x~^0 is read from it.  Returns a list of per-step dicts
    (xt, S, info, terms) with X^i = x~^i 1^T + S^i."""
    m = d.shape[1]
    jmed = dr.upper_median_offset(m)
    Kt = theta_operators(K, M, theta, dt)
    dbar = ch.mean_parameters(d)
    P = ch.DirectPreconditioner(ch.mean_preconditioner(Kt, dbar))
    c, dc = ch.chebyshev_interval(d, dbar)
    Amed = lr.column_operator(Kt, d, jmed)
    lu_med = spla.splu(sp.csc_matrix(Amed))
    X_terms = list(X0_terms)
    xt_prev = sum(A @ C @ B[jmed] for (A, C, B) in X_terms)
    out = []
    for i in range(1, len(b)):
        F = step_rhs(K, M, d, b[i], b[i - 1], X_terms, xt_prev, theta, dt, history)
        FA = np.hstack([t[0] for t in F])
        FC = _block_diag([t[1] for t in F])
        FB = np.hstack([t[2] for t in F])
        # median column's theta step (its own equation, solved directly)
        xt = lu_med.solve(FA @ FC @ FB[jmed])
        # B = F - L_theta(x~ 1^T), the update's right-hand side
        Bt = lr.lr_sum((FA, FC, FB), lr.lr_scale(lr.lr_L(Kt, d, xt[:, None], np.ones(1),
                                                         np.ones((m, 1))), -1.0))
        ref = np.linalg.norm(FA @ FC @ FB.T)
        S, info = ch.chebyshev_t(Kt, d, Bt, P, c, dc, rank_cap, trunc_tol, res_tol, ref,
                                 restart=restart, max_iter=max_iter)
        U, s, V = S
        X_terms = [(xt[:, None], np.eye(1), np.ones((m, 1))), (U, np.diag(s), V)]
        out.append(dict(xt=xt, S=S, info=info, terms=X_terms, F=F, ref=ref))
        xt_prev = xt
    return out


def _block_diag(blocks):
    k = sum(b.shape[0] for b in blocks)
    C = np.zeros((k, k))
    o = 0
    for b in blocks:
        r = b.shape[0]
        C[o:o + r, o:o + r] = b
        o += r
    return C
