"""Mean-based preconditioner, Chebyshev interval and the ChebyshevT iteration.

ChebyshevT (paper Sec. 2.2, Sec. 4.1 and Sec. 5.1, citing the companion paper
for the algorithm, which is not printed here) is read as the classical
Chebyshev acceleration for a spectrum inside the real interval
[d - c, d + c] (centre d, half-width c; the paper's c = 0.1, d = 1 then means
[0.9, 1.1]), applied to the linear operator S -> L(S) = sum_i K_i S D_i with
left preconditioning by I (x) P (paper Sec. 4.2) and a truncation T after every
update of a low-rank quantity.  With sigma = d / c:

    R  <- T(B - L(S));            stop if ||R||_F <= tau * ||F||_F
    Dl <- T(P^-1 R / d);  rho <- c / d
    repeat l times:
        S   <- T(S + Dl)
        R   <- T(B - L(S));       stop if ||R||_F <= tau * ||F||_F
        rho' = 1 / (2 sigma - rho)
        Dl  <- T(rho' rho Dl + (2 rho' / c) P^-1 R);   rho <- rho'
    and restart from the current S (the paper restarts after 6 iterations).

The residual is recomputed from S at every step (not updated recursively), and
the rank-1 term x~ 1^T of the Newton driver is never truncated: this module
only ever sees the Newton update S.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import lowrank as lr


# --------------------------------------------------------------------- preconditioner
def mean_parameters(d, kind="mean"):
    """Centre parameters of a subset.  ``mean``: arithmetic mean of each row of
    d; ``midrange``: (min + max) / 2, the paper's choice in Sec. 4.2."""
    d = np.asarray(d, dtype=np.float64)
    if kind == "mean":
        return d.mean(axis=1)
    if kind == "midrange":
        return 0.5 * (d.min(axis=1) + d.max(axis=1))
    raise ValueError(kind)


def mean_preconditioner(K, dbar):
    """P = sum_i dbar_i K_i, the operator at the centre parameters (Sec. 4.2)."""
    P = dbar[0] * K[0]
    for i in range(1, len(K)):
        P = P + dbar[i] * K[i]
    return sp.csc_matrix(P)


class DirectPreconditioner:
    """Z = P^{-1} R by an exact sparse LU of P (the paper factorises P with
    MATLAB's permuted LU, Sec. 5)."""

    def __init__(self, P):
        self.lu = spla.splu(sp.csc_matrix(P))

    def solve(self, R):
        R = np.asarray(R, dtype=np.float64)
        if R.ndim == 1:
            return self.lu.solve(R)
        return np.column_stack([self.lu.solve(R[:, j]) for j in range(R.shape[1])]) \
            if R.shape[1] else R.copy()


def chebyshev_interval(d, dbar):
    """[lo, hi] enclosing the preconditioned spectra of every column.

    With K_0 + K_0^T and every other K_i symmetric positive semi-definite, the
    generalised Rayleigh quotient of A_j = sum_i d_ij K_i against
    P = sum_i dbar_i K_i is a weighted mean of the ratios d_ij / dbar_i (and of 1
    for the i = 0 term, where d_0j = dbar_0 = 1), so every column's spectrum lies
    in [min, max] of {1} U {d_ij / dbar_i}.  This stands in for the paper's
    eigenvalue estimate at the subset's corner parameters (Sec. 5.1).
    Returns (c, d) = (half-width, centre).
    """
    d = np.asarray(d, dtype=np.float64)
    ratios = d / np.asarray(dbar)[:, None]
    lo = min(1.0, ratios.min())
    hi = max(1.0, ratios.max())
    return 0.5 * (hi - lo), 0.5 * (hi + lo)


# --------------------------------------------------------------------- ChebyshevT
@dataclasses.dataclass
class ChebInfo:
    iters: int = 0
    converged: bool = False
    history: list = dataclasses.field(default_factory=list)   # ||R||_F after each check
    ranks: list = dataclasses.field(default_factory=list)     # rank of S after each update
    prec_applies: int = 0


def residual_factored(K, d, B, S):
    """B - L(S) as one factored triple (B is a triple, S = (U, s, V))."""
    U, s, V = S
    if U.shape[1] == 0:
        return B
    return lr.lr_sum(B, lr.lr_scale(lr.lr_L(K, d, U, s, V), -1.0))


def chebyshev_t(K, d, B, prec, c, dc, rank_cap, trunc_tol, res_tol, ref_norm,
                restart=6, max_iter=200, S0=None, res_rank_cap=None):
    """Solve L(S) = B approximately in low-rank form.

    B: factored right-hand side (A, C, Bm).  prec: object with .solve(R) = P^-1 R.
    c, dc: half-width and centre of the spectrum interval.  rank_cap and
    trunc_tol apply to every truncation (res_rank_cap, if given, to the
    residual's).  Stops when ||T(B - L(S))||_F <= res_tol * ref_norm.
    Returns ((U, s, V), ChebInfo).
    """
    n, m = B[0].shape[0], B[2].shape[0]
    rcap_res = rank_cap if res_rank_cap is None else res_rank_cap
    info = ChebInfo()
    if S0 is None:
        S = (np.zeros((n, 0)), np.zeros(0), np.zeros((m, 0)))
    else:
        S = S0
    sigma = dc / c if c > 0 else np.inf

    def resid(S):
        A, C, Bm = residual_factored(K, d, B, S)
        return lr.truncate(A, C, Bm, rcap_res, trunc_tol)

    def precond(R):
        info.prec_applies += 1
        U, s, V = R
        return prec.solve(U), s, V

    R = resid(S)
    info.history.append(float(np.linalg.norm(R[1])))
    while True:
        if info.history[-1] <= res_tol * ref_norm or R[1].size == 0:
            info.converged = True
            return S, info
        if info.iters >= max_iter:
            return S, info
        # (re)start: first direction from the current residual
        Z, sz, Vz = precond(R)
        Dl = lr.truncate(Z, np.diag(sz / dc), Vz, rank_cap, trunc_tol)
        rho = c / dc
        cycle = restart if restart > 0 else max_iter
        for k in range(cycle):
            S = lr.truncate(*lr.lr_sum(lr.usv(*S), lr.usv(*Dl)), rank_cap, trunc_tol)
            info.iters += 1
            info.ranks.append(S[1].size)
            R = resid(S)
            nr = float(np.linalg.norm(R[1]))
            info.history.append(nr)
            if nr <= res_tol * ref_norm or R[1].size == 0 or info.iters >= max_iter \
                    or k == cycle - 1:
                break
            rho_new = 1.0 / (2.0 * sigma - rho)
            Z, sz, Vz = precond(R)
            Dl = lr.truncate(*lr.lr_sum(lr.lr_scale(lr.usv(*Dl), rho_new * rho),
                                        (Z, np.diag((2.0 * rho_new / c) * sz), Vz)),
                             rank_cap, trunc_tol)
            rho = rho_new


def chebyshev_t3(K, d, B, prec, c, dc, rank_cap, trunc_tol, res_tol, ref_norm,
                 restart=6, max_iter=200, S0=None, res_rank_cap=None):
    """ChebyshevT in the three-term form of the Chebyshev iteration.

    The same polynomial iteration as `chebyshev_t` (same interval [dc - c,
    dc + c], same restarts, stops and residual truncation) written without
    the direction Dl: in exact arithmetic Dl = S_{k+1} - S_k, so the direction
    update of `chebyshev_t` becomes the classical three-term recurrence of the
    Chebyshev polynomials applied to the iterates,

        S_1     <- T(S_0 + P^-1 R_0 / dc),                  rho <- c / dc
        S_{k+1} <- T((1 + rho' rho) S_k - rho' rho S_{k-1} + (2 rho' / c) P^-1 R_k),
        rho' = 1 / (2 sigma - rho),  rho <- rho',

    which truncates once per update instead of twice (the direction and the
    iterate).  With truncation the two forms differ only by where the
    truncation errors enter.  Arguments and result as for `chebyshev_t`.
    """
    n, m = B[0].shape[0], B[2].shape[0]
    rcap_res = rank_cap if res_rank_cap is None else res_rank_cap
    info = ChebInfo()
    S = (np.zeros((n, 0)), np.zeros(0), np.zeros((m, 0))) if S0 is None else S0
    sigma = dc / c if c > 0 else np.inf

    def resid(S):
        A, C, Bm = residual_factored(K, d, B, S)
        return lr.truncate(A, C, Bm, rcap_res, trunc_tol)

    def precond(R):
        info.prec_applies += 1
        U, s, V = R
        return prec.solve(U), s, V

    R = resid(S)
    info.history.append(float(np.linalg.norm(R[1])))
    while True:
        if info.history[-1] <= res_tol * ref_norm or R[1].size == 0:
            info.converged = True
            return S, info
        if info.iters >= max_iter:
            return S, info
        cycle = restart if restart > 0 else max_iter
        rho = c / dc
        S_prev = None
        for k in range(cycle):
            Z, sz, Vz = precond(R)
            if S_prev is None:
                new = lr.lr_sum(lr.usv(*S), (Z, np.diag(sz / dc), Vz))
            else:
                rho_new = 1.0 / (2.0 * sigma - rho)
                a = rho_new * rho
                new = lr.lr_sum(lr.lr_scale(lr.usv(*S), 1.0 + a),
                                lr.lr_scale(lr.usv(*S_prev), -a),
                                (Z, np.diag((2.0 * rho_new / c) * sz), Vz))
                rho = rho_new
            S_prev = S
            S = lr.truncate(*new, rank_cap, trunc_tol)
            info.iters += 1
            info.ranks.append(S[1].size)
            R = resid(S)
            nr = float(np.linalg.norm(R[1]))
            info.history.append(nr)
            if nr <= res_tol * ref_norm or R[1].size == 0 or info.iters >= max_iter:
                break
