"""Parameter clustering and the Newton-on-subset driver (paper Algorithm 1).

* Little-endian order (Sec. 3.3, Definition 'Little Endian Order'): the pair
  (i1, i2) of a tensor grid with m1 values of the first parameter has the
  1-based position i1 + (i2 - 1) m1.
* Subset sizes (Sec. 3.3, eq. clustering1): floor(m / K) for the first K - 1
  subsets, the remainder for the last.
* Upper median index (Sec. 3.3, Definition 'Upper Median Index'): the upper
  median of a subset in little-endian order; for a subset of size s this is the
  1-based position floor(s / 2) + 1, which the paper's example confirms
  ((4,1), (2,3), (1,5) for subsets of sizes 6, 6, 8).
* Newton step on a subset (Sec. 3.4): with the median solution x~ as the common
  initial guess, the update S solves L(S) = F - L(x~ 1^T) =: B, where B has rank
  at most q (rank <= 3 for the paper's three-term equation, Sec. 4.2), and the
  next iterate is X = x~ 1^T + S (eq. matrix_nextiterate1).  For the linear
  stand-in operators used here the median Newton solve is a single direct solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import lowrank as lr
from . import chebyshev as ch


def little_endian_position(i1, i2, m1):
    """1-based position of the multi-index (i1, i2) (both 1-based)."""
    return i1 + (i2 - 1) * m1


def multi_index(p, m1):
    """Inverse map: 1-based column p -> (i1, i2), i1 = ((p-1) mod m1) + 1,
    i2 = ceil(p / m1)  (Sec. 3.4, the column-to-parameter map)."""
    return ((p - 1) % m1) + 1, -(-p // m1)


def subset_sizes(m, K):
    base = m // K
    return [base] * (K - 1) + [m - (K - 1) * base]


def subsets(m, K, sizes=None):
    """Consecutive 0-based column ranges of the subsets in little-endian order."""
    sizes = subset_sizes(m, K) if sizes is None else list(sizes)
    out, off = [], 0
    for s in sizes:
        out.append(np.arange(off, off + s))
        off += s
    assert off == m
    return out


def upper_median_offset(size):
    """0-based offset of the upper median inside a subset of the given size."""
    return size // 2


def median_rhs(K, d, f, xt):
    """B = F - L(x~ 1^T) with F = f 1^T, in factored form
    [f | K_0 x~ | ... | K_{q-1} x~] diag(1, -1, ..., -1) [1 | d_0 | ... | d_{q-1}]^T,
    then compressed exactly (rank <= q when d_0 = 1)."""
    m = d.shape[1]
    A = np.column_stack([f] + [Ki @ xt for Ki in K])
    C = np.diag([1.0] + [-1.0] * len(K))
    Bm = np.column_stack([np.ones(m)] + [d[i] for i in range(len(K))])
    return A, C, Bm


def newton_subset(K, d, f, rank_cap, trunc_tol, res_tol, restart=6, max_iter=200,
                  cheb=None, dbar=None, form="direction"):
    """One Newton step on a subset (Algorithm 1, loop body).

    Returns dict(xt, S=(U, s, V), info, c, d) with X = xt 1^T + U diag(s) V^T.
    The stopping tolerance is relative to ||F||_F = ||f|| sqrt(m).  form:
    "direction" (chebyshev_t) or "three_term" (chebyshev_t3)."""
    m = d.shape[1]
    jmed = upper_median_offset(m)
    Amed = lr.column_operator(K, d, jmed)
    xt = spla.splu(sp.csc_matrix(Amed)).solve(f)
    B = median_rhs(K, d, f, xt)
    dbar = ch.mean_parameters(d) if dbar is None else dbar
    P = ch.mean_preconditioner(K, dbar)
    c, dc = ch.chebyshev_interval(d, dbar) if cheb is None else cheb
    ref = np.linalg.norm(f) * np.sqrt(m)
    solve = {"direction": ch.chebyshev_t, "three_term": ch.chebyshev_t3}[form]
    S, info = solve(K, d, B, ch.DirectPreconditioner(P), c, dc, rank_cap,
                    trunc_tol, res_tol, ref, restart=restart, max_iter=max_iter)
    return dict(xt=xt, S=S, info=info, c=c, d=dc, jmed=jmed)


def solution_terms(res):
    """The Newton iterate X = x~ 1^T + S as a list of factored terms."""
    xt = res["xt"]
    U, s, V = res["S"]
    m = V.shape[0]
    return [(xt[:, None], np.eye(1), np.ones((m, 1))), (U, np.diag(s), V)]


def algorithm1(K, d, f, n_subsets, rank_cap, trunc_tol, res_tol, sizes=None, **kw):
    """Algorithm 1: split the columns into subsets, one Newton step each, and
    return the list of per-subset results (X^k = x~^k 1^T + S_k)."""
    out = []
    for J in subsets(d.shape[1], n_subsets, sizes):
        out.append(dict(cols=J, **newton_subset(K, d[:, J], f, rank_cap, trunc_tol,
                                                 res_tol, **kw)))
    return out
