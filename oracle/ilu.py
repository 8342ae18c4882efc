"""ILU(0): the incomplete LU factorisation without fill, an alternative
centre preconditioner for operators whose exact factors do not fit (Sec. 4.2
names the preconditioner P = A(x~, mu-bar, nu-bar); its factorisation is the
implementer's choice, Sec. 5 uses an exact permuted LU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition: L unit lower triangular and U upper triangular, both confined to
the sparsity pattern of A, with (L U)_ij = A_ij on every (i, j) of that
pattern.  Computed by Gaussian elimination row by row (IKJ order) in which
any update outside the pattern is dropped.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def ilu0(A):
    """(L, U) of A on A's stored pattern (CSR, full diagonal)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    rows = []
    for i in range(n):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        rows.append(dict(zip(cols.tolist(), vals.tolist())))
    return _ilu0_rows(rows)


def ilu0_of_sum(K, w):
    """(L, U) of P = sum_i w_i K_i on the union of the K_i's stored patterns
    (an entry where the terms cancel stays in the pattern with value 0)."""
    n = K[0].shape[0]
    rows = [dict() for _ in range(n)]
    for Ki, wi in zip(K, w):
        Ki = sp.csr_matrix(Ki)
        for i in range(n):
            ri = rows[i]
            for e in range(Ki.indptr[i], Ki.indptr[i + 1]):
                c = int(Ki.indices[e])
                ri[c] = ri.get(c, 0.0) + wi * float(Ki.data[e])
    return _ilu0_rows(rows)


def _ilu0_rows(rows):
    n = len(rows)
    for i in range(n):
        ri = rows[i]
        for k in sorted(c for c in ri if c < i):
            ri[k] = ri[k] / rows[k][k]
            lik = ri[k]
            for j, ukj in rows[k].items():
                if j > k and j in ri:
                    ri[j] -= lik * ukj
        if not np.isfinite(ri[i]) or ri[i] == 0.0:
            raise ZeroDivisionError(f"zero pivot at row {i}")
    Lr, Lc, Lv, Ur, Uc, Uv = [], [], [], [], [], []
    for i, ri in enumerate(rows):
        for j, v in ri.items():
            if j < i:
                Lr.append(i); Lc.append(j); Lv.append(v)
            else:
                Ur.append(i); Uc.append(j); Uv.append(v)
    L = sp.csr_matrix((Lv, (Lr, Lc)), shape=(n, n)) + sp.identity(n, format="csr")
    U = sp.csr_matrix((Uv, (Ur, Uc)), shape=(n, n))
    return sp.csr_matrix(L), sp.csr_matrix(U)


class ILU0Preconditioner:
    """Z = (L U)^-1 R by the two triangular solves; built from P itself, or
    from (K, w) for P = sum_i w_i K_i on the operators' union pattern."""

    def __init__(self, A=None, K=None, w=None):
        self.L, self.U = ilu0(A) if K is None else ilu0_of_sum(K, w)

    def solve(self, R):
        R = np.asarray(R, dtype=np.float64)
        y = spla.spsolve_triangular(self.L, R, lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(self.U, y, lower=False)
