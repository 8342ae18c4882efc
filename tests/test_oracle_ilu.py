"""Pins of the ILU(0) oracle (oracle/ilu.py): with no fill to drop (a
tridiagonal matrix) it is the exact LU, L U = A; on a 2D stencil it matches A
on A's pattern and stays inside it; and on a small matrix it equals dense
Gaussian elimination in the other loop order (KIJ: eliminate column k from
every later row, then the next k) with updates outside the pattern dropped,
which is the same incomplete factorisation reached by a different route."""
import numpy as np
import scipy.sparse as sp

from oracle import ilu as oilu
from workloads import three_term_2d


def test_no_fill_is_exact_lu():
    n = 40
    rng = np.random.default_rng(0)
    A = sp.diags([rng.uniform(-1, 0, n - 1), rng.uniform(3, 4, n), rng.uniform(-1, 0, n - 1)],
                 [-1, 0, 1], format="csr")
    L, U = oilu.ilu0(A)
    assert np.abs((L @ U - A).toarray()).max() <= 1e-14
    assert np.allclose(np.diag(L.toarray()), 1.0)
    assert np.abs(np.triu(L.toarray(), 1)).max() == 0 and np.abs(np.tril(U.toarray(), -1)).max() == 0


def test_pattern_property_on_stencil():
    ops = three_term_2d(9)
    A = sp.csr_matrix(ops.K[0] + 1.2e4 * ops.K[1] + 2.5e4 * ops.K[2])
    L, U = oilu.ilu0(A)
    LU = (L @ U).toarray()
    Ad = A.toarray()
    pat = Ad != 0
    assert np.abs(LU[pat] - Ad[pat]).max() <= 1e-10 * np.abs(Ad).max()
    outside = ~(pat | np.eye(A.shape[0], dtype=bool))
    assert np.abs(L.toarray()[outside]).max() == 0 and np.abs(U.toarray()[outside]).max() == 0
    # fill would have changed something: the factorisation is not exact
    assert np.abs(LU - Ad).max() > 1e-6 * np.abs(Ad).max()


def test_matches_masked_kij_elimination():
    rng = np.random.default_rng(3)
    n = 7
    M = rng.uniform(-1, 1, (n, n)) * (rng.uniform(size=(n, n)) < 0.45)
    M += np.diag(rng.uniform(4, 5, n))
    pat = M != 0
    W = M.copy()
    for k in range(n):
        for i in range(k + 1, n):
            if not pat[i, k]:
                continue
            W[i, k] /= W[k, k]
            for j in range(k + 1, n):
                if pat[i, j] and pat[k, j]:
                    W[i, j] -= W[i, k] * W[k, j]
    L, U = oilu.ilu0(sp.csr_matrix(M))
    Lw = np.tril(W, -1) + np.eye(n)
    Uw = np.triu(W)
    assert np.allclose(L.toarray(), Lw, atol=1e-14) and np.allclose(U.toarray(), Uw, atol=1e-14)


def test_union_pattern_keeps_cancelled_entries():
    """On the operators' union pattern: equal to ILU(0) of the sum when no
    entry cancels; when one cancels exactly it stays a (zero) pattern entry,
    which lets fill through that ILU(0) of the pruned sum would drop."""
    ops = three_term_2d(7)
    K = ops.K
    w = [1.0, 1.3e4, 2.1e4]
    L1, U1 = oilu.ilu0_of_sum(K, w)
    A = sp.csr_matrix(sum(wi * Ki for wi, Ki in zip(w, K)))
    L2, U2 = oilu.ilu0(A)
    assert np.abs((L1 - L2).toarray()).max() <= 1e-12 and np.abs((U1 - U2).toarray()).max() <= 1e-8
    # [[4, 1, 0], [1, 4, 1], [0, 1, 4]] - a term that cancels the (0, 1) pair
    T = sp.csr_matrix(np.array([[4.0, 1, 0], [1, 4, 1], [0, 1, 4]]))
    C = sp.csr_matrix(np.array([[0.0, -1, 0], [-1, 0, 0], [0, 0, 0]]))
    Lz, Uz = oilu.ilu0_of_sum([T, C], [1.0, 1.0])
    assert Lz.toarray()[1, 0] == 0.0 and Uz.toarray()[0, 1] == 0.0
    assert np.allclose((Lz @ Uz).toarray(), (T + C).toarray())
