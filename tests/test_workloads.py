"""The seeded workloads follow the paper's conventions (CPU only)."""
import numpy as np

from oracle import driver as odrv
from workloads import config


def test_four_parameter_columns_are_little_endian():
    """Sec. 4.4: column p of a four-parameter grid holds the multi-index with
    p = i1 + (i2 - 1) m1 + (i3 - 1) m1 m2 + (i4 - 1) m1 m2 m3 (1-based), and
    the seven rows are 1, mu, nu rho, lambda, mu, lambda, rho."""
    cfg = config("q7")
    d = cfg["d"]
    m1, m2, m3, m4 = cfg["m"]
    mu = np.unique(d[1])
    nu_rho = d[2]
    lam = np.unique(d[3])
    rho = np.unique(d[6])
    assert d.shape == (7, m1 * m2 * m3 * m4)
    assert np.array_equal(d[0], np.ones(d.shape[1]))
    assert np.array_equal(d[4], d[1]) and np.array_equal(d[5], d[3])
    for p in range(1, d.shape[1] + 1):
        r = p - 1
        i1, r = r % m1 + 1, r // m1
        i2, r = r % m2 + 1, r // m2
        i3, i4 = r % m3 + 1, r // m3 + 1
        assert p == i1 + (i2 - 1) * m1 + (i3 - 1) * m1 * m2 + (i4 - 1) * m1 * m2 * m3
        assert d[1, p - 1] == mu[i1 - 1] and d[3, p - 1] == lam[i3 - 1]
        assert d[6, p - 1] == rho[i4 - 1]
        nu = nu_rho[p - 1] / rho[i4 - 1]
        assert np.isclose(nu, np.linspace(0.9, 1.1, 3)[i2 - 1])
    # the two-parameter rule of Sec. 3.3 is the m3 = m4 = 1 case
    assert odrv.little_endian_position(3, 2, m1) == 3 + (2 - 1) * m1


def test_seven_term_operators_semidefinite():
    """The spectrum interval used by the preconditioner needs K_0 + K_0^T and
    every other term's symmetric part positive semi-definite (small grid)."""
    from workloads import seven_term_2d
    ops = seven_term_2d(9)
    for i, K in enumerate(ops.K):
        S = (K + K.T).toarray() / 2
        assert np.linalg.eigvalsh(S).min() >= -1e-12 * max(1.0, abs(S).max()), i


def test_three_dimensional_operators():
    """The 3D stand-ins (c5, c5r): K_0 is the 7-point upwind
    convection-diffusion operator (non-positive off-diagonal entries,
    non-negative row sums); K_1, K_2 live on the solid cube only, on the full
    27-point pattern, and are symmetric positive semi-definite; the row of
    K_1 (the Q1 Laplacian) at a node whose 26 neighbours are all solid sums to
    zero (small grid)."""
    from workloads.stencils import three_term_3d
    ops = three_term_3d(7)
    K0, K1, K2 = ops.K
    n = ops.n
    assert n == 343 and ops.dim == 3
    A = K0.toarray()
    off = A - np.diag(np.diag(A))
    assert off.max() <= 0 and (A.sum(axis=1) >= -1e-15).all()
    assert max(np.diff(K0.indptr)) == 7
    solid = ops.solid
    for K in (K1, K2):
        D = K.toarray()
        assert np.allclose(D, D.T, atol=1e-15)
        assert np.linalg.eigvalsh(D).min() >= -1e-12 * abs(D).max()
        rows = np.nonzero(np.diff(K.indptr))[0]
        assert solid[rows].all() and max(np.diff(K.indptr)) == 27
    # Q1 Laplacian rows of nodes whose 26 neighbours are all solid sum to 0
    L1 = K1.toarray()
    N = 7
    idx = np.arange(n).reshape(N, N, N)
    inner = [i for i in range(n) if solid[i] and all(
        solid[idx[tuple(np.clip(np.array(np.unravel_index(i, (N,) * 3)) + o, 0, N - 1))]]
        for o in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).reshape(3, -1).T)]
    assert inner
    for i in inner:
        assert abs(L1[i].sum()) <= 1e-14 * abs(L1[i]).max()


def test_reduced_3d_workload_fits_truncation():
    """c5r keeps c5's operators and parameters at a grid and rank cap whose
    residual concatenation fits 128 columns: 1 + 3 * 40 <= 128."""
    c = config("c5r", small=True)
    assert c["ops"].dim == 3 and c["rank_cap"] * len(c["ops"].K) + 1 <= 128
    assert c["d"].shape == (3, 40)
