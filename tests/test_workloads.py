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
