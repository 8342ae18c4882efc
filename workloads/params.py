"""Seeded parameter sets, right-hand sides and the five workload recipes.

The matrix equation of a Newton step on a subset (paper Sec. 3.4) couples each
operator K_i with a diagonal parameter matrix D_i.  Here D_0 = I, D_1 =
diag(mu_s) and D_2 = diag(lambda_s); the table ``d`` has shape (q, m) and row i
holds diag(D_i).

Parameter ranges follow the workload definitions: mu_s in [0.5, 2]*1e4 and
lambda_s in [1, 4]*1e4.  On a tensor grid the columns are ordered little-endian
with mu fastest (paper Sec. 3.3, Definition 'Little Endian Order').
"""
from __future__ import annotations

import numpy as np

from .stencils import seven_term_2d, three_term_2d, three_term_3d

MU_RANGE = (0.5e4, 2.0e4)
LAM_RANGE = (1.0e4, 4.0e4)

# Sixteen uneven subset sizes in [20, 300] summing to 2000 (batched workload).
C3_SUBSET_SIZES = [20, 300, 45, 210, 130, 60, 275, 95, 20, 180, 150, 35, 240, 110, 70, 60]


def grid_params_little_endian(mu_vals, lam_vals):
    """All (mu, lambda) pairs of a tensor grid, mu index fastest."""
    mu_vals = np.asarray(mu_vals, dtype=np.float64)
    lam_vals = np.asarray(lam_vals, dtype=np.float64)
    mu = np.tile(mu_vals, lam_vals.size)
    lam = np.repeat(lam_vals, mu_vals.size)
    return mu, lam


def random_params(m: int, seed: int):
    """m independent uniform draws: all mu first, then all lambda."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(MU_RANGE[0], MU_RANGE[1], m)
    lam = rng.uniform(LAM_RANGE[0], LAM_RANGE[1], m)
    return mu, lam


def param_table(mu, lam) -> np.ndarray:
    """d[0] = 1 (D_0 = I), d[1] = mu, d[2] = lambda; shape (3, m), float64."""
    mu = np.asarray(mu, dtype=np.float64)
    return np.stack([np.ones_like(mu), mu, np.asarray(lam, dtype=np.float64)])


def rhs_vector(n: int, seed: int = 0) -> np.ndarray:
    """f ~ N(0, 1) from the seed; the right-hand side is F = f 1^T."""
    return np.random.default_rng(seed).standard_normal(n)


def subset_perturbations(K: int, seed: int = 4, spread: float = 0.2):
    """Per-subset factors (1 + spread*U[-1,1]) for nu (column 0) and the wind
    vector (column 1): each subset gets its own linearisation point."""
    rng = np.random.default_rng(seed)
    return 1.0 + spread * rng.uniform(-1.0, 1.0, size=(K, 2))


def config(name: str, small: bool = False) -> dict:
    """Build one workload.  ``small`` shrinks the grid for quick tests while
    keeping the structure (solid box, parameter ranges, seeds)."""
    if name == "c1":
        N = 65
        ops = three_term_2d(N)
        mu, lam = grid_params_little_endian(np.linspace(0.5, 2.0, 10) * 1e4,
                                            np.linspace(1.0, 4.0, 10) * 1e4)
        return dict(name=name, ops=ops, d=param_table(mu, lam), f=rhs_vector(ops.n, 0),
                    rank_cap=20, trunc_tol=1e-8, res_tol=1e-8, m1=10, m2=10)
    if name == "c2":
        N = 129 if small else 513
        m = 200 if small else 1000
        ops = three_term_2d(N)
        mu, lam = random_params(m, 1)
        return dict(name=name, ops=ops, d=param_table(mu, lam), f=rhs_vector(ops.n, 0),
                    rank_cap=40, trunc_tol=1e-8, res_tol=1e-6)
    if name == "c3":
        N = 65 if small else 257
        sizes = list(C3_SUBSET_SIZES)
        if small:
            sizes = [max(4, s // 10) for s in sizes]
        mtot = int(np.sum(sizes))
        mu, lam = random_params(mtot, 3)
        fac = subset_perturbations(len(sizes), 4)
        base = three_term_2d(N)
        subsets = []
        off = 0
        for j, mj in enumerate(sizes):
            opsj = three_term_2d(N, nu=1e-2 * fac[j, 0], wind=(1.0 * fac[j, 1], 0.5 * fac[j, 1]))
            subsets.append(dict(ops=opsj, d=param_table(mu[off:off + mj], lam[off:off + mj])))
            off += mj
        return dict(name=name, base_ops=base, subsets=subsets, f=rhs_vector(base.n, 0),
                    rank_cap=30, trunc_tol=1e-8, res_tol=1e-6, sizes=sizes)
    if name == "c4":
        N = 65 if small else 257
        ops = three_term_2d(N)
        mtr, mte = (40, 60) if small else (200, 500)
        mu_tr, lam_tr = random_params(mtr, 5)
        mu_te, lam_te = random_params(mte, 6)
        return dict(name=name, ops=ops, d_train=param_table(mu_tr, lam_tr),
                    d_test=param_table(mu_te, lam_te), f=rhs_vector(ops.n, 0),
                    rank_cap=30, basis_rank=30, trunc_tol=1e-8, res_tol=1e-6)
    if name == "c5":
        N = 22 if small else 102
        ops = three_term_3d(N)
        mu, lam = random_params(100 if small else 500, 7)
        return dict(name=name, ops=ops, d=param_table(mu, lam), f=rhs_vector(ops.n, 0),
                    rank_cap=60, trunc_tol=1e-8, res_tol=1e-6)
    if name == "c5r":
        # the 3D workload of "c5" on a 48^3 grid (n = 110,592) with rank cap
        # 40, the widest cap whose residual [B | K_0 S | K_1 S | K_2 S] fits
        # the truncation's 128 columns at q = 3; same operators, parameter
        # ranges, seeds and tolerances
        N = 16 if small else 48
        ops = three_term_3d(N)
        mu, lam = random_params(40 if small else 500, 7)
        return dict(name=name, ops=ops, d=param_table(mu, lam), f=rhs_vector(ops.n, 0),
                    rank_cap=40, trunc_tol=1e-8, res_tol=1e-6)
    if name == "q7":
        # one subset of a four-parameter discretisation (mu, nu, lambda, rho;
        # Sec. 4.4) on a little-endian tensor grid, mu fastest, then nu,
        # lambda, rho: 4 x 3 x 4 x 3 = 144 columns around mu = 1.25e4,
        # lambda = 2.5e4, nu = rho = 1.  The truncation tolerance is 1e-10:
        # at 1e-8 the truncation of S itself stalls the residual near 5e-5.
        N = 33 if small else 65
        ops = seven_term_2d(N)
        g = [np.linspace(1.0, 1.5, 4) * 1e4, np.linspace(0.9, 1.1, 3),
             np.linspace(2.0, 3.0, 4) * 1e4, np.linspace(0.9, 1.1, 3)]
        cols = [(a, b, c, e) for e in g[3] for c in g[2] for b in g[1] for a in g[0]]
        d = four_param_table(*np.array(cols).T)
        return dict(name=name, ops=ops, d=d, f=rhs_vector(ops.n, 0), rank_cap=16,
                    trunc_tol=1e-10, res_tol=1e-6, m=(4, 3, 4, 3))
    raise ValueError(f"unknown workload {name!r}")


def four_param_table(mu, nu, lam, rho) -> np.ndarray:
    """Rows of the seven-term equation: 1, mu, nu rho, lambda, mu, lambda, rho
    (D_0 = I, then the parameter of each of K_1..K_6 of seven_term_2d)."""
    mu, nu, lam, rho = (np.asarray(a, dtype=np.float64) for a in (mu, nu, lam, rho))
    return np.stack([np.ones_like(mu), mu, nu * rho, lam, mu, lam, rho])


def mlp_init(seed: int = 11, sizes=(2, 64, 64, 30)):
    """Seeded initial weights [W1, b1, W2, b2, W3, b3] (W is out x in),
    Glorot-normal weights and zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        std = np.sqrt(2.0 / (fan_in + fan_out))
        params.append(rng.standard_normal((fan_out, fan_in)) * std)
        params.append(np.zeros(fan_out))
    return params
