"""Stencil operators that stand in for the FSI finite-element matrices.

The paper's operators (Sec. 3: A_0, A_1, A_2 and the Jacobians J_mu, J_lambda,
J_rho) come from a Q2 FE discretisation of a 3D FSI benchmark that is not
available here.  These stand-ins keep the algebraic structure that the method
relies on (eq. newton_matrix1): one operator K_0 defined on the whole domain
(nonsymmetric, convection-diffusion, playing A_0 + the fluid terms) and
operators K_1, K_2 supported on a 'solid' sub-box only (symmetric positive
semi-definite, playing the shear-modulus and Lame-parameter terms).

Grid: N points per axis at x_i = i*h, i = 1..N, h = 1/(N+1); homogeneous
Dirichlet (neighbours outside the grid are dropped); lexicographic order with
x fastest.  Scaling is FE-like: every operator is h^d times its
finite-difference form, which is what Q1 assembly produces.

Solid membership uses exact integer arithmetic: a coordinate (i+1)h lies in the
closed interval [0.3, 0.7] iff 3(N+1) <= 10(i+1) <= 7(N+1).

Every matrix is returned as a SciPy CSR matrix with sorted column indices,
int64 row pointers and int32 column indices.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Operators:
    """The q operators of  sum_i K_i X D_i  together with grid metadata."""
    K: list            # list of scipy.sparse.csr_matrix, all n x n
    n: int
    dim: int
    N: int             # points per axis
    solid: np.ndarray  # bool mask of solid nodes, length n

    @property
    def q(self) -> int:
        return len(self.K)


def _csr(rows, cols, vals, n) -> sp.csr_matrix:
    A = sp.coo_matrix((np.asarray(vals, dtype=np.float64),
                       (np.asarray(rows, dtype=np.int64), np.asarray(cols, dtype=np.int64))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    return A


def _solid_axis(N: int) -> np.ndarray:
    i1 = np.arange(1, N + 1)
    return (10 * i1 >= 3 * (N + 1)) & (10 * i1 <= 7 * (N + 1))


def solid_mask(N: int, dim: int) -> np.ndarray:
    ax = _solid_axis(N)
    if dim == 2:
        return (ax[None, :] & ax[:, None]).reshape(-1)          # [iy, ix]
    return (ax[None, None, :] & ax[None, :, None] & ax[:, None, None]).reshape(-1)


def _grid_index(N: int, dim: int):
    idx = np.arange(N ** dim).reshape((N,) * dim)   # axis order (z,) y, x ; x fastest
    return idx


def _apply_stencil(N: int, dim: int, stencil: dict, keep_zeros: bool = False,
                   mask: np.ndarray | None = None) -> sp.csr_matrix:
    """Assemble a constant-coefficient stencil {offset(x,y[,z]): value}.

    Offsets are (trial - test) per axis, given in (x, y[, z]) order.  With
    ``mask`` only rows and columns of masked nodes are kept (a principal
    submatrix).  ``keep_zeros`` stores zero-valued stencil entries explicitly,
    as FE assembly on the stencil's full pattern would.
    """
    n = N ** dim
    idx = _grid_index(N, dim)
    coords = np.indices((N,) * dim).reshape(dim, -1)[::-1]      # rows: x, y[, z]
    rows, cols, vals = [], [], []
    for off, v in stencil.items():
        if v == 0.0 and not keep_zeros:
            continue
        tgt = coords + np.asarray(off).reshape(dim, 1)
        ok = np.all((tgt >= 0) & (tgt < N), axis=0)
        src = np.nonzero(ok)[0]
        t = tgt[:, ok]
        col = idx[tuple(t[::-1])]                                 # back to (z,) y, x order
        rows.append(src)
        cols.append(col)
        vals.append(np.full(src.shape, v))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    if mask is not None:
        keep = mask[rows] & mask[cols]
        rows, cols, vals = rows[keep], cols[keep], vals[keep]
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    if keep_zeros:
        A = sp.csr_matrix((A.data, A.indices, A.indptr), shape=(n, n))
    else:
        A.sum_duplicates()
        A.eliminate_zeros()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    return A


# --- 1D Q1 element integrals on a uniform grid, offset o = trial - test -----------
def _mass1(o, h):
    return {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}[o] * h


def _stiff1(o, h):
    return {0: 2.0, 1: -1.0, -1: -1.0}[o] / h


def _trial_deriv1(o, h):   # integral of phi_trial' * phi_test
    return {0: 0.0, 1: 0.5, -1: -0.5}[o]


def _test_deriv1(o, h):    # integral of phi_trial * phi_test'
    return {0: 0.0, 1: -0.5, -1: 0.5}[o]


def q1_form_stencil(dim: int, h: float, pairs) -> dict:
    """Stencil of the Q1 bilinear form  sum_{(a,b) in pairs} int d_a u d_b v.

    Built as tensor products of the 1D element integrals (mass, stiffness and
    the two mixed derivative-mass integrals), i.e. exactly what assembling the
    trilinear/bilinear element matrices on a uniform grid gives.
    """
    st = {}
    for off in itertools.product((-1, 0, 1), repeat=dim):
        val = 0.0
        for a, b in pairs:
            t = 1.0
            for ax in range(dim):
                o = off[ax]
                if ax == a and ax == b:
                    t *= _stiff1(o, h)
                elif ax == a:
                    t *= _trial_deriv1(o, h)
                elif ax == b:
                    t *= _test_deriv1(o, h)
                else:
                    t *= _mass1(o, h)
            val += t
        st[off] = val
    return st


# --- 2D operators -----------------------------------------------------------------
def conv_diff_2d(N: int, nu: float = 1e-2, wind=(1.0, 0.5)) -> sp.csr_matrix:
    """K_0 = nu*L5 + h*(w_x D_x + w_y D_y), upwind one-sided differences."""
    h = 1.0 / (N + 1)
    st = {(0, 0): 4.0 * nu, (1, 0): -nu, (-1, 0): -nu, (0, 1): -nu, (0, -1): -nu}
    for ax, w in enumerate(wind):
        up = -1 if w >= 0 else 1                    # upwind neighbour
        o = [0, 0]
        o[ax] = up
        st[(0, 0)] += h * abs(w)
        st[tuple(o)] = st.get(tuple(o), 0.0) - h * abs(w)
    return _apply_stencil(N, 2, st)


def laplace5_solid_2d(N: int) -> sp.csr_matrix:
    """K_1 = Pi_S L5 Pi_S: 5-point Laplacian restricted to the solid box."""
    st = {(0, 0): 4.0, (1, 0): -1.0, (-1, 0): -1.0, (0, 1): -1.0, (0, -1): -1.0}
    return _apply_stencil(N, 2, st, mask=solid_mask(N, 2))


def graddiv9_solid_2d(N: int) -> sp.csr_matrix:
    """K_2 = Pi_S G9 Pi_S, G9 = Q1 form of (d_x+d_y)u (d_x+d_y)v (9 points)."""
    h = 1.0 / (N + 1)
    st = q1_form_stencil(2, h, [(a, b) for a in range(2) for b in range(2)])
    return _apply_stencil(N, 2, st, mask=solid_mask(N, 2))


def three_term_2d(N: int, nu: float = 1e-2, wind=(1.0, 0.5)) -> Operators:
    K = [conv_diff_2d(N, nu, wind), laplace5_solid_2d(N), graddiv9_solid_2d(N)]
    return Operators(K=K, n=N * N, dim=2, N=N, solid=solid_mask(N, 2))


def seven_term_2d(N: int, nu: float = 1e-2, wind=(1.0, 0.5)) -> Operators:
    """Stand-in for the four-parameter equation's seven terms (eq.
    matrix_fourpars1): K_0 the convection-diffusion operator (D_0 = I); then
    four solid terms and two fluid terms, each with a positive parameter row:
    K_1 = solid 5-point Laplacian (mu), K_2 = fluid 5-point Laplacian (nu rho),
    K_3 = solid Q1 (d_x + d_y)^2 (lambda), K_4 = solid Q1 (d_x - d_y)^2 (the mu
    Jacobian term), K_5 = h^2 times the solid identity (the lambda Jacobian
    term), K_6 = upwind convection restricted to the fluid (the rho Jacobian
    term).  Every K_i, i >= 1, is a principal submatrix of a positive
    semi-definite (K_6: semi-definite symmetric part) operator."""
    h = 1.0 / (N + 1)
    solid = solid_mask(N, 2)
    fluid = ~solid
    lap = {(0, 0): 4.0, (1, 0): -1.0, (-1, 0): -1.0, (0, 1): -1.0, (0, -1): -1.0}
    gd = q1_form_stencil(2, h, [(0, 0), (0, 1), (1, 0), (1, 1)])
    gm = q1_form_stencil(2, h, [(0, 0), (1, 1)])
    for off, v in q1_form_stencil(2, h, [(0, 1), (1, 0)]).items():
        gm[off] = gm.get(off, 0.0) - v
    conv = {(0, 0): h * (abs(wind[0]) + abs(wind[1])), (-1, 0): -h * abs(wind[0]),
            (0, -1): -h * abs(wind[1])}
    K = [conv_diff_2d(N, nu, wind),
         _apply_stencil(N, 2, lap, mask=solid),
         _apply_stencil(N, 2, lap, mask=fluid),
         _apply_stencil(N, 2, gd, mask=solid),
         _apply_stencil(N, 2, gm, mask=solid),
         _apply_stencil(N, 2, {(0, 0): h * h}, mask=solid),
         _apply_stencil(N, 2, conv, mask=fluid)]
    return Operators(K=K, n=N * N, dim=2, N=N, solid=solid)


# --- 3D operators -----------------------------------------------------------------
def conv_diff_3d(N: int, nu: float = 1e-2, wind=(1.0, 0.5, 0.25)) -> sp.csr_matrix:
    """K_0 = h*nu*L7 + h^2*(w . D), upwind one-sided differences (7 points)."""
    h = 1.0 / (N + 1)
    st = {(0, 0, 0): 6.0 * h * nu}
    for ax in range(3):
        for s in (-1, 1):
            o = [0, 0, 0]
            o[ax] = s
            st[tuple(o)] = -h * nu
    for ax, w in enumerate(wind):
        o = [0, 0, 0]
        o[ax] = -1 if w >= 0 else 1
        st[(0, 0, 0)] += h * h * abs(w)
        st[tuple(o)] -= h * h * abs(w)
    return _apply_stencil(N, 3, st)


def three_term_3d(N: int, nu: float = 1e-2, wind=(1.0, 0.5, 0.25)) -> Operators:
    """K_1: Q1 Laplacian, K_2: Q1 (d_x+d_y+d_z)^2 form, both on the solid cube,
    stored on the full 27-point pattern (explicit zeros kept)."""
    h = 1.0 / (N + 1)
    mask = solid_mask(N, 3)
    lap = q1_form_stencil(3, h, [(a, a) for a in range(3)])
    gd = q1_form_stencil(3, h, [(a, b) for a in range(3) for b in range(3)])
    K = [conv_diff_3d(N, nu, wind),
         _apply_stencil(N, 3, lap, keep_zeros=True, mask=mask),
         _apply_stencil(N, 3, gd, keep_zeros=True, mask=mask)]
    return Operators(K=K, n=N ** 3, dim=3, N=N, solid=mask)
