"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package builds the problem data of the parameter-dependent matrix
equation  sum_i K_i X D_i = F  (the Newton step on a parameter subset, paper
Sec. 3.4, eq. newton_matrix1): sparse operators K_i in CSR form, the diagonal
parameter matrices D_i (as a q x m table of diagonals) and the right-hand side.
It holds none of the solver's arithmetic: no truncation, no preconditioner, no
Chebyshev recurrence, no residual.  The FSI operators of the paper (Sec. 5,
Q2 hexahedral FE on a 3D channel) are not available, so stencil operators of
the same algebraic structure stand in for them (see ``stencils``).
"""
from .stencils import (Operators, conv_diff_2d, laplace5_solid_2d, graddiv9_solid_2d,
                       three_term_2d, three_term_3d, seven_term_2d)
from .params import (grid_params_little_endian, random_params, param_table,
                     C3_SUBSET_SIZES, rhs_vector, config, mlp_init, MU_RANGE, LAM_RANGE,
                     four_param_table)

__all__ = [
    "Operators", "conv_diff_2d", "laplace5_solid_2d", "graddiv9_solid_2d",
    "three_term_2d", "three_term_3d", "seven_term_2d", "four_param_table", "grid_params_little_endian", "random_params",
    "param_table", "C3_SUBSET_SIZES", "rhs_vector", "config", "mlp_init", "MU_RANGE",
    "LAM_RANGE",
]
