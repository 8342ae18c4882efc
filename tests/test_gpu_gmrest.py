"""GMREST (restarted GMRES with truncation, the paper's second low-rank
solver, Sec. 4.1 and Table 1) through the C ABI (lrc_opts.solver) against
the oracle (oracle/gmrest.py): the tolerance is met (checked densely on the
host), the Arnoldi step count is the oracle's +-1, and the error against the
exact column-wise solution is of the oracle's size.  Both solvers reach the
same accuracy; GMREST needs no spectrum interval."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import chebyshev as och
from oracle import driver as odrv
from oracle import gmrest as ogm
from oracle import lowrank as olr
from workloads import config

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_2008_10275_amd import lrcheb
    return lrcheb


@pytest.mark.parametrize("name,tol", [("c1", 1e-8), ("q7", 1e-6)])
def test_gmrest_matches_oracle(L, name, tol):
    cfg = config(name)
    K, d, f = cfg["ops"].K, cfg["d"], cfg["f"]
    m = d.shape[1]
    cap, tt = cfg["rank_cap"], cfg["trunc_tol"]
    say("gmrest", name, len(K), m, cap)
    ctx = L.Context(0)
    ops = L.Operators(ctx, K)
    prob = L.Problem(ops, d, f[:, None], np.ones((m, 1)))
    prob.precondition()
    # the oracle solves the median column directly: the GPU's median solve
    # runs to 1e-12 here, so that both start from the same right-hand side
    # (at the default 1e-6 its error is ~100x the c1 target, which restarted
    # GMRES spends a cycle on)
    code, info = prob.solve(rank_cap=cap, trunc_tol=tt, res_tol=tol, init=L.LRC_INIT_MEDIAN,
                            solver=L.LRC_SOLVER_GMREST, median_tol=1e-12)
    # oracle: the same Newton-step form (median guess, B = F - L(x~ 1^T))
    jmed = odrv.upper_median_offset(m)
    xt = spla.splu(sp.csc_matrix(olr.column_operator(K, d, jmed))).solve(f)
    B = odrv.median_rhs(K, d, f, xt)
    P = och.mean_preconditioner(K, och.mean_parameters(d))
    ref = np.linalg.norm(f) * np.sqrt(m)
    S, oinfo = ogm.gmrest(K, d, B, och.DirectPreconditioner(P), cap, tt, tol, ref)
    say("gpu", info["iters"], info["relres"], "oracle", oinfo.iters, oinfo.cycles)
    assert code == 0 and info["relres"] <= tol and oinfo.converged
    assert abs(info["iters"] - oinfo.iters) <= 1
    U, s, V = prob.solution()
    X = U @ np.diag(s) @ V.T
    F = np.outer(f, np.ones(m))
    assert olr.relres_dense(K, d, X, F) <= 1.01 * tol
    Xs = olr.solve_columns(K, d, F)
    Xo = np.outer(xt, np.ones(m)) + S[0] @ np.diag(S[1]) @ S[2].T
    e_gpu = np.linalg.norm(X - Xs) / np.linalg.norm(Xs)
    e_orc = np.linalg.norm(Xo - Xs) / np.linalg.norm(Xs)
    say("error vs exact", e_gpu, e_orc)
    assert e_gpu <= 10 * e_orc + 1e-12
