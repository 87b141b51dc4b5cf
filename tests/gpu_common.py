"""Shared helpers of the GPU parity tests (test code only: the oracle is the reference, the HIP
path is reached through the C ABI via paper_2306_08994_amd.Plan)."""
import numpy as np

from oracle import factor as ofac
from oracle import residual as ores
from oracle import solve as osol
from oracle.tree import build_tree

# Factor-entry tolerance per front F: |dL_ij| <= TOL * max(|L_ij|, max|L_F|) (same for U).  The
# GPU uses fused multiply-adds and a blocked order, so entries differ from the oracle by rounding
# only; entrywise relative error alone is meaningless on entries that cancel to ~0.
TOL_FACTOR = 1e-10
TOL_SOLVE = 1e-10        # ||x - x_oracle|| / ||x_oracle|| per right-hand side
TOL_RELRES = 1e-12


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def oracle_factor(problem):
    tree = build_tree(problem.meshes)
    conn = ofac.global_connectivity(problem)
    return tree, conn, ofac.factor(tree, problem.K, conn)


def front_violation(Lg, Lo):
    """max over entries of |dL| / (max(|L_ij|, max|L_F|)) for one front."""
    if Lo.size == 0:
        return 0.0
    scale = np.maximum(np.abs(Lo), np.abs(Lo).max())
    scale[scale == 0] = 1.0
    return float(np.max(np.abs(Lg - Lo) / scale))


def factor_violation(Ls, Us, fac, fronts=None):
    worst = 0.0
    idx = range(len(fac.L)) if fronts is None else fronts
    for f in idx:
        worst = max(worst, front_violation(Ls[f], fac.L[f]), front_violation(Us[f], fac.U[f]))
    return worst


def rel_err(x, xo):
    x2 = x.reshape(x.shape[0], -1)
    xo2 = xo.reshape(xo.shape[0], -1)
    return float(np.max(np.linalg.norm(x2 - xo2, axis=0) / np.linalg.norm(xo2, axis=0)))


def relres(problem, conn, x):
    return ores.relres(problem.K, conn, x, problem.b)


def oracle_solve(tree, fac, b, transpose=False):
    return osol.solve_t(tree, fac, b) if transpose else osol.solve(tree, fac, b)
