"""Oracle: gradients through the linear solve (test infrastructure only).

Not a step of the paper; it differentiates the paper's solve.  For u = A^{-1} b with
A = sum_e P_e^T K_e P_e and a loss L(u), the adjoint identities are
    lambda = A^{-T} dL/du,   dL/db = lambda,   dL/dK_e[a, b] = -sum_r lambda_r[a_e] u_r[b_e],
and with K_e = k_e S_e + M_e (+ advection), dL/dk_e = sum_ab dL/dK_e[a, b] S_e[a, b].
``dense_*`` forms A explicitly; ``mf_*`` uses the multifrontal factor and its transposed solve.
"""
from __future__ import annotations

import numpy as np

from . import dense, factor as mfac, solve as msol
from .tree import Tree


def loss(u: np.ndarray, u_t: np.ndarray) -> float:
    return float(np.sum((u - u_t) ** 2))


def elem_grad(conn: np.ndarray, lam: np.ndarray, u: np.ndarray) -> np.ndarray:
    """dL/dK_e[a, b] = -sum_r lam[conn[e, a], r] * u[conn[e, b], r]  -> (E, npe, npe)."""
    lam2 = lam.reshape(lam.shape[0], -1)
    u2 = u.reshape(u.shape[0], -1)
    return -np.einsum("ear,ebr->eab", lam2[conn], u2[conn])


def dense_grads(K, conn, n, b, u_t, S):
    A = dense.assemble(K, conn, n)
    u = np.linalg.solve(A, b)
    g = 2.0 * (u - u_t)
    lam = np.linalg.solve(A.T, g)
    gK = elem_grad(conn, lam, u)
    gk = np.einsum("eab,ab->e", gK, S)
    return u, lam, gK, gk


def mf_grads(tree: Tree, K, conn, b, u_t, S):
    fac = mfac.factor(tree, K, conn)
    u = msol.solve(tree, fac, b)
    g = 2.0 * (u - u_t)
    lam = msol.solve_t(tree, fac, g)
    gK = elem_grad(conn, lam, u)
    gk = np.einsum("eab,ab->e", gK, S)
    return u, lam, gK, gk
