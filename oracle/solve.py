"""Oracle: substitution over the elimination tree (test infrastructure only).

The paper solves after factorization by substitution that walks the tree from the root back to
the leaves (Sec. 1.1; the final step of the multifrontal driver in Table 2).  With A permuted to
elimination order equal to L U (L lower with the pivots on its diagonal, U unit upper, as the
division tasks of Sec. 3 produce), the solve is
  forward   L y = b : classes 0..H, fronts in ascending id, pivots in order:
            y_p = w_p / L_pp, then w_i -= L_ip y_p for the later rows i of the front;
  backward  U x = y : classes H..0, fronts in descending id, pivots in reverse order:
            x_p = y_p - sum_{j > p} U_pj x_j over the front's later columns.
Transposed (A^T lambda = g, used by the adjoint):
  U^T z = g : classes 0..H, pivots in order: z_p final, then z_j -= U_pj z_p for later j;
  L^T lam = z : classes H..0, pivots in reverse: lam_p = (z_p - sum_{i>p} L_ip lam_i) / L_pp.
All vectors are (n, nrhs) and updated in place on a global copy; the classes run sequentially,
so there is no concurrency to resolve here.
"""
from __future__ import annotations

import numpy as np

from .factor import Factors
from .tree import Tree


def forward(tree: Tree, fac: Factors, b: np.ndarray) -> np.ndarray:
    y = np.array(b, dtype=np.float64, copy=True)
    for lvl in tree.levels():
        for f in lvl:
            f = int(f)
            idx = tree.index_list(f)
            L = fac.L[f]
            for p in range(int(tree.npiv[f])):
                y[idx[p]] = y[idx[p]] / L[p, p]
                y[idx[p + 1:]] -= np.multiply.outer(L[p + 1:, p], y[idx[p]])
    return y


def backward(tree: Tree, fac: Factors, y: np.ndarray) -> np.ndarray:
    x = np.array(y, dtype=np.float64, copy=True)
    for lvl in reversed(tree.levels()):
        for f in lvl[::-1]:
            f = int(f)
            idx = tree.index_list(f)
            U = fac.U[f]
            for p in range(int(tree.npiv[f]) - 1, -1, -1):
                x[idx[p]] = x[idx[p]] - U[p, p + 1:] @ x[idx[p + 1:]]
    return x


def solve(tree: Tree, fac: Factors, b: np.ndarray) -> np.ndarray:
    b2 = b.reshape(b.shape[0], -1)
    return backward(tree, fac, forward(tree, fac, b2)).reshape(b.shape)


def forward_t(tree: Tree, fac: Factors, g: np.ndarray) -> np.ndarray:
    z = np.array(g, dtype=np.float64, copy=True)
    for lvl in tree.levels():
        for f in lvl:
            f = int(f)
            idx = tree.index_list(f)
            U = fac.U[f]
            for p in range(int(tree.npiv[f])):
                z[idx[p + 1:]] -= np.multiply.outer(U[p, p + 1:], z[idx[p]])
    return z


def backward_t(tree: Tree, fac: Factors, z: np.ndarray) -> np.ndarray:
    lam = np.array(z, dtype=np.float64, copy=True)
    for lvl in reversed(tree.levels()):
        for f in lvl[::-1]:
            f = int(f)
            idx = tree.index_list(f)
            L = fac.L[f]
            for p in range(int(tree.npiv[f]) - 1, -1, -1):
                lam[idx[p]] = (lam[idx[p]] - L[p + 1:, p] @ lam[idx[p + 1:]]) / L[p, p]
    return lam


def solve_t(tree: Tree, fac: Factors, g: np.ndarray) -> np.ndarray:
    g2 = g.reshape(g.shape[0], -1)
    return backward_t(tree, fac, forward_t(tree, fac, g2)).reshape(g.shape)
