"""Oracle: dense cross-checks on small systems (test infrastructure only).

* ``assemble``: the global matrix A = sum_e P_e^T K_e P_e (the left-hand side assembled "by
  combining the elemental matrices based on mesh connectivity", Sec. 2.4 step 2).
* ``elimination_order``: pivots of every front, classes 0..H, fronts ascending, pivots in
  index-list order -- the order in which the multifrontal method eliminates unknowns.
* ``lu_nopivot``: right-looking Gaussian elimination without pivoting of a dense matrix with the
  same division task (row scaled by its pivot, Sec. 3), giving A = L U with diag(L) = pivots and
  U unit upper.  Without pivoting this factorization is unique, so on the permuted matrix it is
  exactly what the multifrontal method must reproduce (Sec. 1.1: the method is LU / Gaussian
  elimination organised over the tree).
"""
from __future__ import annotations

import numpy as np

from .tree import Tree


def assemble(K: np.ndarray, conn: np.ndarray, n: int) -> np.ndarray:
    A = np.zeros((n, n))
    for e in range(conn.shape[0]):
        idx = conn[e]
        A[np.ix_(idx, idx)] += K[e]
    return A


def elimination_order(tree: Tree) -> np.ndarray:
    out = []
    for lvl in tree.levels():
        for f in lvl:
            out.extend(int(v) for v in tree.pivots(int(f)))
    return np.array(out, dtype=np.int64)


def lu_nopivot(A: np.ndarray):
    W = np.array(A, dtype=np.float64, copy=True)
    n = W.shape[0]
    L = np.zeros((n, n))
    U = np.eye(n)
    for p in range(n):
        piv = W[p, p]
        if piv == 0.0 or not np.isfinite(piv):
            raise ZeroDivisionError(f"zero pivot at {p}")
        t1 = W[p, p + 1:] / piv
        W[p + 1:, p + 1:] = W[p + 1:, p + 1:] - np.multiply.outer(W[p + 1:, p], t1)
        L[p:, p] = W[p:, p]
        U[p, p + 1:] = t1
    return L, U


def brute_solve(K: np.ndarray, conn: np.ndarray, n: int, b: np.ndarray, transpose=False):
    A = assemble(K, conn, n)
    return np.linalg.solve(A.T if transpose else A, b)
