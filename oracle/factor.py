"""Oracle: sequential FP64 multifrontal partial LU (test infrastructure only).

Follows the multifrontal driver and the front computation of Table 2 together with the Schur
complement algebra of Sec. 2.2:
  * classes (tree levels) are processed in order 0..H, fronts of one class in ascending id;
  * a front is assembled from zero: a leaf receives its element matrix, an internal front the
    contribution blocks of its left then right child through the extend-add maps (the "join"
    of adjacent fronts, Sec. 2.3/2.4);
  * for each of its k pivots p, in index-list order: the division task
        t1[j] = F[p, j] / F[p, p]              for j > p,
    then the multiplication task  t2[i, j] = t1[j] * F[i, p]  and the subtraction task
        F[i, j] = F[i, j] - t2[i, j]            for i, j > p
    (Sec. 3 task alphabet, division -> multiplication -> subtraction, each a separate IEEE
    operation: no fused multiply-add);
  * the factor keeps L[:, p] = F[p:, p] (pivot included) and U[p, j] = t1[j] (unit diagonal), so
    the assembled matrix permuted to elimination order equals L U;
  * the trailing block F[k:, k:] is the Schur complement (contribution block) handed to the
    parent; at the root it is empty.
There is no pivoting (the paper divides by F[p, p] unconditionally); a zero or non-finite pivot
raises ZeroPivot.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tree import Tree


class ZeroPivot(ArithmeticError):
    def __init__(self, front: int, pivot: int, value: float):
        super().__init__(f"zero or non-finite pivot {value!r} in front {front}, pivot {pivot}")
        self.front, self.pivot, self.value = front, pivot, value


@dataclass
class Factors:
    L: list     # per front: (m, k) lower trapezoid, L[i, p] = 0 for i < p, diagonal = pivots
    U: list     # per front: (k, m) unit upper trapezoid, U[p, j] = 0 for j < p


def assemble_front(tree: Tree, f: int, K: np.ndarray, conn: np.ndarray, cbs: list) -> np.ndarray:
    m = tree.m(f)
    Fm = np.zeros((m, m))
    e = int(tree.leaf_elem[f])
    if e >= 0:
        pos = tree.leaf_map(f, conn[e])
        Fm[np.ix_(pos, pos)] += K[e]
    else:
        for c in (int(tree.left[f]), int(tree.right[f])):
            pos = tree.child_map(f, c)
            Fm[np.ix_(pos, pos)] += cbs[c]
            cbs[c] = None           # consumed
    return Fm


def eliminate(Fm: np.ndarray, k: int, front: int = -1):
    """Partial elimination of the first k pivots of the dense front Fm (modified in place).
    Returns (L, U); Fm[k:, k:] is left holding the Schur complement."""
    m = Fm.shape[0]
    L = np.zeros((m, k))
    U = np.zeros((k, m))
    for p in range(k):
        piv = Fm[p, p]
        if piv == 0.0 or not np.isfinite(piv):
            raise ZeroPivot(front, p, float(piv))
        t1 = Fm[p, p + 1:] / piv                       # division tasks
        t2 = np.multiply.outer(Fm[p + 1:, p], t1)      # multiplication tasks
        Fm[p + 1:, p + 1:] = Fm[p + 1:, p + 1:] - t2   # subtraction tasks
        L[p:, p] = Fm[p:, p]
        U[p, p] = 1.0
        U[p, p + 1:] = t1
    return L, U


def factor(tree: Tree, K: np.ndarray, conn: np.ndarray) -> Factors:
    """Multifrontal factorization of the system given by element matrices K (sum E, npe, npe)
    and global connectivity conn (sum E, npe) (node ids already offset for a batch)."""
    F = tree.n_fronts
    L = [None] * F
    U = [None] * F
    cbs = [None] * F
    for lvl in tree.levels():
        for f in lvl:
            f = int(f)
            Fm = assemble_front(tree, f, K, conn, cbs)
            k = int(tree.npiv[f])
            L[f], U[f] = eliminate(Fm, k, f)
            cbs[f] = Fm[k:, k:].copy()
    return Factors(L, U)


def global_connectivity(problem) -> np.ndarray:
    """Element connectivity of a batch with node ids offset by each mesh's node prefix sum."""
    offs = problem.node_offsets
    return np.concatenate([m.conn.astype(np.int64) + offs[i] for i, m in enumerate(problem.meshes)])
