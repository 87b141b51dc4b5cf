"""Oracle: residuals of a computed solution (test infrastructure only).

A is never formed: r = b - sum_e P_e^T K_e P_e x applies the element matrices one by one, the
same "combine the elemental matrices by connectivity" assembly of Sec. 2.4 used as an operator.
Reported figures:
  relres    max over right-hand sides of ||b - A x||_2 / ||b||_2;
  backward  normwise backward error ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf), per RHS max,
            with ||A||_inf taken from the assembled sparse matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def apply(K: np.ndarray, conn: np.ndarray, x: np.ndarray) -> np.ndarray:
    x2 = x.reshape(x.shape[0], -1)
    y = np.zeros_like(x2, dtype=np.float64)
    xe = x2[conn]                                  # (E, npe, nrhs)
    ye = np.einsum("eab,ebr->ear", K, xe)
    np.add.at(y, conn.reshape(-1), ye.reshape(-1, x2.shape[1]))
    return y.reshape(x.shape)


def residual(K, conn, x, b):
    return b - apply(K, conn, x)


def relres(K, conn, x, b) -> float:
    r = residual(K, conn, x, b).reshape(b.shape[0], -1)
    b2 = b.reshape(b.shape[0], -1)
    return float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(b2, axis=0)))


def sparse_matrix(K, conn, n):
    npe = conn.shape[1]
    rows = np.repeat(conn, npe, axis=1).reshape(-1)
    cols = np.tile(conn, (1, npe)).reshape(-1)
    return sp.coo_matrix((K.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()


def backward_error(K, conn, x, b) -> float:
    n = b.shape[0]
    A = sparse_matrix(K, conn, n)
    a_inf = float(np.max(np.abs(A).sum(axis=1)))
    r = residual(K, conn, x, b).reshape(n, -1)
    x2 = x.reshape(n, -1)
    b2 = b.reshape(n, -1)
    num = np.max(np.abs(r), axis=0)
    den = a_inf * np.max(np.abs(x2), axis=0) + np.max(np.abs(b2), axis=0)
    return float(np.max(num / den))
