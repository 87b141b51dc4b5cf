"""Pins of the oracle's residual figures (oracle/residual.py) against values worked by hand.

The relative residual is the refinement's stopping test: max over right-hand sides r of
||b_r - A x_r||_2 / ||b_r||_2.  The normwise backward error is, per right-hand side,
||r||_inf / (||A||_inf ||x||_inf + ||b||_inf), and its maximum over right-hand sides is reported.

The system below is assembled from two 1D two-node "elements" on nodes (0, 1) and (1, 2):

    K_0 = [[4, 1], [0, 0.5]],   K_1 = [[0.5, 0], [1, 1]]   ->   A = [[4, 1, 0],
                                                                   [0, 1, 0],
                                                                   [0, 1, 1]]

A is nonsymmetric on purpose: ||A||_inf = 5 (row sums 5, 1, 2) differs from ||A||_1 = 4.  With

    x = [[1, 0], [0, 2], [0, 0]]      A x = [[4, 2], [0, 2], [0, 2]]
    r = [[0, 1], [3, 0], [4, 0]]      b = A x + r = [[4, 3], [3, 2], [4, 2]]

the column ratios are ||r_0||/||b_0|| = 5/sqrt(41) and ||r_1||/||b_1|| = 1/sqrt(17), so the
maximum (5/sqrt(41) = 0.7809) differs from the Frobenius ratio sqrt(26/58) = 0.6695, from the
mean of the two ratios and from the ratios of row norms.  The backward errors per column are
4/(5*1 + 4) = 4/9 and 1/(5*2 + 3) = 1/13; the reported 4/9 differs from the figure of the
whole block at once (4/(5*2 + 4) = 2/7) and from the one with ||A||_1 (4/(4 + 4) = 1/2).
"""
import numpy as np
import pytest

from oracle import residual

CONN = np.array([[0, 1], [1, 2]], dtype=np.int64)
K = np.array([[[4.0, 1.0], [0.0, 0.5]],
              [[0.5, 0.0], [1.0, 1.0]]])
X = np.array([[1.0, 0.0], [0.0, 2.0], [0.0, 0.0]])
R = np.array([[0.0, 1.0], [3.0, 0.0], [4.0, 0.0]])
B = np.array([[4.0, 3.0], [3.0, 2.0], [4.0, 2.0]])


def test_hand_system_assembles_and_applies():
    A = residual.sparse_matrix(K, CONN, 3).toarray()
    np.testing.assert_array_equal(A, [[4, 1, 0], [0, 1, 0], [0, 1, 1]])
    np.testing.assert_array_equal(residual.apply(K, CONN, X), [[4, 2], [0, 2], [0, 2]])
    np.testing.assert_array_equal(residual.residual(K, CONN, X, B), R)


def test_relres_is_max_over_rhs_of_column_ratios():
    got = residual.relres(K, CONN, X, B)
    assert got == pytest.approx(5.0 / np.sqrt(41.0), rel=1e-15)
    # what a plausible mistake would give instead
    assert abs(got - np.sqrt(26.0 / 58.0)) > 0.1                      # Frobenius ratio
    assert abs(got - 0.5 * (5 / np.sqrt(41) + 1 / np.sqrt(17))) > 0.1  # mean over columns
    assert abs(got - 1.0 / np.sqrt(17.0)) > 0.1                        # min over columns


def test_relres_single_rhs_vector():
    got = residual.relres(K, CONN, X[:, 1], B[:, 1])
    assert got == pytest.approx(1.0 / np.sqrt(17.0), rel=1e-15)
    assert residual.relres(K, CONN, X[:, 0], B[:, 0]) == pytest.approx(5 / np.sqrt(41), rel=1e-15)


def test_relres_zero_for_exact_solution():
    b = residual.apply(K, CONN, X)
    assert residual.relres(K, CONN, X, b) == 0.0


def test_backward_error_per_rhs_max():
    got = residual.backward_error(K, CONN, X, B)
    assert got == pytest.approx(4.0 / 9.0, rel=1e-15)
    assert abs(got - 2.0 / 7.0) > 0.1      # the whole block's norms at once
    assert abs(got - 0.5) > 0.05           # ||A||_1 in place of ||A||_inf
    assert residual.backward_error(K, CONN, X[:, 1], B[:, 1]) == pytest.approx(1 / 13, rel=1e-15)


def test_backward_error_scale_invariance():
    # scaling A and b together (x fixed) leaves the backward error unchanged; scaling x and b
    # together (A fixed) does too -- both follow from the definition, not from the code
    e0 = residual.backward_error(K, CONN, X, B)
    assert residual.backward_error(3.0 * K, CONN, X, 3.0 * B) == pytest.approx(e0, rel=1e-14)
    assert residual.backward_error(K, CONN, 0.25 * X, 0.25 * B) == pytest.approx(e0, rel=1e-14)
