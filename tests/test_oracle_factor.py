"""Pins for the oracle's multifrontal factorization and solves.

  * Dense unpivoted LU (the exact definition of what the method computes) is itself pinned by
    reconstruction (L U = A, L lower, U unit upper), then the multifrontal factors are compared
    entry by entry with it in elimination order;
  * entries of the dense factor outside a front's index list are exactly 0.0 (the front
    pattern holds all fill);
  * sum log|L_pp| = log|det A| and the sign matches (numpy slogdet);
  * symmetric (SPD) systems: L_ip = L_pp U_pi and every pivot positive;
  * one element: the factor is the dense LU of the element matrix;
  * solves against numpy.linalg.solve (plain and transposed), residual below 1e-12;
  * zero coefficient: the paper's L2-projection mass system; a zero corner diagonal: ZeroPivot.
"""
import numpy as np
import pytest

from fixtures import config_problem, structured_q1
from fixtures.mesh import element_matrices, reaction_diffusion
from oracle import dense, residual
from oracle.factor import ZeroPivot, factor, global_connectivity
from oracle.solve import solve, solve_t
from oracle.tree import build_tree


def _problem(shape, seed=0, kind="lognormal", sigma=1.0, nrhs=2):
    return reaction_diffusion("t", shape, np.random.default_rng(seed), kind, sigma, nrhs)


def _global_factors(tree, fac, order):
    n = tree.n
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    L = np.zeros((n, n))
    U = np.zeros((n, n))
    for f in range(tree.n_fronts):
        idx = pos[tree.index_list(f)]
        k = int(tree.npiv[f])
        if k == 0:
            continue
        L[np.ix_(idx, idx[:k])] = fac.L[f]
        U[np.ix_(idx[:k], idx)] = fac.U[f]
    return L, U


def test_dense_lu_definition():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(9, 9)) + 9 * np.eye(9)
    L, U = dense.lu_nopivot(A)
    assert np.allclose(np.triu(L, 1), 0) and np.allclose(np.tril(U, -1), 0)
    np.testing.assert_array_equal(np.diag(U), 1.0)
    np.testing.assert_allclose(L @ U, A, rtol=0, atol=1e-13)


SHAPES = [(1, 1), (1, 2), (2, 2), (4, 4), (3, 5), (2, 2, 2), (3, 2, 2), (16, 16)]


@pytest.mark.parametrize("shape", SHAPES)
def test_multifrontal_equals_dense_lu(shape):
    p = _problem(shape)
    conn = global_connectivity(p)
    t = build_tree(p.meshes)
    fac = factor(t, p.K, conn)
    A = dense.assemble(p.K, conn, p.n)
    order = dense.elimination_order(t)
    AP = A[np.ix_(order, order)]
    Ld, Ud = dense.lu_nopivot(AP)
    np.testing.assert_allclose(Ld @ Ud, AP, rtol=0, atol=1e-12 * np.abs(A).max())
    Lm, Um = _global_factors(t, fac, order)
    scale = np.abs(Ld).max()
    np.testing.assert_allclose(Lm, Ld, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(Um, Ud, rtol=0, atol=1e-12 * max(1.0, np.abs(Ud).max()))
    # the front pattern holds every nonzero of the dense factor (fill stays inside fronts)
    assert np.all(Ld[Lm == 0] == 0.0) and np.all(Ud[Um == 0] == 0.0)
    # determinant
    sign, logdet = np.linalg.slogdet(A)
    piv = np.diag(Lm)
    assert np.prod(np.sign(piv)) == sign
    assert abs(np.log(np.abs(piv)).sum() - logdet) <= 1e-10 * max(1.0, abs(logdet))
    # symmetric positive definite: positive pivots, L_ip = L_pp U_pi
    assert np.all(piv > 0)
    np.testing.assert_allclose(Lm, (Um * piv[:, None]).T, rtol=0, atol=1e-12 * scale)


def test_single_element_is_dense_lu_of_element_matrix():
    p = _problem((1, 1))
    t = build_tree(p.meshes)
    fac = factor(t, p.K, global_connectivity(p))
    assert t.n_fronts == 1 and t.npiv[0] == 4
    L, U = dense.lu_nopivot(p.K[0])
    np.testing.assert_allclose(fac.L[0], L, rtol=1e-14, atol=0)
    np.testing.assert_allclose(fac.U[0], U, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("shape", [(1, 1), (4, 4), (3, 5), (2, 3, 2), (16, 16)])
def test_solve_matches_numpy(shape):
    p = _problem(shape, nrhs=3)
    conn = global_connectivity(p)
    t = build_tree(p.meshes)
    fac = factor(t, p.K, conn)
    A = dense.assemble(p.K, conn, p.n)
    x = solve(t, fac, p.b)
    np.testing.assert_allclose(x, np.linalg.solve(A, p.b), rtol=1e-11, atol=1e-12)
    assert residual.relres(p.K, conn, x, p.b) <= 1e-12
    assert residual.backward_error(p.K, conn, x, p.b) <= 1e-15
    xt = solve_t(t, fac, p.b)
    np.testing.assert_allclose(xt, np.linalg.solve(A.T, p.b), rtol=1e-11, atol=1e-12)


def test_nonsymmetric_batched_solve():
    p = config_problem(4, n_mesh=3, side_range=(2, 6))
    conn = global_connectivity(p)
    t = build_tree(p.meshes)
    fac = factor(t, p.K, conn)
    A = dense.assemble(p.K, conn, p.n)
    assert not np.allclose(A, A.T)
    x = solve(t, fac, p.b)
    np.testing.assert_allclose(x, np.linalg.solve(A, p.b), rtol=1e-10, atol=1e-12)
    xt = solve_t(t, fac, p.b)
    np.testing.assert_allclose(xt, np.linalg.solve(A.T, p.b), rtol=1e-10, atol=1e-12)
    assert residual.relres(p.K, conn, x, p.b) <= 1e-12


def test_config1_residual():
    p = config_problem(1)
    conn = global_connectivity(p)
    t = build_tree(p.meshes)
    x = solve(t, factor(t, p.K, conn), p.b)
    assert residual.relres(p.K, conn, x, p.b) <= 1e-13


def test_mass_matrix_l2_projection():
    p = _problem((4, 3), kind="zero")
    conn = global_connectivity(p)
    t = build_tree(p.meshes)
    x = solve(t, factor(t, p.K, conn), p.b)
    np.testing.assert_allclose(x, dense.brute_solve(p.K, conn, p.n, p.b), rtol=1e-11)


def test_zero_pivot_raises():
    p = _problem((3, 3))
    K = p.K.copy()
    K[0, 0, 0] = 0.0           # element 0, local node 0 = domain corner: a leaf pivot
    t = build_tree(p.meshes)
    with pytest.raises(ZeroPivot) as ei:
        factor(t, K, global_connectivity(p))
    assert t.leaf_elem[ei.value.front] == 0


def test_residual_operator_matches_sparse_product():
    p = _problem((5, 4), nrhs=2)
    conn = global_connectivity(p)
    x = np.random.default_rng(1).normal(size=(p.n, 2))
    A = residual.sparse_matrix(p.K, conn, p.n)
    np.testing.assert_allclose(residual.apply(p.K, conn, x), A @ x, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(A.toarray(), dense.assemble(p.K, conn, p.n), atol=1e-15)
