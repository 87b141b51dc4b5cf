"""Pins for the quadratic and cubic (Q2, Q3) inputs and the oracle on them: the paper's
benchmark axis of linear, quadratic and cubic bases (Sec. 5) on its model problem, the L2
projection (Sec. 2.1).

  * 1D element matrices against the textbook closed forms (p = 2, 3);
  * the Q_p construction at p = 1 against the hand-written Q1 matrices, in 2D and 3D;
  * partition of unity: the mass matrix sums to the element volume, stiffness rows sum to 0;
  * the L2 projection reproduces any function of the space exactly: for f of degree <= p per
    axis the solved coefficients equal f at the nodes (the mathematics fixes this, independent
    of the oracle's tree, factors and solves);
  * the multifrontal factors equal the dense unpivoted LU in the tree's elimination order, and
    the solves match numpy on Q2/Q3 systems;
  * interior nodes of an element are pivots of its leaf front, so every leaf eliminates at
    least (p-1)^dim unknowns.
"""
import numpy as np
import pytest

from fixtures import (l2_projection, l2_workload, node_coords, q1_reference_matrices,
                      qp_reference_matrices, structured_qp, L2_SHAPES)
from fixtures.mesh import element_matrices
from oracle import dense
from oracle.factor import factor, global_connectivity
from oracle.solve import solve, solve_t
from oracle.tree import build_tree


def test_1d_closed_forms():
    h = 0.37
    S2, M2, _ = qp_reference_matrices((h,), 2)
    np.testing.assert_allclose(M2, h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(S2, 1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]),
                               rtol=0, atol=1e-13)
    S3, M3, _ = qp_reference_matrices((h,), 3)
    M3t = h / 1680 * np.array([[128, 99, -36, 19], [99, 648, -81, -36], [-36, -81, 648, 99],
                               [19, -36, 99, 128]])
    S3t = 1 / (40 * h) * np.array([[148, -189, 54, -13], [-189, 432, -297, 54],
                                   [54, -297, 432, -189], [-13, 54, -189, 148]])
    np.testing.assert_allclose(M3, M3t, rtol=0, atol=1e-15)
    np.testing.assert_allclose(S3, S3t, rtol=0, atol=1e-12)


@pytest.mark.parametrize("h", [(0.3, 0.5), (0.3, 0.5, 0.7)])
def test_p1_matches_q1(h):
    a = q1_reference_matrices(h)
    b = qp_reference_matrices(h, 1)
    for x, y in zip(a[:2], b[:2]):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-14)
    for x, y in zip(a[2], b[2]):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_partition_of_unity(dim, p):
    h = (0.3, 0.5, 0.7)[:dim]
    S, M, C = qp_reference_matrices(h, p)
    assert abs(M.sum() - np.prod(h)) < 1e-14
    assert np.abs(S.sum(axis=1)).max() < 1e-11
    for d in range(dim):
        assert np.abs(C[d].sum(axis=1)).max() < 1e-13      # derivative of the constant 1


def test_mesh_numbering():
    m = structured_qp((3, 2), 3)
    assert m.npe == 16 and m.n_nodes == 10 * 7
    assert sorted(np.unique(m.conn)) == list(range(m.n_nodes))
    # element (1, 1): lattice origin (3, 3), local node c_x + 4 c_y
    e = 1 + 3 * 1
    assert m.conn[e, 0] == 3 + 10 * 3 and m.conn[e, 15] == 6 + 10 * 6


@pytest.mark.parametrize("shape,p", [((3, 4), 2), ((3, 2), 3), ((2, 2, 3), 2), ((2, 1, 2), 3),
                                     ((5, 5), 3)])
def test_l2_projection_reproduces_the_space(shape, p):
    def f(x):
        return np.prod(1.0 + x + 0.5 * x ** p, axis=1)
    pr = l2_projection("t", shape, p, np.random.default_rng(0), 1, f=f)
    t = build_tree(pr.meshes)
    fac = factor(t, pr.K, global_connectivity(pr))
    u = solve(t, fac, pr.b)[:, 0]
    exact = f(node_coords(pr.meshes[0]))
    assert np.abs(u - exact).max() <= 1e-11 * np.abs(exact).max()


@pytest.mark.parametrize("shape,p", [((3, 3), 2), ((2, 3), 3), ((2, 1, 2), 2)])
def test_factors_are_the_dense_lu(shape, p):
    m = structured_qp(shape, p)
    coef = np.exp(np.random.default_rng(1).normal(0, 1, m.n_elem))
    K = element_matrices(m, coef)
    t = build_tree([m])
    conn = m.conn.astype(np.int64)
    fac = factor(t, K, conn)
    order = dense.elimination_order(t)
    A = dense.assemble(K, conn, m.n_nodes)[np.ix_(order, order)]
    Ld, Ud = dense.lu_nopivot(A)
    pos = np.empty(m.n_nodes, dtype=np.int64)
    pos[order] = np.arange(m.n_nodes)
    L = np.zeros_like(A)
    U = np.zeros_like(A)
    for fr in range(t.n_fronts):
        k = int(t.npiv[fr])
        if k:
            idx = pos[t.index_list(fr)]
            L[np.ix_(idx, idx[:k])] = fac.L[fr]
            U[np.ix_(idx[:k], idx)] = fac.U[fr]
    np.testing.assert_allclose(L, Ld, rtol=0, atol=1e-11 * np.abs(Ld).max())
    np.testing.assert_allclose(U, Ud, rtol=0, atol=1e-11 * np.abs(Ud).max())
    b = np.random.default_rng(2).normal(size=(m.n_nodes, 2))
    Af = dense.assemble(K, conn, m.n_nodes)
    np.testing.assert_allclose(solve(t, fac, b), np.linalg.solve(Af, b), rtol=0, atol=1e-10)
    np.testing.assert_allclose(solve_t(t, fac, b), np.linalg.solve(Af.T, b), rtol=0, atol=1e-10)


@pytest.mark.parametrize("shape,p", [((4, 4), 2), ((3, 3), 3), ((2, 2, 2), 2)])
def test_leaves_eliminate_interior_nodes(shape, p):
    m = structured_qp(shape, p)
    t = build_tree([m])
    leaves = np.nonzero(t.leaf_elem >= 0)[0]
    assert np.all(t.npiv[leaves] >= (p - 1) ** m.dim)


def test_l2_workload_sizes():
    for p, shape in L2_SHAPES.items():
        nodes = int(np.prod([p * s + 1 for s in shape]))
        assert nodes == 547 * 547 and nodes <= 300_000
    pr = l2_workload(2, shape=(4, 3), nrhs=2)
    assert pr.b.shape == (pr.n, 2) and pr.meshes[0].p == 2
