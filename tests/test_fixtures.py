"""Pins for the seeded input generator: element matrices against textbook closed forms and an
independent tensor-product construction, mesh numbering, and the workload recipes."""
import numpy as np
import pytest

from fixtures import config_problem, q1_reference_matrices, structured_q1


def _1d(h):
    k = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    c = np.array([[-0.5, 0.5], [-0.5, 0.5]])          # int phi_a phi_b'
    return k, m, c


def test_unit_square_closed_forms():
    S, M, C = q1_reference_matrices((1.0, 1.0))
    S_ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    M_ref = np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]]) / 36.0
    np.testing.assert_allclose(S, S_ref, rtol=0, atol=1e-15)
    np.testing.assert_allclose(M, M_ref, rtol=0, atol=1e-16)


@pytest.mark.parametrize("h", [(0.25, 0.5), (1 / 3, 1 / 7), (0.5, 0.25, 0.125), (1.0, 1.0, 1.0)])
def test_tensor_product_construction(h):
    S, M, C = q1_reference_matrices(h)
    parts = [_1d(x) for x in h]
    # local index a = c_x + 2 c_y (+4 c_z): kron with the last axis outermost
    def kron(mats):
        out = mats[-1]
        for A in mats[-2::-1]:
            out = np.kron(out, A)
        return out
    dim = len(h)
    S_ref = sum(kron([parts[e][0] if e == d else parts[e][1] for e in range(dim)])
                for d in range(dim))
    M_ref = kron([p[1] for p in parts])
    np.testing.assert_allclose(S, S_ref, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(M, M_ref, rtol=1e-13, atol=1e-17)
    for d in range(dim):
        C_ref = kron([parts[e][2] if e == d else parts[e][1] for e in range(dim)])
        np.testing.assert_allclose(C[d], C_ref, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(C[d].sum(axis=1), 0.0, atol=1e-15)
    np.testing.assert_allclose(S.sum(axis=1), 0.0, atol=1e-13)
    assert abs(M.sum() - np.prod(h)) < 1e-15


def test_mesh_numbering_2x2():
    m = structured_q1((2, 2))
    # element (i,j) id i + 2j; node (i,j) id i + 3j; local a = cx + 2 cy
    np.testing.assert_array_equal(m.conn, [[0, 1, 3, 4], [1, 2, 4, 5], [3, 4, 6, 7], [4, 5, 7, 8]])
    np.testing.assert_array_equal(m.ijk, [[0, 0], [1, 0], [0, 1], [1, 1]])
    assert m.n_nodes == 9 and m.n_elem == 4


def test_mesh_numbering_3d():
    m = structured_q1((2, 1, 1))
    np.testing.assert_array_equal(m.conn[1], [1, 2, 4, 5, 7, 8, 10, 11])
    np.testing.assert_array_equal(m.ijk, [[0, 0, 0], [1, 0, 0]])


def test_recipes():
    p1 = config_problem(1)
    assert p1.n == 289 and p1.K.shape == (256, 4, 4) and p1.b.shape == (289, 1)
    assert p1.coef.min() >= 0.5 and p1.coef.max() <= 2.0
    p5 = config_problem(5, shape=(8, 8))
    assert p5.b.shape == (81, 64) and "k_target" in p5.extra
    # batched recipe: sides drawn first from the config seed
    rng = np.random.default_rng(4)
    sides = rng.integers(32, 129, size=(256, 2))
    assert int(((sides[:, 0] + 1) * (sides[:, 1] + 1)).sum()) == 1717098
    assert int((sides[:, 0] * sides[:, 1]).sum()) == 1675297


def test_peclet_bound_and_row_sums():
    p = config_problem(4, n_mesh=3, side_range=(4, 9))
    off = 0
    for mesh in p.meshes:
        D = p.coef[off:off + mesh.n_elem]
        v = p.vel[off:off + mesh.n_elem]
        pe = np.linalg.norm(v, axis=1) * max(mesh.h) / (2 * D)
        assert pe.max() <= 0.9 + 1e-12
        off += mesh.n_elem
    # diffusion + advection rows sum to the mass row sums (stiffness and advection rows sum to 0)
    M_rows = np.concatenate([np.repeat(M.sum(axis=1)[None], m.n_elem, 0)
                             for M, m in zip(p.M, p.meshes)])
    np.testing.assert_allclose(p.K.sum(axis=2), M_rows, atol=1e-12)


def test_zero_coefficient_is_mass_matrix():
    from fixtures.mesh import reaction_diffusion
    p = reaction_diffusion("l2", (3, 2), np.random.default_rng(0), "zero", 0.0, 1)
    _, M, _ = q1_reference_matrices(p.meshes[0].h)
    np.testing.assert_array_equal(p.K, np.repeat(M[None], 6, 0))
