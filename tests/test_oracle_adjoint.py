"""Pins for the oracle's adjoint: dense adjoint vs multifrontal adjoint, and both against central
finite differences of the loss (a construction that never uses the adjoint identities)."""
import numpy as np

from fixtures.mesh import element_matrices, reaction_diffusion
from oracle import adjoint
from oracle.factor import global_connectivity
from oracle.tree import build_tree


def _setup(shape=(3, 4), nrhs=2):
    p = reaction_diffusion("adj", shape, np.random.default_rng(5), "lognormal", 0.5, nrhs)
    kt = np.exp(np.random.default_rng(50).normal(0, 0.5, p.meshes[0].n_elem))
    Kt = element_matrices(p.meshes[0], kt)
    conn = global_connectivity(p)
    from oracle import dense
    u_t = np.linalg.solve(dense.assemble(Kt, conn, p.n), p.b)
    return p, conn, u_t


def _loss_at(p, conn, k, b, u_t):
    from oracle import dense
    K = element_matrices(p.meshes[0], k)
    return adjoint.loss(np.linalg.solve(dense.assemble(K, conn, p.n), b), u_t)


def test_mf_adjoint_equals_dense_adjoint():
    p, conn, u_t = _setup((4, 5), 3)
    t = build_tree(p.meshes)
    S = p.S[0]
    ud, lamd, gKd, gkd = adjoint.dense_grads(p.K, conn, p.n, p.b, u_t, S)
    um, lamm, gKm, gkm = adjoint.mf_grads(t, p.K, conn, p.b, u_t, S)
    np.testing.assert_allclose(um, ud, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(lamm, lamd, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(gkm, gkd, rtol=1e-10, atol=1e-13)


def test_adjoint_against_finite_differences():
    p, conn, u_t = _setup((3, 4), 2)
    _, lam, gK, gk = adjoint.dense_grads(p.K, conn, p.n, p.b, u_t, p.S[0])
    h = 1e-6
    for e in range(p.meshes[0].n_elem):
        kp = p.coef.copy(); kp[e] += h
        km = p.coef.copy(); km[e] -= h
        fd = (_loss_at(p, conn, kp, p.b, u_t) - _loss_at(p, conn, km, p.b, u_t)) / (2 * h)
        assert abs(fd - gk[e]) <= 1e-6 * max(abs(gk[e]), 1e-2 * np.abs(gk).max())
    for i, r in [(0, 0), (5, 1), (p.n - 1, 0)]:
        bp = p.b.copy(); bp[i, r] += h
        bm = p.b.copy(); bm[i, r] -= h
        fd = (_loss_at(p, conn, p.coef, bp, u_t) - _loss_at(p, conn, p.coef, bm, u_t)) / (2 * h)
        assert abs(fd - lam[i, r]) <= 1e-6 * max(abs(lam[i, r]), 1e-2 * np.abs(lam).max())
