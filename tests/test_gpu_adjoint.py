"""GPU: the differentiable solve (torch.autograd.Function over the transposed multifrontal
solve) against the oracle's dense adjoint on small meshes, and against finite differences on 32
seeded coefficients at the 128 x 128, 64-RHS workload (central h = 1e-6, and a fourth-order
stencil at H = 1e-4)."""
import numpy as np
import pytest

from fixtures import config_problem
from fixtures.mesh import element_matrices, reaction_diffusion
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _loss(plan, k, b, S, M, u_t):
    import torch
    from paper_2306_08994_amd import mf_solve
    K = k[:, None, None] * S + M
    u = mf_solve(K, b, plan)
    return ((u - u_t) ** 2).sum()


@pytest.mark.parametrize("shape,nrhs", [((4, 5), 3), ((3, 3, 2), 2), ((17, 9), 4)])
def test_adjoint_matches_oracle_dense(shape, nrhs):
    import torch
    from oracle import adjoint as oadj
    from oracle.factor import global_connectivity
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = reaction_diffusion("adj", shape, np.random.default_rng(7), "lognormal", 0.5, nrhs)
    conn = global_connectivity(p)
    kt = np.exp(np.random.default_rng(50).normal(0, 0.5, p.meshes[0].n_elem))
    from oracle import dense
    u_t = np.linalg.solve(dense.assemble(element_matrices(p.meshes[0], kt), conn, p.n), p.b)
    _, lam_o, _, gk_o = oadj.dense_grads(p.K, conn, p.n, p.b, u_t, p.S[0])
    plan = Plan(p.meshes)
    k = torch.tensor(p.coef, device=dev, requires_grad=True)
    b = torch.tensor(p.b, device=dev, requires_grad=True)
    S = torch.tensor(p.S[0], device=dev)
    M = torch.tensor(p.M[0], device=dev)
    loss = _loss(plan, k, b, S, M, torch.tensor(u_t, device=dev))
    loss.backward()
    # normwise: the dense adjoint uses LAPACK (partial pivoting), the GPU the no-pivot factors
    gk = k.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    assert np.linalg.norm(gk - gk_o) <= 1e-10 * np.linalg.norm(gk_o)
    assert G.rel_err(gb, lam_o) <= 1e-10


def test_adjoint_finite_differences_full_size():
    """128 x 128 Q1, k ~ lognormal(0, 0.5) as a parameter, 64 RHS, u_t from k_target."""
    import torch
    from paper_2306_08994_amd import Plan, mf_solve
    dev = G.torch_dev()
    p = config_problem(5)
    plan = Plan(p.meshes)
    S = torch.tensor(p.S[0], device=dev)
    M = torch.tensor(p.M[0], device=dev)
    b = torch.tensor(p.b, device=dev)
    with torch.no_grad():
        kt = torch.tensor(p.extra["k_target"], device=dev)
        u_t = mf_solve(kt[:, None, None] * S + M, b, plan)
    k = torch.tensor(p.coef, device=dev, requires_grad=True)
    bb = b.clone().requires_grad_(True)
    loss = _loss(plan, k, bb, S, M, u_t)
    loss.backward()
    gk = k.grad.cpu().numpy()
    gb = bb.grad.cpu().numpy()
    rng = np.random.default_rng(55)
    coords = rng.choice(p.meshes[0].n_elem, size=32, replace=False)
    h = 1e-6

    def u_of(kk, bb_):
        return mf_solve(kk[:, None, None] * S + M, bb_, plan)

    def dloss(up, um):
        # L(+) - L(-) = sum (u+ - u-)(u+ + u- - 2 u_t): the same central difference, summed
        # without cancelling two large losses against each other
        return float(((up - um) * (up + um - 2 * u_t)).sum())

    # The central difference at h = 1e-6 is limited by rounding at this size: cond(A) * eps / h
    # is ~1e-4 relative (measured the same with an independent sparse LU on the CPU), so it is
    # held to 1e-3; a fourth-order stencil at H = 1e-4 (truncation ~H^4) is held to 2e-5.
    H = 1e-4
    worst2 = worst4 = 0.0
    with torch.no_grad():
        for e in coords:
            def u_at(dk):
                kk = k.detach().clone()
                kk[e] += dk
                return u_of(kk, b)
            fd = dloss(u_at(h), u_at(-h)) / (2 * h)
            u1, u2, u3, u4 = u_at(2 * H), u_at(H), u_at(-H), u_at(-2 * H)
            fd4 = (-dloss(u1, u4) + 8 * dloss(u2, u3)) / (12 * H)
            scale = max(abs(gk[e]), 1e-2 * np.abs(gk).max())
            worst2 = max(worst2, abs(fd - gk[e]) / scale)
            worst4 = max(worst4, abs(fd4 - gk[e]) / scale)
            assert abs(fd - gk[e]) <= 1e-3 * scale, (e, fd, gk[e])
            assert abs(fd4 - gk[e]) <= 2e-5 * scale, (e, fd4, gk[e])
        kd = k.detach()
        for (i, r) in zip(rng.choice(p.n, 4, replace=False), rng.choice(p.nrhs, 4)):
            bp = b.clone(); bp[i, r] += h
            bm = b.clone(); bm[i, r] -= h
            fd = dloss(u_of(kd, bp), u_of(kd, bm)) / (2 * h)
            assert abs(fd - gb[i, r]) <= 1e-5 * max(abs(gb[i, r]), 1e-2 * np.abs(gb).max())
    print(f"finite differences vs adjoint on 32 coefficients: central h=1e-6 worst rel "
          f"{worst2:.2e}, 4-point H=1e-4 worst rel {worst4:.2e}")


def test_stale_factors_rejected():
    import torch
    from paper_2306_08994_amd import Plan, mf_solve
    dev = G.torch_dev()
    p = reaction_diffusion("adj", (3, 3), np.random.default_rng(1), "lognormal", 0.5, 1)
    plan = Plan(p.meshes)
    K = torch.tensor(p.K, device=dev, requires_grad=True)
    b = torch.tensor(p.b, device=dev)
    u = mf_solve(K, b, plan)
    with torch.no_grad():
        mf_solve(K * 2, b, plan)          # refactors the same plan
    with pytest.raises(RuntimeError):
        u.sum().backward()
