"""mf_factor_refine: the factorization and the refined solve in one call, with the forward sweep
of the first solve overlapped with the factorization on a second stream.  The same kernels run
in the same per-class order as mf_factor followed by mf_refine, so the factors and x must be
bit-identical to those two calls (replayed from their captured graphs or launched eagerly), and
the refined solution meets the residual bar against the oracle's operator."""
import numpy as np
import pytest

from fixtures import config_problem, reaction_diffusion
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _problem(case):
    rng = np.random.default_rng(3)
    if case == "2d-lds":
        return reaction_diffusion("t", (37, 29), rng, "lognormal", 1.0, 8), (0, 0, 0, 0)
    if case == "2d-tiled":
        return reaction_diffusion("t", (70, 61), rng, "lognormal", 1.0, 3), (64, 32, -1, 32)
    if case == "3d":
        return reaction_diffusion("t", (9, 8, 7), rng, "lognormal", 1.0, 2), (0, 0, 0, 0)
    if case == "batch":
        return config_problem(4, n_mesh=5, side_range=(8, 24), nrhs=2), (0, 0, 0, 0)
    raise ValueError(case)


def _plan(p, tuning):
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    plan = Plan(p.meshes)
    if any(tuning):
        plan.set_tuning(*tuning)
    return plan, torch.from_numpy(p.K).to(dev), torch.from_numpy(p.b).to(dev)


@pytest.mark.parametrize("case", ["2d-lds", "2d-tiled", "3d", "batch"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_equals_factor_then_refine(case, prec):
    import torch
    p, tuning = _problem(case)
    conn = G.ofac.global_connectivity(p)
    plan, K, b = _plan(p, tuning)
    ref_plan, _, _ = _plan(p, tuning)
    x = torch.empty_like(b)
    for rep in range(3):                          # repeated calls on the same buffers
        Kr = (K * (1.0 + 0.5 * rep)).contiguous()
        ref_plan.factor(Kr, prec)
        xr, itr, rrr = ref_plan.refine(Kr, b, tol=1e-12, max_it=30)
        Lr, Ur = ref_plan.export_factors()
        xg, its, rr = plan.factor_refine(Kr, b, prec, tol=1e-12, max_it=30, x=x)
        Lg, Ug = plan.export_factors()
        for f in range(len(Lr)):
            np.testing.assert_array_equal(Lr[f], Lg[f])
            np.testing.assert_array_equal(Ur[f], Ug[f])
        torch.testing.assert_close(xg, xr, rtol=0, atol=0)
        assert (its, rr) == (itr, rrr)
        if rep == 0:                              # Kr = K: the oracle's operator
            assert G.relres(p, conn, xg.cpu().numpy()) <= 1e-12
        plan.solve(b)                             # eager work between the replays


def test_equals_profiled_run():
    import torch
    p, tuning = _problem("2d-tiled")
    plan, K, b = _plan(p, tuning)
    plan.profile(True)                            # every launch bracketed by events
    xe, ite, rre = plan.factor_refine(K, b)
    xe = xe.clone()
    plan.profile(False)
    for _ in range(2):
        xg, itg, rrg = plan.factor_refine(K, b)
        torch.testing.assert_close(xg, xe, rtol=0, atol=0)
        assert (itg, rrg) == (ite, rre)


def test_zero_pivot_and_recovery():
    from paper_2306_08994_amd import MFError
    from paper_2306_08994_amd import _lib
    p, tuning = _problem("2d-lds")
    plan, K, b = _plan(p, tuning)
    Kbad = K.clone()
    Kbad[0, 0, 0] = 0.0                           # the domain corner is a leaf pivot
    with pytest.raises(MFError) as ei:
        plan.factor_refine(Kbad, b)
    assert ei.value.code == _lib.MF_EZERO_PIVOT
    with pytest.raises(MFError) as ei:
        plan.solve(b)
    assert ei.value.code == _lib.MF_ESTATE
    x, its, rr = plan.factor_refine(K, b)
    assert rr <= 1e-12
    with pytest.raises(ValueError):
        plan.factor_refine(K, b, precision="fp16")


def test_full_size_equals_factor_then_refine():
    """The 256 x 256 workload with 8 right-hand sides in the benchmark's configuration."""
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(2)
    conn = G.ofac.global_connectivity(p)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    ref = Plan(p.meshes)
    ref.set_tuning(64, 32, -1, 32)
    ref.factor(K)
    xr, itr, rrr = ref.refine(K, b, tol=1e-12, max_it=5)
    plan = Plan(p.meshes)
    plan.set_tuning(64, 32, -1, 32)
    x = torch.empty_like(b)
    for _ in range(2):
        xg, its, rr = plan.factor_refine(K, b, tol=1e-12, max_it=5, x=x)
        torch.testing.assert_close(xg, xr, rtol=0, atol=0)
    assert (its, rr) == (itr, rrr) and rr <= 1e-12
    assert G.relres(p, conn, xg.cpu().numpy()) <= 1e-12


def test_plan_without_graphs_equals_graph_replay(monkeypatch):
    """MF_GRAPHS=0 at plan creation: the same launch sequences issued eagerly give the same bits
    as the captured graphs (factor, solve, transposed solve)."""
    import torch
    p, tuning = _problem("2d-tiled")
    graphed, K, b = _plan(p, tuning)
    monkeypatch.setenv("MF_GRAPHS", "0")
    eager, _, _ = _plan(p, tuning)
    for plan in (graphed, eager):
        for _ in range(2):                        # the second call replays a captured graph
            plan.factor(K)
    Lg, Ug = graphed.export_factors()
    Le, Ue = eager.export_factors()
    for f in range(len(Lg)):
        np.testing.assert_array_equal(Lg[f], Le[f])
        np.testing.assert_array_equal(Ug[f], Ue[f])
    for tr in (False, True):
        xg = graphed.solve(b, transpose=tr)
        xg = graphed.solve(b, transpose=tr).clone()
        xe = eager.solve(b, transpose=tr)
        torch.testing.assert_close(xg, xe, rtol=0, atol=0)
