"""mf_solve_noalloc (the solve for callers that cannot allocate device memory) against mf_solve
through the C ABI: the same kernels, so the same bits, on two calls in a row -- the second with
a smaller plan and fewer right-hand sides, so the static scratch holds the first call's
contributions when the second starts -- plus its transposed form, the oracle's solution, and the
rejection of a right-hand-side block larger than the scratch."""
import numpy as np
import pytest

from tests import gpu_common as G
from tests.test_gpu_parity import _rd

pytestmark = pytest.mark.gpu


def _factored(shape, seed, nrhs, smax=0):
    import torch
    from paper_2306_08994_amd import Plan
    p = _rd(shape, seed=seed, nrhs=nrhs)
    plan = Plan(p.meshes)
    if smax:
        plan.set_tuning(smax, 0, 0, 0, 0)
    dev = G.torch_dev()
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    plan.factor(K)
    return p, plan, b


def _check(p, plan, b, transpose=False):
    import torch
    ref = plan.solve(b, transpose=transpose)
    out = torch.full_like(b, float("nan"))
    plan.solve_noalloc(b, out, transpose=transpose)
    torch.cuda.synchronize()
    got, want = out.cpu().numpy(), ref.cpu().numpy()
    assert np.array_equal(got, want)
    tree, conn, fac = G.oracle_factor(p)
    assert G.rel_err(got, G.oracle_solve(tree, fac, p.b, transpose=transpose)) <= G.TOL_SOLVE


def test_noalloc_solve_equals_solve_two_calls():
    # a plan whose upper classes take the block and rectangular solves (LDS limit 40)
    p1, plan1, b1 = _factored((40, 33), seed=3, nrhs=8, smax=40)
    _check(p1, plan1, b1)
    # the second call: a smaller plan, fewer right-hand sides, on the same scratch
    p2, plan2, b2 = _factored((9, 7), seed=4, nrhs=3)
    _check(p2, plan2, b2)
    _check(p2, plan2, b2, transpose=True)
    _check(p1, plan1, b1, transpose=True)


def test_noalloc_solve_rejects_oversized_and_unfactored():
    import torch
    from paper_2306_08994_amd import MFError, Plan
    from paper_2306_08994_amd import _lib
    p, plan, b = _factored((6, 5), seed=5, nrhs=1)
    t = plan.export_tree()
    sum_c = int((np.diff(t["front_ptr"]) - t["npiv"]).sum())    # contribution-block widths
    nrhs = _lib.MF_NOALLOC_SCRATCH_DOUBLES // sum_c + 1
    big = torch.zeros((plan.n, nrhs), dtype=torch.float64, device=b.device)
    with pytest.raises(MFError) as ei:
        plan.solve_noalloc(big, torch.empty_like(big))
    assert ei.value.code == _lib.MF_EINVAL and "above its limit" in str(ei.value)
    fresh = Plan(p.meshes)
    with pytest.raises(MFError) as ei:
        fresh.solve_noalloc(b, torch.empty_like(b))
    assert ei.value.code == _lib.MF_ESTATE
