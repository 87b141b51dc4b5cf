"""GPU parity of the chunked triangle solves: the pivot triangles of a class's fronts solved in
launches of 128 pivots, one workgroup per 128-row tile of the rows each chunk updates (every
workgroup solving the chunk's own triangle from the diagonal-block inverses).

Forced on meshes the oracle handles in seconds (min_pivots small), with fronts of one chunk, of
several chunks with a ragged last one, with and without contribution rows (which then take the
rectangular launches), several fronts per class, and right-hand sides spanning two LDS chunks;
checked against the oracle's solutions and against the one-workgroup block solves of the same
factors (the same arithmetic in another order: agreement to rounding).  Transposed solves keep
the block route and must be unaffected."""
import numpy as np
import pytest

from fixtures.mesh import reaction_diffusion
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _plan(shape, nrhs, seed=3):
    import torch
    from paper_2306_08994_amd import Plan
    p = reaction_diffusion("t", shape, np.random.default_rng(seed), "lognormal", 1.0, nrhs)
    dev = G.torch_dev()
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    return p, plan, K, b


# (20,20,20): root 441 pivots (chunks 128, 128, 128, 57), 210-pivot fronts with contribution
# rows; (13,12,11): a 156-pivot root (one chunk taking the remainder: 128 + 28); (16,16,12):
# 221-pivot root, 20 right-hand sides (two LDS passes); (130,97): 2D, every chunk single
@pytest.mark.parametrize("shape,nrhs,minp", [((20, 20, 20), 3, 1), ((20, 20, 20), 1, 200),
                                             ((16, 16, 12), 20, 1), ((130, 97), 2, 1),
                                             ((14, 11, 9), 8, 100), ((13, 12, 11), 2, 150)])
def test_chunked_solve_matches_oracle_and_block_route(shape, nrhs, minp):
    import torch
    p, plan, K, b = _plan(shape, nrhs)
    tree, conn, fac = G.oracle_factor(p)
    print(shape, nrhs, minp, flush=True)
    plan.set_chunked_solve(0)
    plan.factor(K)
    ref = [plan.solve(b, transpose=t).cpu().numpy() for t in (False, True)]
    plan.set_chunked_solve(minp)
    xs = [plan.solve(b, transpose=t).cpu().numpy() for t in (False, True)]
    for trans, x in zip((False, True), xs):
        assert G.rel_err(x, G.oracle_solve(tree, fac, p.b, trans)) <= G.TOL_SOLVE, trans
    assert G.rel_err(xs[0], ref[0]) <= 1e-12
    np.testing.assert_array_equal(xs[1], ref[1])          # transposed: the block route
    assert G.relres(p, conn, xs[0]) <= G.TOL_RELRES
    # in place (b and x alias)
    bb = b.clone()
    plan.solve(bb, out=bb)
    torch.testing.assert_close(bb, torch.from_numpy(xs[0]).to(bb.device), rtol=0, atol=0)


def test_chunked_factor_refine_and_noalloc():
    """The overlapped factor + solve (forward sweep on the plan's second stream) and the
    allocation-free solve (the chunk workspace inside the static scratch) on the chunked route."""
    import torch
    p, plan, K, b = _plan((20, 20, 20), 2)
    tree, conn, fac = G.oracle_factor(p)
    plan.set_chunked_solve(1)
    x, its, rr = plan.factor_refine(K, b, tol=1e-12, max_it=5)
    assert rr <= 1e-12
    xo = G.oracle_solve(tree, fac, p.b)
    assert G.rel_err(x.cpu().numpy(), xo) <= G.TOL_SOLVE
    out = torch.empty_like(b)
    plan.solve_noalloc(b, out)
    torch.testing.assert_close(out, plan.solve(b), rtol=0, atol=0)


def test_chunked_setting_errors():
    from paper_2306_08994_amd import MFError
    _, plan, _, _ = _plan((5, 4, 3), 1)
    with pytest.raises(MFError):
        plan.set_chunked_solve(-1)
