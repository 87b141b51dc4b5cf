"""GPU parity of the bottom-subtree launches: the leading Foata classes of the tiny factor route
and of the wave solves as one launch each (one workgroup per unit: a front whose parent lies
above the fused classes, with its descendants; a workgroup barrier between classes).

Forced on meshes the oracle handles in seconds (min_units=1), they are checked against the
oracle (factors entry by entry, solve and transposed solve) and against the per-class launches
of the same plan, which must give bit-identical factors and solutions (same fronts, same
arithmetic, only the launch structure differs).  Irregular trees: a batch of meshes of
different sizes (units rooted in different classes), the connectivity-only tree of a relabelled
mesh (carried fronts, uneven heights), Q2 elements."""
import numpy as np
import pytest

from fixtures import config_problem, structured_q1
from fixtures.mesh import element_matrices, reaction_diffusion, structured_qp
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _problem(case, nrhs):
    rng = np.random.default_rng(21)
    if case.startswith("rd"):
        shape = {"rd2d": (40, 33), "rd2d_sq": (64, 64), "rd3d": (9, 9, 9),
                 "rd3d_ragged": (11, 7, 5)}[case]
        return reaction_diffusion("t", shape, rng, "lognormal", 1.0, nrhs)
    if case == "batch":
        p = config_problem(4, n_mesh=6, side_range=(3, 24))
        p.b = rng.normal(size=(p.b.shape[0], nrhs))
        return p
    if case == "relabelled":
        m = structured_q1((30, 25))
        perm = rng.permutation(m.n_nodes)
        m.conn = perm[m.conn].astype(np.int32)
        m.conn = m.conn[rng.permutation(m.n_elem)]
        m.ijk = None
    else:   # q2
        m = structured_qp((13, 11), 2)
    coef = np.exp(rng.normal(0, 1, m.n_elem))
    p = reaction_diffusion("t", (1, 1), rng, "lognormal", 1.0, nrhs)
    p.meshes = [m]
    p.K = element_matrices(m, coef)
    p.coef = coef
    p.b = rng.normal(size=(m.n_nodes, nrhs))
    return p


def _run(plan, K, b):
    plan.factor(K)
    Ls, Us = plan.export_factors()
    xs = [plan.solve(b, transpose=t).cpu().numpy() for t in (False, True)]
    return Ls, Us, xs


@pytest.mark.parametrize("case,nrhs", [("rd2d", 3), ("rd2d_sq", 1), ("rd3d", 2),
                                       ("rd3d_ragged", 20), ("batch", 2), ("relabelled", 3),
                                       ("q2", 2)])
def test_subtree_launch_matches_oracle_and_per_class(case, nrhs):
    import torch
    from paper_2306_08994_amd import Plan
    p = _problem(case, nrhs)
    tree, conn, fac = G.oracle_factor(p)
    dev = G.torch_dev()
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(p.b)).to(dev)
    plan = Plan(p.meshes)
    plan.set_subtree_launch(-1, 1)
    info = plan.subtree_launch_info()
    print(case, info, flush=True)
    assert info["factor_classes"] >= 2 and info["solve_classes"] >= 2, info
    Ls, Us, xs = _run(plan, K, b)
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    for trans, x in zip((False, True), xs):
        assert G.rel_err(x, G.oracle_solve(tree, fac, p.b, trans)) <= G.TOL_SOLVE, trans
    # the per-class launches of the same plan: bit-identical
    plan.set_subtree_launch(0, 1)
    assert plan.subtree_launch_info()["factor_classes"] == 0
    L0, U0, x0 = _run(plan, K, b)
    for f in range(len(L0)):
        np.testing.assert_array_equal(Ls[f], L0[f])
        np.testing.assert_array_equal(Us[f], U0[f])
    for a, c in zip(xs, x0):
        np.testing.assert_array_equal(a, c)


def test_subtree_class_limits_agree():
    """Every number of fused classes (2, 3, as many as the routes allow) gives the same bits."""
    import torch
    from paper_2306_08994_amd import Plan
    p = _problem("rd2d", 4)
    dev = G.torch_dev()
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    plan = Plan(p.meshes)
    ref = None
    seen = set()
    for mc in (2, 3, -1):
        plan.set_subtree_launch(mc, 1)
        info = plan.subtree_launch_info()
        seen.add((info["factor_classes"], info["solve_classes"]))
        if mc > 0:
            assert info["factor_classes"] == mc and info["solve_classes"] == mc, info
        out = _run(plan, K, b)
        if ref is None:
            ref = out
            continue
        for f in range(len(ref[0])):
            np.testing.assert_array_equal(out[0][f], ref[0][f])
            np.testing.assert_array_equal(out[1][f], ref[1][f])
        for a, c in zip(out[2], ref[2]):
            np.testing.assert_array_equal(a, c)
    assert len(seen) == 3


def test_subtree_default_threshold_and_errors():
    """Off by default; on, below the default unit threshold a small mesh keeps per-class
    launches; bad settings are rejected."""
    from paper_2306_08994_amd import MFError, Plan
    G.torch_dev()
    p = _problem("rd2d", 1)
    plan = Plan(p.meshes)
    info = plan.subtree_launch_info()
    assert info["factor_classes"] == 0 and info["solve_classes"] == 0, info
    plan.set_subtree_launch(-1)
    info = plan.subtree_launch_info()
    assert info["factor_classes"] == 0 and info["solve_classes"] == 0, info
    with pytest.raises(MFError):
        plan.set_subtree_launch(-2, 1)
    with pytest.raises(MFError):
        plan.set_subtree_launch(-1, 0)
