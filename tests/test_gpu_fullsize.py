"""GPU checks at the full workload sizes, in the launch configuration the benchmark times
(default tuning, hipGraph replay).  The oracle cannot factor these in test time as a whole, so
the checks are (a) fronts sampled from the lower classes, whose subtrees the oracle factors
front by front, compared entry by entry; (b) properties that hold at any size: relative residual
<= 1e-12 after FP64 refinement, agreement with the FP64 path for the mixed-precision variants,
and the batch equal to its meshes solved one by one; (c) graph replays identical to eager runs.
"""
import numpy as np
import pytest

from fixtures import config_problem
from oracle import factor as ofac
from oracle.tree import build_tree
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _subtree_oracle(tree, p, conn, roots):
    """Oracle factors of the fronts in the subtrees of `roots` (post-order ids: the subtree of
    f is the contiguous id range ending at f)."""
    sizes = {}
    L, U = {}, {}
    cbs = {}
    todo = set()
    for r in roots:
        stack = [r]
        while stack:
            f = stack.pop()
            todo.add(f)
            if tree.left[f] >= 0:
                stack += [int(tree.left[f]), int(tree.right[f])]
    for f in sorted(todo):                     # children have smaller ids
        Fm = ofac.assemble_front(tree, f, p.K, conn, cbs)
        k = int(tree.npiv[f])
        L[f], U[f] = ofac.eliminate(Fm, k, f)
        cbs[f] = Fm[k:, k:].copy()
    return L, U


@pytest.mark.parametrize("cfg,levels", [(2, (6, 9)), (3, (5, 7)), (5, (8, 10))])
def test_sampled_fronts_match_oracle(cfg, levels):
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(cfg)
    tree = build_tree(p.meshes)
    conn = ofac.global_connectivity(p)
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    rng = np.random.default_rng(cfg)
    roots = []
    for l in levels:
        cand = np.flatnonzero(tree.level == l)
        roots += [int(f) for f in rng.choice(cand, size=min(3, len(cand)), replace=False)]
    L, U = _subtree_oracle(tree, p, conn, roots)
    worst = 0.0
    for f in L:
        worst = max(worst, G.front_violation(Ls[f], L[f]), G.front_violation(Us[f], U[f]))
    assert worst <= G.TOL_FACTOR, worst


@pytest.mark.parametrize("cfg", [2, 5])
def test_full_size_residual(cfg):
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(cfg)
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    plan.factor(K)
    x0 = plan.solve(b)
    x, its, rr = plan.refine(K, b, tol=1e-12, max_it=5)
    assert rr <= 1e-12
    conn = ofac.global_connectivity(p)
    assert G.relres(p, conn, x.cpu().numpy()) <= 1e-12
    print(f"cfg{cfg}: direct relres {G.relres(p, conn, x0.cpu().numpy()):.2e}, "
          f"{its} corrections -> {rr:.2e}")


def test_mixed_precision_3d_full_size():
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(3)
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    conn = ofac.global_connectivity(p)
    plan.factor(K)
    x64, _, rr64 = plan.refine(K, b, tol=1e-12, max_it=5)
    x64 = x64.clone()
    for prec, max_it in (("fp32", 20), ("bf16", 80)):
        plan.factor(K, prec)
        x, its, rr = plan.refine(K, b, tol=1e-12, max_it=max_it)
        assert rr <= 1e-12
        assert G.relres(p, conn, x.cpu().numpy()) <= 1e-12
        err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        assert err <= 1e-9
        print(f"{prec}: {its} corrections, relres {rr:.2e}, error vs FP64 {err:.2e}")


def test_batched_full_size_equals_per_mesh():
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(4)
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    plan.factor(K)
    x, its, rr = plan.refine(K, b, tol=1e-12, max_it=5)
    assert rr <= 1e-12
    xb = plan.solve(b).cpu().numpy()
    noff, eoff = p.node_offsets, p.elem_offsets
    for i in np.random.default_rng(4).choice(len(p.meshes), 6, replace=False):
        pl = Plan([p.meshes[i]])
        pl.factor(K[eoff[i]:eoff[i + 1]].contiguous())
        xi = pl.solve(b[noff[i]:noff[i + 1]].contiguous()).cpu().numpy()
        # a lone mesh may take other kernel routes (class widths differ from the batch's), so
        # the two agree to rounding, not bit for bit
        ref = xb[noff[i]:noff[i + 1]]
        assert G.rel_err(xi, ref) <= 1e-12


def test_graph_replay_matches_eager():
    """Captured launch sequences replayed several times, with eager work in between, give the
    same bits as eager launches (profiling mode runs eagerly)."""
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(2, shape=(64, 48), nrhs=3)
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    x = torch.empty_like(b)
    for rep in range(3):
        Kr = K * (1.0 + 0.25 * rep)
        plan.profile(True)                      # eager
        plan.factor(Kr)
        Le, Ue = plan.export_factors()
        xe = plan.solve(b).clone()
        xte = plan.solve(b, transpose=True).clone()
        plan.profile(False)
        K.copy_(Kr)                             # same pointer, new contents
        plan.factor(K)                          # graph replay (captured on first use)
        Lg, Ug = plan.export_factors()
        for f in range(len(Le)):
            np.testing.assert_array_equal(Le[f], Lg[f])
            np.testing.assert_array_equal(Ue[f], Ug[f])
        plan.solve(b, out=x)
        torch.testing.assert_close(x, xe, rtol=0, atol=0)
        torch.testing.assert_close(plan.solve(b, transpose=True), xte, rtol=0, atol=0)
        K.copy_(torch.from_numpy(p.K).to(dev))


def test_profile_report():
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(2, shape=(64, 64), nrhs=2)
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    plan.profile(True)
    plan.factor(K)
    plan.solve(b)
    rep = plan.profile_report()
    plan.profile(False)
    names = {k["name"] for k in rep["kernels"]}
    assert {"factor_tiny", "solve_down_wave", "solve_up_wave"} <= names
    fl = sum(k["flops"] for k in rep["kernels"] if k["name"].startswith(("factor", "gemm", "panel")))
    # factor tasks (blocked accounting on the tiled path) plus extend-add additions
    assert 0.95 * plan.info["factor_flops"] <= fl <= 1.5 * plan.info["factor_flops"]
    for k in rep["kernels"]:
        assert k["ms"] > 0 and k["launches"] > 0


def test_connectivity_only_tree_full_size():
    """The 256 x 256 model problem on the Table 3 tree (no element coordinates).  Its class of
    height 9 holds 126 fronts of width 771 whose panel steps launch more workgroups than the
    chip holds at once, so workgroups of one front run one after another: every front of the
    classes up to height 12 (all of their subtrees) against the oracle, then the residual."""
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = config_problem(2)
    for m in p.meshes:
        m.ijk = None
    tree = build_tree(p.meshes)
    conn = ofac.global_connectivity(p)
    plan = Plan(p.meshes)
    plan.set_tuning(64, 32, -1, 32)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    L, U = _subtree_oracle(tree, p, conn, [int(f) for f in np.flatnonzero(tree.level == 12)])
    worst = max(max(G.front_violation(Ls[f], L[f]), G.front_violation(Us[f], U[f])) for f in L)
    assert worst <= G.TOL_FACTOR, worst
    x0 = plan.solve(b)
    rr0 = G.relres(p, conn, x0.cpu().numpy())
    assert rr0 <= 1e-10, rr0
    x, its, rr = plan.refine(K, b, tol=1e-12, max_it=5)
    assert rr <= 1e-12
    print(f"Table 3 tree 256x256: {len(L)} fronts {worst:.1e}, direct relres {rr0:.2e}")


@pytest.mark.parametrize("deg", [1, 2, 3])
def test_l2_projection_full_size(deg):
    """The paper's benchmark axis at its largest size (Sec. 5): L2 projection with linear,
    quadratic and cubic bases at 299,209 unknowns.  Sampled fronts against the oracle, then the
    relative residual of the direct solve and after FP64 refinement, and the reproduction of a
    function of the space (f of degree <= p per axis is its own projection)."""
    import torch
    from fixtures import l2_projection, l2_workload, node_coords, L2_SHAPES
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    p = l2_workload(deg)
    tree = build_tree(p.meshes)
    conn = ofac.global_connectivity(p)
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    rng = np.random.default_rng(deg)
    roots = []
    for l in (5, 7):
        cand = np.flatnonzero(tree.level == l)
        roots += [int(f) for f in rng.choice(cand, size=min(3, len(cand)), replace=False)]
    L, U = _subtree_oracle(tree, p, conn, roots)
    worst = max(max(G.front_violation(Ls[f], L[f]), G.front_violation(Us[f], U[f])) for f in L)
    assert worst <= G.TOL_FACTOR, worst
    x0 = plan.solve(b)
    rr0 = G.relres(p, conn, x0.cpu().numpy())
    x, its, rr = plan.refine(K, b, tol=1e-12, max_it=5)
    assert rr <= 1e-12 and G.relres(p, conn, x.cpu().numpy()) <= 1e-12

    def f(xy):
        return np.prod(1.0 + xy + 0.5 * xy ** deg, axis=1)
    pf = l2_projection("f", L2_SHAPES[deg], deg, None, 1, f=f)
    u = plan.solve(torch.from_numpy(pf.b).to(dev)).cpu().numpy()[:, 0]
    exact = f(node_coords(pf.meshes[0]))
    err = np.abs(u - exact).max() / np.abs(exact).max()
    assert err <= 1e-10, err
    print(f"L2 projection p={deg}: sampled fronts {worst:.1e}, direct relres {rr0:.2e}, "
          f"{its} corrections -> {rr:.2e}, reproduction error {err:.1e}")
