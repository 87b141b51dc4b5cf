"""Every front of the full-size workloads against the oracle, in the schedules the benchmark
times, and the solutions of the mixed-precision and batched variants against the oracle's.

The oracle factors the whole 256 x 256 workload in a few seconds and the 3D 32^3 one in under a
minute on one host core, so the comparison is entry by entry over all fronts (reading 18's
tolerance per front), not sampled.  Mixed-precision factors are approximations refined in FP64;
their solutions after refinement to relres <= 1e-12 are compared with the oracle's solution
(O-6: ||x - x_O||_2 / ||x_O||_2 per right-hand side).
"""
import functools

import numpy as np
import pytest

from fixtures import config_problem
from fixtures.mesh import Problem
from oracle import factor as ofac
from oracle import solve as osol
from oracle.tree import build_tree
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

TOL_MIXED_VS_ORACLE = 1e-9     # refined mixed-precision solution against the oracle's


@functools.lru_cache(maxsize=None)
def _oracle(cfg):
    """(problem, tree, connectivity, oracle factors, oracle solution) of a workload."""
    p = config_problem(cfg)
    tree = build_tree(p.meshes)
    conn = ofac.global_connectivity(p)
    fac = ofac.factor(tree, p.K, conn)
    x = osol.solve(tree, fac, p.b)
    return p, tree, conn, fac, x


def _setup(p):
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    plan = Plan(p.meshes)
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    return plan, K, b


def _per_class_violation(Ls, Us, fac, tree):
    worst = np.zeros(int(tree.level.max()) + 1)
    for f in range(len(fac.L)):
        v = max(G.front_violation(Ls[f], fac.L[f]), G.front_violation(Us[f], fac.U[f]))
        lv = int(tree.level[f])
        worst[lv] = max(worst[lv], v)
    return worst


@pytest.mark.parametrize("schedule", ["autotuned", "32,0,32,64"])
def test_256x256_every_front_matches_oracle(schedule):
    """The benchmark's workload and call (factor_refine): all 131,071 fronts, and the solution."""
    p, tree, conn, fac, xo = _oracle(2)
    plan, K, b = _setup(p)
    if schedule == "autotuned":
        chosen = plan.autotune(K, reps=3)["chosen"]
    else:
        t, fu, nb, sm = (int(v) for v in schedule.split(","))
        plan.set_tuning(sm, nb, fu if fu > 0 else -1, t)
        chosen = schedule
    x, its, rr = plan.factor_refine(K, b, tol=1e-12, max_it=5)
    Ls, Us = plan.export_factors()
    worst = _per_class_violation(Ls, Us, fac, tree)
    assert worst.max() <= G.TOL_FACTOR, (chosen, worst)
    err = G.rel_err(x.cpu().numpy(), xo)
    assert rr <= 1e-12 and err <= G.TOL_SOLVE, (rr, err)
    print(f"256x256 [{chosen}]: worst per class {np.array2string(worst, precision=1)}, "
          f"solution error {err:.2e}, {its} corrections, relres {rr:.2e}")


def test_128x128_64rhs_every_front_matches_oracle():
    p, tree, conn, fac, xo = _oracle(5)
    plan, K, b = _setup(p)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    worst = _per_class_violation(Ls, Us, fac, tree)
    assert worst.max() <= G.TOL_FACTOR, worst
    x = plan.solve(b).cpu().numpy()
    assert G.rel_err(x, xo) <= G.TOL_SOLVE
    xt = plan.solve(b, transpose=True).cpu().numpy()
    assert G.rel_err(xt, osol.solve_t(tree, fac, p.b)) <= G.TOL_SOLVE


def test_3d_fp64_every_front_matches_oracle():
    """3D 32^3: fronts up to 1617 wide (classes 8-15 on the tiled route), autotuned schedule."""
    p, tree, conn, fac, xo = _oracle(3)
    plan, K, b = _setup(p)
    chosen = plan.autotune(K, "fp64", reps=2)["chosen"]
    x, its, rr = plan.factor_refine(K, b, "fp64", tol=1e-12, max_it=5)
    Ls, Us = plan.export_factors()
    worst = _per_class_violation(Ls, Us, fac, tree)
    assert worst.max() <= G.TOL_FACTOR, (chosen, worst)
    err = G.rel_err(x.cpu().numpy(), xo)
    assert rr <= 1e-12 and err <= G.TOL_SOLVE, (rr, err)
    print(f"3D fp64 [{chosen}]: worst per class {np.array2string(worst, precision=1)}, "
          f"solution error {err:.2e}")


@pytest.mark.parametrize("prec,max_it", [("fp32", 20), ("bf16", 80)])
def test_3d_mixed_solution_matches_oracle(prec, max_it):
    p, tree, conn, fac, xo = _oracle(3)
    plan, K, b = _setup(p)
    plan.autotune(K, prec, reps=2)
    x, its, rr = plan.factor_refine(K, b, prec, tol=1e-12, max_it=max_it)
    xn = x.cpu().numpy()
    err = G.rel_err(xn, xo)
    assert rr <= 1e-12 and G.relres(p, conn, xn) <= 1e-12
    assert err <= TOL_MIXED_VS_ORACLE, err
    print(f"3D {prec}: {its} corrections, relres {rr:.2e}, error vs oracle {err:.2e}")


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_3d_mixed_gmres_matches_oracle(prec):
    """GMRES refinement preconditioned by the narrow-Schur factors reaches relres <= 1e-12 and
    the oracle's solution, in fewer preconditioned steps than plain refinement needs."""
    p, tree, conn, fac, xo = _oracle(3)
    plan, K, b = _setup(p)
    plan.factor(K, prec)
    _, its_ir, _ = plan.refine(K, b, tol=1e-12, max_it=80)
    x, its, rr = plan.refine_gmres(K, b, tol=1e-12, max_it=60, restart=20)
    xn = x.cpu().numpy()
    err = G.rel_err(xn, xo)
    assert rr <= 1e-12 and G.relres(p, conn, xn) <= 1e-12
    assert err <= TOL_MIXED_VS_ORACLE, err
    assert its <= its_ir
    print(f"3D {prec} GMRES: {its} steps (refinement: {its_ir}), relres {rr:.2e}, error {err:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_solution_matches_oracle(prec):
    """The 256-mesh batch: sampled meshes solved by the oracle one by one against the batch's
    solution (FP64, and FP32-Schur refined in FP64)."""
    p = config_problem(4)
    plan, K, b = _setup(p)
    plan.autotune(K, prec, reps=2)
    x, its, rr = plan.factor_refine(K, b, prec, tol=1e-12, max_it=30)
    assert rr <= 1e-12
    xb = x.cpu().numpy()
    noff, eoff = p.node_offsets, p.elem_offsets
    tol = G.TOL_SOLVE if prec == "fp64" else TOL_MIXED_VS_ORACLE
    worst = 0.0
    for i in np.random.default_rng(40).choice(len(p.meshes), 8, replace=False):
        sub = Problem(p.name, [p.meshes[i]], p.K[eoff[i]:eoff[i + 1]], p.b[noff[i]:noff[i + 1]],
                      p.coef[eoff[i]:eoff[i + 1]], [p.S[i]], [p.M[i]])
        tree = build_tree(sub.meshes)
        conn = ofac.global_connectivity(sub)
        xo = osol.solve(tree, ofac.factor(tree, sub.K, conn), sub.b)
        worst = max(worst, G.rel_err(xb[noff[i]:noff[i + 1]], xo))
    assert worst <= tol, worst
    print(f"batch {prec}: {its} corrections, relres {rr:.2e}, sampled error vs oracle {worst:.2e}")
