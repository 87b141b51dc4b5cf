"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Sizes are chosen so the oracle finishes in seconds while the fronts still span several GEMM
tiles, several panels and ragged tails; the tiled path is forced on small meshes by lowering
the LDS threshold.  Full-size workloads are checked in test_gpu_fullsize.py."""
import numpy as np
import pytest

from fixtures import config_problem, structured_q1
from fixtures.mesh import reaction_diffusion
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _setup(problem, small_max_m=0, nb=0, fused=0, tile=0, persistent=0):
    import torch
    from paper_2306_08994_amd import Plan
    dev = G.torch_dev()
    plan = Plan(problem.meshes)
    if small_max_m or nb or fused or tile or persistent:
        plan.set_tuning(small_max_m, nb, fused, tile, persistent)
    K = torch.from_numpy(problem.K).to(dev)
    b = torch.from_numpy(problem.b).to(dev)
    return plan, K, b


def _rd(shape, seed=0, nrhs=2, sigma=1.0):
    return reaction_diffusion("t", shape, np.random.default_rng(seed), "lognormal", sigma, nrhs)


SMALL = [(1, 1), (2, 1), (4, 4), (5, 3), (16, 16), (2, 2, 2), (3, 4, 2), (5, 5, 5)]


@pytest.mark.parametrize("shape", SMALL)
def test_factor_lds_path(shape):
    p = _rd(shape)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR


# (shape, LDS limit, panel width of separate panel launches, fused-route limit (-1 = off),
#  GEMM tile (0 = default 64))
TILED = [((64, 48), 8, 16, -1, 0), ((96, 80), 24, 32, -1, 32), ((70, 53), 40, 64, -1, 0),
         ((10, 9, 8), 16, 32, -1, 32), ((12, 12, 12), 40, 16, 100, 32),
         ((14, 11, 9), 24, 64, -1, 0), ((12, 12, 12), 100, 32, 0, 0), ((64, 48), 8, 32, 0, 0),
         ((14, 11, 9), 24, 32, 0, 32), ((20, 20, 20), 0, 0, 0, 0), ((20, 20, 20), 0, 64, 0, 32)]


# every case on the route of one launch per panel step (persistent -1), and each distinct
# (shape, LDS limit, tile) on the persistent class launches (panel width 32, no fused route)
TILED_PERSISTENT = sorted({(shape, smax, tile) for shape, smax, _, _, tile in TILED})


@pytest.mark.parametrize("shape,smax,nb,fused,tile", TILED)
def test_factor_tiled_path(shape, smax, nb, fused, tile):
    p = _rd(shape, seed=1)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p, smax, nb, fused, tile, persistent=-1)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    ms = np.diff(tree.front_ptr)
    assert ms.max() > 64 and (ms > smax).sum() > 0   # several tiles on the tiled path
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR


@pytest.mark.parametrize("shape,smax,tile", TILED_PERSISTENT)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_factor_persistent_class_launch(shape, smax, tile, prec):
    """The tiled fronts of each class in one persistent launch: extend-add strips, panel
    chunks, update tiles and Schur tiles ordered by per-front counters.  FP64 entry by entry
    against the oracle; the FP32-Schur factor refines to the oracle's solution."""
    p = _rd(shape, seed=1)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p, smax, 0, 0, tile, persistent=1)
    if prec == "fp32":
        plan.factor(K, "fp32")
        x, its, rr = plan.refine(K, b, tol=1e-12, max_it=20)
        assert rr <= 1e-12
        assert G.rel_err(x.cpu().numpy(), G.oracle_solve(tree, fac, p.b)) <= 1e-9
        return
    plan.factor(K)
    Ls, Us = plan.export_factors()
    ms = np.diff(tree.front_ptr)
    assert ms.max() > 64 and (ms > smax).sum() > 0   # several tiles on the tiled path
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR


@pytest.mark.parametrize("shape,smax,nrhs,fused", [((4, 4), 0, 1, 0), ((16, 16), 0, 3, 0),
                                                   ((24, 20), 8, 8, -1), ((5, 4, 3), 0, 2, 0),
                                                   ((8, 8, 8), 40, 5, 0), ((12, 10), 0, 130, 0),
                                                   ((9, 9, 9), 0, 1, 0), ((40, 33), 0, 70, 0),
                                                   ((16, 16, 16), 0, 3, -1)])
def test_solve_parity(shape, smax, nrhs, fused):
    import torch
    p = _rd(shape, seed=2, nrhs=nrhs)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p, smax, 0, fused)
    plan.factor(K)
    for trans in (False, True):
        x = plan.solve(b, transpose=trans).cpu().numpy()
        xo = G.oracle_solve(tree, fac, p.b, trans)
        assert G.rel_err(x, xo) <= G.TOL_SOLVE, trans
    x = plan.solve(b).cpu().numpy()
    assert G.relres(p, conn, x) <= G.TOL_RELRES
    # in-place (b and x alias)
    bb = b.clone()
    plan.solve(bb, out=bb)
    torch.testing.assert_close(bb, torch.from_numpy(x).to(bb.device), rtol=0, atol=0)


@pytest.mark.parametrize("nrhs", [3, 20])
def test_solve_parity_split_rectangular_parts(nrhs):
    """A 3D mesh whose upper classes solve the rectangular parts of their fronts in launches of
    their own (c k >= 8K up, >= 16K down), with few enough slabs to take the 16-row quarter form;
    20 right-hand sides span two chunks of 16.  Solve and transposed solve against the oracle."""
    p = _rd((16, 16, 12), seed=2, nrhs=nrhs)
    tree, conn, fac = G.oracle_factor(p)
    ms = np.diff(tree.front_ptr)
    ck = (ms - tree.npiv) * tree.npiv
    assert ck.max() >= 16384 and (ck >= 8192).sum() >= 4
    plan, K, b = _setup(p)
    plan.factor(K)
    for trans in (False, True):
        x = plan.solve(b, transpose=trans).cpu().numpy()
        assert G.rel_err(x, G.oracle_solve(tree, fac, p.b, trans)) <= G.TOL_SOLVE, trans


def test_residual_and_elem_grad_kernels():
    import torch
    from oracle import adjoint as oadj
    from oracle import residual as ores
    p = _rd((7, 6), seed=3, nrhs=3)
    plan, K, b = _setup(p)
    conn = np.concatenate([m.conn for m in p.meshes]).astype(np.int64)
    x = np.random.default_rng(4).normal(size=b.shape)
    xt = torch.from_numpy(x).to(b.device)
    r = plan.residual(K, xt, b).cpu().numpy()
    np.testing.assert_allclose(r, ores.residual(p.K, conn, x, p.b), rtol=1e-13, atol=1e-13)
    lam = np.random.default_rng(5).normal(size=b.shape)
    gK = plan.elem_grad(torch.from_numpy(lam).to(b.device), xt).cpu().numpy()
    np.testing.assert_allclose(gK, oadj.elem_grad(conn, lam, x), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nrhs", [1, 2, 3, 8, 12])
def test_residual_and_refinement_norms(nrhs):
    """The residual kernel and, when nrhs divides 256, its per-block column sums of r^2 that the
    refinement's norms add up (else a separate column-norm kernel computes them): r against the
    oracle's, and the relative residual the refinement reports for a system it does not solve
    exactly (factored with K, residual with 1.01 K, so relres = 1e-2) against the oracle's
    relative residual of the returned x."""
    import torch
    from oracle import residual as ores
    p = _rd((9, 7), seed=6, nrhs=nrhs)
    plan, K, b = _setup(p)
    conn = np.concatenate([m.conn for m in p.meshes]).astype(np.int64)
    x = np.random.default_rng(7).normal(size=p.b.shape)
    r = plan.residual(K, torch.from_numpy(x).to(b.device), b).cpu().numpy()
    np.testing.assert_allclose(r, ores.residual(p.K, conn, x, p.b), rtol=1e-13, atol=1e-13)
    plan.factor(K)
    xs, its, rr = plan.refine((1.01 * K).contiguous(), b, tol=1.0, max_it=0)
    ro = ores.relres(1.01 * p.K, conn, xs.cpu().numpy(), p.b)
    assert its == 0 and ro > 1e-6
    assert abs(rr - ro) <= 1e-10 * ro, (rr, ro)


def test_batched_equals_unbatched():
    import torch
    from paper_2306_08994_amd import Plan
    p = config_problem(4, n_mesh=5, side_range=(3, 14))
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    xb = plan.solve(b).cpu().numpy()
    assert G.relres(p, conn, xb) <= G.TOL_RELRES
    # mesh by mesh
    noff, eoff, foff = p.node_offsets, p.elem_offsets, 0
    for i, mesh in enumerate(p.meshes):
        pl = Plan([mesh])
        Ki = K[eoff[i]:eoff[i + 1]].contiguous()
        pl.factor(Ki)
        Li, Ui = pl.export_factors()
        for f in range(len(Li)):
            np.testing.assert_array_equal(Li[f], Ls[foff + f])
            np.testing.assert_array_equal(Ui[f], Us[foff + f])
        foff += len(Li)
        xi = pl.solve(b[noff[i]:noff[i + 1]].contiguous()).cpu().numpy()
        np.testing.assert_array_equal(xi, xb[noff[i]:noff[i + 1]])


def test_nonsymmetric_tiled():
    p = config_problem(4, n_mesh=2, side_range=(20, 30))
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p, 24, 16)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    x = plan.solve(b).cpu().numpy()
    assert G.rel_err(x, G.oracle_solve(tree, fac, p.b)) <= G.TOL_SOLVE
    xt = plan.solve(b, transpose=True).cpu().numpy()
    assert G.rel_err(xt, G.oracle_solve(tree, fac, p.b, True)) <= G.TOL_SOLVE


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_precision_refines_to_fp64(prec):
    p = _rd((10, 9, 8), seed=6, nrhs=2)
    tree, conn, fac = G.oracle_factor(p)
    xo = G.oracle_solve(tree, fac, p.b)
    plan, K, b = _setup(p, 40, 32)
    plan.factor(K, prec)
    Ls, Us = plan.export_factors()
    err_factor = G.factor_violation(Ls, Us, fac)
    assert err_factor > 1e-14          # the Schur update really ran in reduced precision
    x, its, rr = plan.refine(K, b, tol=1e-12, max_it=40)
    assert rr <= 1e-12
    xn = x.cpu().numpy()
    assert G.relres(p, conn, xn) <= 1e-12
    assert G.rel_err(xn, xo) <= 1e-9
    print(f"{prec}: factor deviation {err_factor:.2e}, {its} corrections, relres {rr:.2e}")


@pytest.mark.parametrize("prec,nrhs", [("bf16", 3), ("bf16", 8), ("fp32", 1), ("fp64", 2)])
def test_gmres_refinement(prec, nrhs):
    """GMRES refinement (FP64, preconditioned by the stored factors) against the oracle's
    solution; nrhs 3 takes the separate column-norm path, 8 the fused one."""
    from paper_2306_08994_amd import MFError
    from paper_2306_08994_amd import _lib
    p = _rd((12, 12, 12), seed=4, nrhs=nrhs)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p, 40, 0, 0, 0, 0)
    plan.factor(K, prec)
    x, its, rr = plan.refine_gmres(K, b, tol=1e-12, max_it=60, restart=8)
    xn = x.cpu().numpy()
    assert rr <= 1e-12 and G.relres(p, conn, xn) <= 1e-12
    assert G.rel_err(xn, G.oracle_solve(tree, fac, p.b)) <= 1e-9
    if prec == "fp64":
        assert its <= 1
    with pytest.raises(MFError) as ei:
        plan.refine_gmres(K, b, restart=0)
    assert ei.value.code == _lib.MF_EINVAL
    with pytest.raises(MFError) as ei:
        plan.refine_gmres(K, b, tol=0.0, max_it=2)
    assert ei.value.code == _lib.MF_ENOCONV
    print(f"{prec} nrhs {nrhs}: {its} GMRES steps, relres {rr:.2e}")


def test_persistent_launch_wait_limit_abandons_and_recovers(monkeypatch):
    """A bound of zero on the persistent class launch's device-side waits (set from the host
    before the plan is made): the first task that has to wait gives up, every other workgroup
    leaves, the launch ends normally and the factorization reports the abort; a plan with the
    default bound then factors the same matrix."""
    from paper_2306_08994_amd import MFError
    from paper_2306_08994_amd import _lib
    p = _rd((20, 20, 20), seed=1)
    monkeypatch.setenv("MF_WAIT_LIMIT_US", "0")
    plan, K, b = _setup(p, 40, 0, 0, 0, persistent=1)
    monkeypatch.delenv("MF_WAIT_LIMIT_US")
    with pytest.raises(MFError) as ei:
        plan.factor(K)
    assert ei.value.code == _lib.MF_EHIP and "exceeded its limit" in str(ei.value)
    with pytest.raises(MFError) as ei:
        plan.solve(b)
    assert ei.value.code == _lib.MF_ESTATE
    plan2, _, _ = _setup(p, 40, 0, 0, 0, persistent=1)
    plan2.factor(K)
    x, its, rr = plan2.refine(K, b, tol=1e-12, max_it=5)
    assert rr <= 1e-12


def test_zero_pivot_message_names_mesh_and_node():
    from paper_2306_08994_amd import MFError
    from paper_2306_08994_amd import _lib
    p = config_problem(4, n_mesh=3, side_range=(2, 6))
    plan, K, b = _setup(p)
    Kbad = K.clone()
    Kbad[int(p.elem_offsets[2]), 0, 0] = 0.0     # node 0 of mesh 2: its corner, a leaf pivot
    with pytest.raises(MFError) as ei:
        plan.factor(Kbad)
    assert ei.value.code == _lib.MF_EZERO_PIVOT
    msg = str(ei.value)
    assert "mesh 2" in msg and "= node 0 of that mesh" in msg, msg
    assert f"node {int(p.node_offsets[2])} " in msg, msg
    plan.factor(K)                                 # recovers


def test_error_paths():
    import torch
    from paper_2306_08994_amd import MFError, Plan
    from paper_2306_08994_amd import _lib
    p = _rd((3, 3))
    plan, K, b = _setup(p)
    with pytest.raises(MFError) as ei:
        plan.solve(b)
    assert ei.value.code == _lib.MF_ESTATE
    Kbad = K.clone()
    Kbad[0, 0, 0] = 0.0             # the domain corner is a leaf pivot
    with pytest.raises(MFError) as ei:
        plan.factor(Kbad)
    assert ei.value.code == _lib.MF_EZERO_PIVOT
    with pytest.raises(MFError) as ei:
        plan.solve(b)
    assert ei.value.code == _lib.MF_ESTATE
    Knan = K.clone()
    Knan[4, 1, 1] = float("nan")
    with pytest.raises(MFError):
        plan.factor(Knan)
    plan.factor(K)                  # recovers
    x = plan.solve(b)
    with pytest.raises(MFError) as ei:
        plan.refine(K, b, tol=0.0, max_it=0)
    assert ei.value.code == _lib.MF_ENOCONV
    with pytest.raises(TypeError):
        plan.factor(K.cpu())
    with pytest.raises(TypeError):
        plan.factor(K.float())


def test_autotune_keeps_a_correct_schedule():
    p = _rd((20, 20, 20), seed=9, nrhs=2)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p)
    rep = plan.autotune(K, reps=1)
    assert len(rep["candidates"]) >= 2 and "chosen" in rep
    ncls = int(plan.info["height"]) + 1
    assert all(len(c["class_ms"]) == ncls for c in rep["candidates"])
    assert rep["chosen"]["mode"] in ("per_class", "global") and len(rep["chosen"]["classes"]) == ncls
    Ls, Us = plan.export_factors()              # autotune leaves the plan factored
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    x = plan.solve(b).cpu().numpy()
    assert G.rel_err(x, G.oracle_solve(tree, fac, p.b)) <= G.TOL_SOLVE


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_per_class_schedule(prec):
    """Every class on a schedule of its own: LDS limits, panel widths, fused route, GEMM tiles
    and the persistent launch alternate from class to class.  FP64 entry by entry against the
    oracle; FP32-Schur refined to the oracle's solution."""
    from paper_2306_08994_amd import MFError
    p = _rd((12, 12, 12), seed=2)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p)
    ncls = int(plan.info["height"]) + 1
    menu = [dict(small_max_m=40, nb=16, fused_max_m=0, tile=32, persistent=0),
            dict(small_max_m=128, nb=64, fused_max_m=0, tile=64, persistent=0),
            dict(small_max_m=24, nb=32, fused_max_m=0, tile=64, persistent=1),
            dict(small_max_m=64, nb=32, fused_max_m=576, tile=32, persistent=0)]
    classes = [menu[l % len(menu)] for l in range(ncls)]
    plan.set_class_tuning(classes)
    ms = np.diff(tree.front_ptr)
    assert ms.max() > 128
    if prec == "fp32":
        plan.factor(K, "fp32")
        x, its, rr = plan.refine(K, b, tol=1e-12, max_it=20)
        assert rr <= 1e-12
        assert G.rel_err(x.cpu().numpy(), G.oracle_solve(tree, fac, p.b)) <= 1e-9
    else:
        plan.factor(K)
        Ls, Us = plan.export_factors()
        assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
        x = plan.solve(b).cpu().numpy()
        assert G.rel_err(x, G.oracle_solve(tree, fac, p.b)) <= G.TOL_SOLVE
    with pytest.raises(MFError):
        plan.set_class_tuning(classes[:-1])      # one class short
    plan.set_class_tuning([])                    # back to one schedule for every class
    plan.factor(K)
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR


# Quadratic and cubic elements: larger leaves that eliminate interior unknowns, fronts built
# from edge/face nodes.  (shape, p, LDS limit, fused-route limit) -- the limits force the
# tiled routes on small meshes.
HIGH_ORDER = [((6, 5), 2, 0, 0), ((5, 4), 3, 0, 0), ((3, 3, 2), 2, 0, 0), ((2, 2, 2), 3, 0, 0),
              ((24, 20), 2, 40, -1), ((16, 13), 3, 40, 0), ((5, 5, 4), 2, 64, 0)]


@pytest.mark.parametrize("shape,deg,smax,fused", HIGH_ORDER)
def test_high_order_parity(shape, deg, smax, fused):
    from fixtures import l2_projection
    from fixtures.mesh import element_matrices, structured_qp
    p = l2_projection("t", shape, deg, np.random.default_rng(8), 3)
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p, smax, 0, fused)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    for trans in (False, True):
        x = plan.solve(b, transpose=trans).cpu().numpy()
        assert G.rel_err(x, G.oracle_solve(tree, fac, p.b, trans)) <= G.TOL_SOLVE, trans
    # diffusion with a lognormal coefficient on the same mesh
    m = structured_qp(shape, deg)
    p.K = element_matrices(m, np.exp(np.random.default_rng(9).normal(0, 1, m.n_elem)))
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p, smax, 0, fused)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    x = plan.solve(b).cpu().numpy()
    xo = G.oracle_solve(tree, fac, p.b)
    assert G.rel_err(x, xo) <= G.TOL_SOLVE
    # a direct FP64 solve of this system (cond ~4e5) leaves relres ~1.5e-12 in the oracle too:
    # hold the direct solve to the oracle's residual, and the refined one to 1e-12
    assert G.relres(p, conn, x) <= max(G.TOL_RELRES, 4 * G.relres(p, conn, xo))
    _, its, rr = plan.refine(K, b, tol=1e-12, max_it=5)
    assert rr <= G.TOL_RELRES


def test_high_order_residual_and_elem_grad():
    import torch
    from fixtures import l2_projection
    from oracle import adjoint as oadj
    from oracle import residual as ores
    p = l2_projection("t", (4, 3, 2), 3, np.random.default_rng(3), 2)
    plan, K, b = _setup(p)
    conn = p.meshes[0].conn.astype(np.int64)
    x = np.random.default_rng(4).normal(size=b.shape)
    xt = torch.from_numpy(x).to(b.device)
    r = plan.residual(K, xt, b).cpu().numpy()
    np.testing.assert_allclose(r, ores.residual(p.K, conn, x, p.b), rtol=1e-13, atol=1e-13)
    lam = np.random.default_rng(5).normal(size=b.shape)
    gK = plan.elem_grad(torch.from_numpy(lam).to(b.device), xt).cpu().numpy()
    np.testing.assert_allclose(gK, oadj.elem_grad(conn, lam, x), rtol=1e-13, atol=1e-13)


def _relabelled(shape, seed):
    m = structured_q1(shape)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m.n_nodes)
    m.conn = perm[m.conn].astype(np.int32)
    order = rng.permutation(m.n_elem)
    m.conn, m.ijk = m.conn[order], None
    return m


@pytest.mark.parametrize("case", ["2d", "3d", "relabelled", "q2"])
def test_connectivity_only_tree_parity(case):
    """Trees of Table 3 (connectivity only): uneven heights from carried fronts, fronts joining
    elements that share no node; factor and both solves against the oracle."""
    from fixtures import l2_projection
    from fixtures.mesh import element_matrices, structured_qp
    rng = np.random.default_rng(11)
    if case == "2d":
        m = structured_q1((37, 23))
    elif case == "3d":
        m = structured_q1((9, 7, 6))
    elif case == "q2":
        m = structured_qp((13, 11), 2)
    else:
        m = _relabelled((30, 25), 5)
    m.ijk = None
    coef = np.exp(rng.normal(0, 1, m.n_elem))
    p = reaction_diffusion("t", (1, 1), rng, "lognormal", 1.0, 2)
    p.meshes = [m]
    p.K = element_matrices(m, coef)
    p.coef = coef
    p.b = rng.normal(size=(m.n_nodes, 3))
    tree, conn, fac = G.oracle_factor(p)
    plan, K, b = _setup(p)
    plan.factor(K)
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    for trans in (False, True):
        x = plan.solve(b, transpose=trans).cpu().numpy()
        assert G.rel_err(x, G.oracle_solve(tree, fac, p.b, trans)) <= G.TOL_SOLVE, trans
