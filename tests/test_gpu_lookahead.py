"""GPU parity of the look-ahead panel step (32-pivot panels, one launch per step) on fronts of odd
and of even width with at least two full panels: a full panel stores its L21 rows in 16-byte
pairs, which start 8 bytes past a 16-byte boundary on every other row of an odd-width front,
and each substitution result is stored as soon as it is final.  Factors and solves against the
oracle, for both GEMM tiles of the launch (32 and 64); and a non-finite pivot inside a later
panel of the root, which every panel route (look-ahead, two-launch, fused, persistent class
launch) must report by front and pivot."""
import numpy as np
import pytest

from fixtures.mesh import reaction_diffusion
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

# panel width 32, persistent class launches and fused route off: every front wider than the
# LDS limit takes the look-ahead steps
SMAX, NB, FUSED_OFF, PERSISTENT_OFF = 24, 32, -1, -1


def _problem(shape, nrhs=3):
    return reaction_diffusion("t", shape, np.random.default_rng(3), "lognormal", 1.0, nrhs)


@pytest.mark.parametrize("shape,parity", [((96, 80), 1), ((14, 11, 9), 0)])
@pytest.mark.parametrize("tile", [32, 64])
def test_lookahead_full_panels(shape, parity, tile):
    import torch
    from paper_2306_08994_amd import Plan
    p = _problem(shape)
    tree, conn, fac = G.oracle_factor(p)
    ms, ks = np.diff(tree.front_ptr), np.asarray(tree.npiv)
    tiled = ms > SMAX
    # fronts of this width parity with two full panels and rows below them
    assert (tiled & (ks >= 2 * NB) & (ms % 2 == parity)).any()
    dev = G.torch_dev()
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(p.b)).to(dev)
    plan = Plan(p.meshes)
    plan.set_tuning(SMAX, NB, FUSED_OFF, tile, PERSISTENT_OFF)
    plan.profile(True)
    plan.factor(K)
    kinds = {k["name"] for k in plan.profile_report()["kernels"] if k["launches"] > 0}
    plan.profile(False)
    assert "panel_lookahead" in kinds and "panel_lu_trsm" not in kinds, kinds
    Ls, Us = plan.export_factors()
    assert G.factor_violation(Ls, Us, fac) <= G.TOL_FACTOR
    for trans in (False, True):
        x = plan.solve(b, transpose=trans).cpu().numpy()
        assert G.rel_err(x, G.oracle_solve(tree, fac, p.b, trans)) <= G.TOL_SOLVE, trans


# (panel width, fused-route limit, GEMM tile, persistent) of each route the root can take, and
# the kernel kind (profile report) that factors the panels on it
ROUTES = {"lookahead_t32": (32, FUSED_OFF, 32, PERSISTENT_OFF, "panel_lookahead"),
          "lookahead_t64": (32, FUSED_OFF, 64, PERSISTENT_OFF, "panel_lookahead"),
          "two_launch_nb16": (16, FUSED_OFF, 32, PERSISTENT_OFF, "panel_lu_trsm"),
          "two_launch_nb64": (64, FUSED_OFF, 32, PERSISTENT_OFF, "panel_lu_trsm"),
          "fused": (32, 128, 32, PERSISTENT_OFF, "front_panels"),
          "persistent": (32, FUSED_OFF, 32, 1, "class_tiled")}


@pytest.mark.parametrize("route", sorted(ROUTES))
def test_bad_pivot_inside_a_later_panel(route):
    """A NaN on the diagonal of a root pivot's element row reaches no pivot below the root (the
    node is a contribution-block entry there) and becomes the root's pivot 40 (the second panel
    at widths 16 and 32, inside the first at 64); each panel route reports that front and pivot,
    and the plan then factors the intact matrix."""
    import torch
    from paper_2306_08994_amd import MFError, Plan
    from paper_2306_08994_amd import _lib
    p = _problem((96, 80))
    plan = Plan(p.meshes)
    tree = plan.export_tree()
    root = int(np.where(tree["parent"] < 0)[0][0])
    assert tree["npiv"][root] > 48
    node = int(tree["front_idx"][tree["front_ptr"][root] + 40])
    conn = np.asarray(p.meshes[0].conn)
    e = int(np.where((conn == node).any(axis=1))[0][0])
    a = int(np.where(conn[e] == node)[0][0])
    dev = G.torch_dev()
    K = torch.from_numpy(p.K).to(dev)
    Kbad = K.clone()
    Kbad[e, a, a] = float("nan")
    nb, fused, tile, persistent, kind = ROUTES[route]
    plan.set_tuning(SMAX, nb, fused, tile, persistent)
    plan.profile(True)
    with pytest.raises(MFError) as ei:
        plan.factor(Kbad)
    kinds = {k["name"] for k in plan.profile_report()["kernels"] if k["launches"] > 0}
    plan.profile(False)
    assert kind in kinds, kinds
    assert ei.value.code == _lib.MF_EZERO_PIVOT
    msg = str(ei.value)
    assert f"front {root}, pivot 40 " in msg and f"node {node} " in msg, msg
    plan.factor(K)                                 # recovers
    Ls, Us = plan.export_factors()
    assert all(np.isfinite(L).all() for L in Ls)
