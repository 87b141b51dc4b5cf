"""The C++ analyser behind the C ABI against the oracle's tree: bit-exact arrays on small and
batched meshes, SHA-256 digests of the full-size workloads (written by
tests/golden/make_tree_hashes.py from the oracle), operation counts, the exported symbol set
and the host-side error paths.  Host work only: no GPU is touched."""
import ctypes
import hashlib
import json
import os
import re

import numpy as np
import pytest

from fixtures import config_problem, structured_q1, structured_qp
from oracle.tree import build_tree, front_flops

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

lib_mod = pytest.importorskip("paper_2306_08994_amd._lib")
if not os.path.exists(lib_mod.LIB_PATH):
    pytest.skip("libmf.so not built", allow_module_level=True)

from paper_2306_08994_amd import MFError, Plan  # noqa: E402

KEYS = ["parent", "level", "npiv", "front_ptr", "front_idx", "leaf_elem"]
DT = {"parent": np.int32, "level": np.int32, "npiv": np.int32, "front_ptr": np.int64,
      "front_idx": np.int32, "leaf_elem": np.int64}


def _compare(meshes):
    t = Plan(meshes).export_tree()
    o = build_tree(meshes)
    for k in KEYS:
        np.testing.assert_array_equal(t[k], getattr(o, k), err_msg=k)
    return t, o


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 5), (7, 4), (16, 16),
                                   (1, 1, 1), (2, 2, 2), (3, 2, 5), (4, 4, 4)])
def test_tree_bit_exact(shape):
    _compare([structured_q1(shape)])


@pytest.mark.parametrize("shape,p", [((3, 5), 2), ((4, 4), 3), ((7, 4), 2), ((2, 3, 2), 2),
                                     ((2, 2, 2), 3)])
def test_high_order_tree_bit_exact(shape, p):
    """Quadratic and cubic elements: interior and edge nodes change pivots and front widths."""
    _compare([structured_qp(shape, p)])


def _no_coords(mesh):
    mesh.ijk = None
    return mesh


@pytest.mark.parametrize("shape,p", [((1, 1), 1), ((3, 1), 1), ((5, 4), 1), ((7, 3), 2),
                                     ((2, 3, 2), 1), ((16, 16), 1), ((6, 5), 3)])
def test_connectivity_only_tree_bit_exact(shape, p):
    """Table 3's pairing (no element coordinates) against the oracle's."""
    _compare([_no_coords(structured_qp(shape, p))])


def test_connectivity_only_relabelled_mesh():
    """Node ids and element order scrambled: the pairing follows the lowest node ids."""
    m = structured_q1((6, 5))
    rng = np.random.default_rng(3)
    perm = rng.permutation(m.n_nodes)
    m.conn = perm[m.conn].astype(np.int32)
    m.conn = m.conn[rng.permutation(m.n_elem)]
    _compare([_no_coords(m)])


def test_connectivity_only_batch_mixed():
    a = structured_q1((4, 3))
    b = _no_coords(structured_q1((5, 2)))
    _compare([a, b])


def test_batched_tree_bit_exact():
    p = config_problem(4, n_mesh=6, side_range=(1, 9))
    _compare(p.meshes)


def test_permuted_element_order():
    """Element ids need not follow the grid: the tree depends on elem_ijk only."""
    m = structured_q1((5, 3))
    perm = np.random.default_rng(0).permutation(m.n_elem)
    m.conn = m.conn[perm]
    m.ijk = m.ijk[perm]
    _compare([m])


def _digest(t):
    h = hashlib.sha256()
    for k in KEYS:
        h.update(np.ascontiguousarray(t[k], dtype=DT[k]).tobytes())
    return h.hexdigest()


GOLD = json.load(open(os.path.join(HERE, "golden", "tree_hashes.json")))


@pytest.mark.parametrize("cfg", [1, 2, 3, 5, 4])
def test_full_size_trees_match_oracle_digest(cfg):
    key = f"cfg{cfg}"
    if key not in GOLD:
        pytest.skip(f"no golden digest for {key}")
    g = GOLD[key]
    p = config_problem(cfg)
    pl = Plan(p.meshes)
    t = pl.export_tree()
    assert _digest(t) == g["sha256"]
    inf = pl.info
    assert inf["n"] == g["n"] and inf["n_fronts"] == g["fronts"] and inf["height"] == g["height"]
    assert inf["max_m"] == g["max_m"]
    assert inf["factor_flops"] == g["factor_flops"]
    assert inf["solve_flops_per_rhs"] == g["solve_flops_per_rhs"]
    assert inf["sum_cb2"] == g["sum_cb2"]


def test_counts_match_oracle_formula():
    ms = [structured_q1((6, 5))]
    pl = Plan(ms)
    fac, sol, cb2 = front_flops(build_tree(ms))
    assert (pl.info["factor_flops"], pl.info["solve_flops_per_rhs"], pl.info["sum_cb2"]) == (fac, sol, cb2)


def test_exported_symbols_match_header():
    hdr = open(os.path.join(ROOT, "include", "mf.h")).read()
    declared = set(re.findall(r"^(?:int|void|const char)\s*\*?\s*(mf_\w+)\s*\(", hdr, re.M))
    assert declared == set(lib_mod.EXPORTED)
    lib = ctypes.CDLL(lib_mod.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _bad(meshes, msg):
    with pytest.raises(MFError) as ei:
        Plan(meshes)
    assert ei.value.code == lib_mod.MF_EINVAL
    assert msg in str(ei.value)


def test_error_paths():
    m = structured_q1((2, 2))
    bad = structured_q1((2, 2)); bad.conn = bad.conn.copy(); bad.conn[0, 0] = 99
    _bad([bad], "out of range")
    dup = structured_q1((2, 2)); dup.ijk = dup.ijk.copy(); dup.ijk[1] = dup.ijk[0]
    _bad([dup], "duplicate")
    rep = structured_q1((2, 2)); rep.conn = rep.conn.copy(); rep.conn[0, 1] = rep.conn[0, 0]
    _bad([rep], "repeated")
    unused = structured_q1((2, 2)); unused.conn = unused.conn.copy(); unused.conn[0, 0] = 1
    unused.conn[0, 1] = 2   # node 0 no longer used
    _bad([unused], "not used")
    _bad([m, structured_q1((2, 2, 2))], "same dim")
    _bad([m, structured_qp((2, 2), 2)], "same npe")
    odd = structured_qp((2, 2), 2); odd.conn = odd.conn[:, :8].copy()
    _bad([odd], "npe must be")
