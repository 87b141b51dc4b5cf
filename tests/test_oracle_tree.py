"""Pins for the oracle's elimination tree, Foata levels and front structure.

Each property is checked against a construction other than the oracle's own:
  * counts in closed form (F = 2E - 1, height, root separator, every node a pivot once);
  * the paper's bottom-up tree generation (sort fronts, join adjacent pairs, carry an odd one;
    Table 3) applied to the Morton-ordered element list, which on 2^a grids must give exactly
    the nested-dissection tree;
  * pivot and contribution-block sets by brute-force set containment over element sets;
  * interior-box front sizes in closed form (perimeter nodes + separator);
  * Foata classes by peeling minimal fronts, and a planted mistake that the check must catch.
"""
import numpy as np
import pytest

from fixtures import structured_q1
from oracle import foata
from oracle.tree import build_tree, front_flops


def _tree(shape):
    m = structured_q1(shape)
    return m, build_tree([m])


def _elem_sets(tree):
    sets = [None] * tree.n_fronts
    for f in range(tree.n_fronts):
        if tree.leaf_elem[f] >= 0:
            sets[f] = frozenset([int(tree.leaf_elem[f])])
        else:
            sets[f] = sets[tree.left[f]] | sets[tree.right[f]]
    return sets


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 2), (3, 5), (4, 4), (7, 3), (16, 16),
                                   (2, 2, 2), (3, 2, 4), (4, 4, 4)])
def test_counts(shape):
    mesh, t = _tree(shape)
    E = mesh.n_elem
    assert t.n_fronts == 2 * E - 1
    assert t.n == mesh.n_nodes
    assert int(t.npiv.sum()) == mesh.n_nodes
    piv = np.concatenate([t.pivots(f) for f in range(t.n_fronts)])
    assert np.array_equal(np.sort(piv), np.arange(mesh.n_nodes))
    assert (t.parent == -1).sum() == 1 and t.parent[-1] == -1
    assert t.m(t.n_fronts - 1) == t.npiv[-1]          # root: no contribution block


@pytest.mark.parametrize("a,dim", [(1, 2), (2, 2), (3, 2), (4, 2), (1, 3), (2, 3)])
def test_height_and_root_separator(a, dim):
    s = 1 << a
    mesh, t = _tree((s,) * dim)
    assert t.height == dim * a
    # root splits x at s/2: the separator is the plane x = s/2, (s+1)^(dim-1) nodes
    assert int(t.npiv[-1]) == (s + 1) ** (dim - 1)
    root_piv = t.pivots(t.n_fronts - 1)
    assert np.all(root_piv % (s + 1) == s // 2)


def _morton(ijk, a):
    dim = ijk.shape[1]
    code = np.zeros(ijk.shape[0], dtype=np.int64)
    for bit in range(a):
        for d in range(dim):
            # lowest significance: last axis; highest: x  (x splits first at the top)
            code |= ((ijk[:, d] >> bit) & 1).astype(np.int64) << (dim * bit + (dim - 1 - d))
    return code


def _table3_tree(order):
    fronts = [frozenset([int(e)]) for e in order]
    levels = [list(fronts)]
    while len(fronts) > 1:
        new = [fronts[i] | fronts[i + 1] for i in range(0, len(fronts) - 1, 2)]
        if len(fronts) % 2 == 1:
            new.append(fronts[-1])
        fronts = new
        levels.append(list(fronts))
    return levels


@pytest.mark.parametrize("a,dim", [(1, 2), (2, 2), (3, 2), (4, 2), (1, 3), (2, 3)])
def test_nested_dissection_equals_table3_pairing_in_morton_order(a, dim):
    mesh, t = _tree((1 << a,) * dim)
    order = np.argsort(_morton(mesh.ijk, a), kind="stable")
    levels = _table3_tree(order)
    sets = _elem_sets(t)
    for l, fronts in enumerate(levels):
        got = sorted(sorted(sets[f]) for f in np.flatnonzero(t.level == l))
        assert got == sorted(sorted(s) for s in fronts), f"class {l} differs"


@pytest.mark.parametrize("shape", [(4, 4), (5, 3), (2, 7), (3, 2, 2), (2, 3, 3)])
def test_pivots_and_cb_by_set_containment(shape):
    mesh, t = _tree(shape)
    sets = _elem_sets(t)
    elems_of = [set() for _ in range(mesh.n_nodes)]
    for e, row in enumerate(mesh.conn):
        for v in row:
            elems_of[int(v)].add(e)
    for f in range(t.n_fronts):
        S = sets[f]
        nodes = set(int(v) for e in S for v in mesh.conn[e])
        inside = {v for v in nodes if elems_of[v] <= S}
        if t.leaf_elem[f] >= 0:
            piv = inside
        else:
            piv = {v for v in inside if not elems_of[v] <= sets[t.left[f]]
                   and not elems_of[v] <= sets[t.right[f]]}
        cb = nodes - inside
        assert list(t.pivots(f)) == sorted(piv)
        assert list(t.cb(f)) == sorted(cb)


def test_interior_box_sizes_closed_form():
    s = 64
    mesh, t = _tree((s, s))
    sets = _elem_sets(t)
    checked = 0
    for f in range(t.n_fronts):
        if t.leaf_elem[f] >= 0:
            continue
        ij = mesh.ijk[sorted(sets[f])]
        lo, hi = ij.min(0), ij.max(0) + 1
        if lo.min() == 0 or hi.max() == s:
            continue                                    # touches the domain boundary
        sx, sy = hi - lo
        split_x = sx >= sy
        assert t.m(f) - t.npiv[f] == 2 * (sx + sy)      # box perimeter nodes
        assert t.npiv[f] == (sy - 1 if split_x else sx - 1)   # separator minus its two ends
        checked += 1
    assert checked > 1000


def test_2d_level_widths_256():
    """Widest front per class of the 256x256 mesh: interior boxes give 2(sx+sy) + separator up
    to class 12; classes 13-16 are boxes touching the boundary, counted by hand from geometry."""
    s = 256
    mesh, t = _tree((s, s))
    ms = np.diff(t.front_ptr)
    widths = [int(ms[t.level == l].max()) for l in range(t.height + 1)]
    interior = []
    sx = sy = 1
    for l in range(13):
        if l == 0:
            interior.append(4)
            continue
        # going up, a square box doubles in y, a 1:2 box doubles in x
        if sx == sy:
            sy *= 2
            interior.append(2 * (sx + sy) + sx - 1)
        else:
            sx *= 2
            interior.append(2 * (sx + sy) + sy - 1)
    assert widths[:13] == interior
    # class 13: 64x128 boxes next to the left/right sides share 3 sides with the interior
    # (2*64 + 128 + 1 CB nodes) and a 63-node separator plus its end on the domain side
    # class 14: 128x128 quarter boxes: CB 2*128+1, separator 129 minus the end on the centre
    # class 15: 128x256 halves: CB = 257 nodes of the centre line, separator 128 nodes
    # class 16: the root, separator 257, no CB
    assert widths[13:] == [384, 385, 385, 257]
    assert int(t.npiv[-1]) == 257


@pytest.mark.parametrize("shape", [(16, 16), (5, 9), (3, 3, 3), (2, 5, 3)])
def test_foata_levels(shape):
    _, t = _tree(shape)
    assert foata.check(t, t.level) == []
    np.testing.assert_array_equal(foata.fnf_classes(t), t.level)


def test_foata_check_catches_planted_mistake():
    _, t = _tree((4, 4))
    bad = t.level.copy()
    leaf = int(np.flatnonzero(t.leaf_elem >= 0)[0])
    bad[leaf] = 1                       # a leaf moved to class 1: not the Foata normal form
    assert foata.check(t, bad) != []
    bad2 = t.level.copy()
    bad2[-1] = bad2[-2]                 # the root placed in its child's class
    errs = foata.check(t, bad2)
    assert any("ancestor" in e for e in errs)


def test_batched_tree_is_union_of_meshes():
    ms = [structured_q1((3, 4)), structured_q1((5, 2))]
    tb = build_tree(ms)
    t0, t1 = build_tree([ms[0]]), build_tree([ms[1]])
    F0 = t0.n_fronts
    assert tb.n_fronts == F0 + t1.n_fronts
    np.testing.assert_array_equal(tb.level[:F0], t0.level)
    np.testing.assert_array_equal(tb.level[F0:], t1.level)
    np.testing.assert_array_equal(tb.parent[F0:], np.where(t1.parent >= 0, t1.parent + F0, -1))
    np.testing.assert_array_equal(tb.front_idx[t0.front_ptr[-1]:], t1.front_idx + ms[0].n_nodes)


def test_flop_counts_config1():
    _, t = _tree((16, 16))
    fac, sol, cb2 = front_flops(t)
    # the division tasks alone: one per entry right of each pivot
    div = sum(t.m(f) - p - 1 for f in range(t.n_fronts) for p in range(int(t.npiv[f])))
    mul = sum((t.m(f) - p - 1) ** 2 for f in range(t.n_fronts) for p in range(int(t.npiv[f])))
    assert fac == div + 2 * mul
    assert (fac, sol, cb2) == (106228, 14225, 22618)


# ---- Table 3 (connectivity only): sort by lowest node id, join adjacent pairs, carry odd ----

def _pairing_tree(shape):
    m = structured_q1(shape)
    m.ijk = None
    return m, build_tree([m])


def test_pairing_strip_of_power_of_two_is_bisection():
    """On a 1 x 2^a strip the lowest-node order is the element order, so pairing adjacent fronts
    round by round is exactly halving: the bisection tree."""
    for a in (1, 2, 3, 4):
        m = structured_q1((1 << a, 1))
        t_bis = build_tree([m])
        m2, t_pair = _pairing_tree((1 << a, 1))
        np.testing.assert_array_equal(t_bis.parent, t_pair.parent)
        np.testing.assert_array_equal(t_bis.leaf_elem, t_pair.leaf_elem)
        np.testing.assert_array_equal(t_bis.front_idx, t_pair.front_idx)


def test_pairing_carries_the_odd_front():
    """Five elements in a row: rounds [01][23] 4 -> [0123] 4 -> [[0123] 4].  Post-order ids:
    e0 0, e1 1, (01) 2, e2 3, e3 4, (23) 5, (0123) 6, e4 7, root 8."""
    m, t = _pairing_tree((5, 1))
    np.testing.assert_array_equal(t.parent, [2, 2, 6, 5, 5, 6, 8, 8, -1])
    np.testing.assert_array_equal(t.leaf_elem, [0, 1, -1, 2, 3, -1, -1, 4, -1])
    np.testing.assert_array_equal(t.level, [0, 0, 1, 0, 0, 1, 2, 0, 3])
    # the carried element's own nodes (its far edge) are eliminated at the root only if shared:
    # node 5 (bottom right corner of e4) belongs to e4 alone -> pivot of its leaf
    assert 5 in t.pivots(7)


@pytest.mark.parametrize("E", [1, 2, 3, 7, 12, 33])
def test_pairing_counts(E):
    """F = 2E - 1 fronts and height ceil(log2 E) (each round halves the list, rounding up)."""
    m, t = _pairing_tree((E, 1))
    assert t.n_fronts == 2 * E - 1
    assert t.height == int(np.ceil(np.log2(E))) if E > 1 else t.height == 0
    # every node is a pivot exactly once
    piv = np.concatenate([t.pivots(f) for f in range(t.n_fronts)])
    assert sorted(piv.tolist()) == list(range(m.n_nodes))
