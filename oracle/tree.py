"""Oracle: elimination tree, Foata levels and front structure of a (batch of) Q1 mesh(es).

Test infrastructure only (see the package docstring).

What the paper fixes (Sec. 2.4): the leaves of the elimination tree are the element matrices;
fronts are joined pairwise into a binary tree that follows the mesh; the root is the largest,
fully assembled front.  Sec. 3.2 reorders every front so that the pivots eliminated at the
current level come first, followed by the entries still shared with other fronts; entries
eliminated at lower levels do not reappear.  A pivot is eliminated in the (unique) front that
owns it alone (Table 2's membership-count condition).  Sec. 3.3 executes the fronts class by
class in Foata normal form.

Readings taken where the paper is not explicit:
  * Tree rule (meshes with element coordinates): recursive coordinate bisection of the element
    index box (nested dissection).
    Split the axis with the most elements (ties: lowest axis), cut at lo + floor(len/2), lower
    half is the left child, recurse down to single elements.  Fronts are numbered in post-order
    (left subtree, right subtree, node).  Without coordinates (connectivity only) the tree is
    Table 3 literally: sort the element fronts by lowest node id (ties: element id), join
    adjacent pairs round after round, carry an odd last front to the next round.
  * Node v is a pivot of front F iff F is the lowest common ancestor of all elements that
    contain v (the first front whose element set holds every element touching v).
  * Contribution block: CB(leaf) = element nodes minus its pivots;
    CB(F) = (CB(left) u CB(right)) minus pivots(F).
  * Front index list: pivots ascending by global id, then CB ascending by global id.
  * level(F) = 0 for a leaf, else 1 + max(level(children)) -- the Foata class of F in the
    front-level trace where each front depends on its children.
  * Batch: each mesh keeps its own tree; fronts of mesh 0 come first, then mesh 1, ...; node ids
    are offset by the prefix sum of node counts.  The batch's class l is the union of the meshes'
    class l (the Foata normal form of a disjoint union is the class-wise union).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Tree:
    parent: np.ndarray      # (F,) int32, -1 for a root
    left: np.ndarray        # (F,) int32, -1 for a leaf
    right: np.ndarray       # (F,) int32, -1 for a leaf
    leaf_elem: np.ndarray   # (F,) int64 global element id, -1 for internal fronts
    mesh_of: np.ndarray     # (F,) int32 mesh index
    level: np.ndarray       # (F,) int32 Foata class (0-based)
    npiv: np.ndarray        # (F,) int32 number of pivots k
    front_ptr: np.ndarray   # (F+1,) int64 offsets into front_idx
    front_idx: np.ndarray   # (sum m,) int32 global node ids: pivots ascending, then CB ascending
    n: int

    @property
    def n_fronts(self) -> int:
        return int(self.parent.shape[0])

    @property
    def height(self) -> int:
        return int(self.level.max())

    def m(self, f: int) -> int:
        return int(self.front_ptr[f + 1] - self.front_ptr[f])

    def index_list(self, f: int) -> np.ndarray:
        return self.front_idx[self.front_ptr[f]:self.front_ptr[f + 1]]

    def pivots(self, f: int) -> np.ndarray:
        return self.index_list(f)[: self.npiv[f]]

    def cb(self, f: int) -> np.ndarray:
        return self.index_list(f)[self.npiv[f]:]

    def levels(self):
        """Fronts of each class, ascending front id (the oracle's 'tree order' inside a class)."""
        return [np.flatnonzero(self.level == l) for l in range(self.height + 1)]

    def child_map(self, f: int, child: int) -> np.ndarray:
        """Extend-add map: position of each CB entry of ``child`` in the index list of ``f``."""
        pos = {int(v): i for i, v in enumerate(self.index_list(f))}
        return np.array([pos[int(v)] for v in self.cb(child)], dtype=np.int64)

    def leaf_map(self, f: int, conn_row: np.ndarray) -> np.ndarray:
        """Position of each local element node in the index list of leaf ``f``."""
        pos = {int(v): i for i, v in enumerate(self.index_list(f))}
        return np.array([pos[int(v)] for v in conn_row], dtype=np.int64)


def _bisect(ijk: np.ndarray, elems: np.ndarray, out: list) -> int:
    """Recursive coordinate bisection; appends fronts in post-order, returns the subtree root."""
    if elems.size == 1:
        out.append((-1, -1, int(elems[0])))
        return len(out) - 1
    sub = ijk[elems]
    lo = sub.min(axis=0)
    ln = sub.max(axis=0) - lo + 1
    axis = int(np.argmax(ln))               # first maximum: ties go to the lowest axis
    cut = lo[axis] + ln[axis] // 2
    mask = sub[:, axis] < cut
    l = _bisect(ijk, elems[mask], out)
    r = _bisect(ijk, elems[~mask], out)
    out.append((l, r, -1))
    return len(out) - 1


def _pairing(conn: np.ndarray, out: list) -> int:
    """Table 3: element fronts sorted by lowest node id (ties: element id), joined in adjacent
    pairs round after round, an odd last front carried; appends fronts in post-order."""
    order = sorted(range(conn.shape[0]), key=lambda e: (int(conn[e].min()), e))
    items = [("leaf", e) for e in order]
    while len(items) > 1:
        joined = [(items[i], items[i + 1]) for i in range(0, len(items) - 1, 2)]
        if len(items) % 2 == 1:
            joined.append(items[-1])
        items = joined

    def emit(node) -> int:
        if node[0] == "leaf":
            out.append((-1, -1, int(node[1])))
            return len(out) - 1
        left = emit(node[0])
        right = emit(node[1])
        out.append((left, right, -1))
        return len(out) - 1

    return emit(items[0])


def _one_mesh(conn: np.ndarray, ijk, n_nodes: int):
    E = conn.shape[0]
    if E < 1:
        raise ValueError("empty mesh")
    if ijk is not None and np.unique(ijk, axis=0).shape[0] != E:
        raise ValueError("duplicate element coordinates")
    if conn.min() < 0 or conn.max() >= n_nodes:
        raise ValueError("node id out of range")
    nodes = []
    if ijk is None:
        _pairing(conn, nodes)
    else:
        _bisect(np.asarray(ijk).astype(np.int64), np.arange(E, dtype=np.int64), nodes)
    F = len(nodes)
    left = np.array([t[0] for t in nodes], dtype=np.int64)
    right = np.array([t[1] for t in nodes], dtype=np.int64)
    elem = np.array([t[2] for t in nodes], dtype=np.int64)
    parent = np.full(F, -1, dtype=np.int64)
    for f in range(F):
        if left[f] >= 0:
            parent[left[f]] = f
            parent[right[f]] = f
    # level = height (post-order guarantees children come first)
    level = np.zeros(F, dtype=np.int64)
    for f in range(F):
        if left[f] >= 0:
            level[f] = 1 + max(level[left[f]], level[right[f]])
    depth = np.zeros(F, dtype=np.int64)
    for f in range(F - 1, -1, -1):            # parents have larger ids
        if parent[f] >= 0:
            depth[f] = depth[parent[f]] + 1
    leaf_of_elem = np.empty(E, dtype=np.int64)
    for f in range(F):
        if elem[f] >= 0:
            leaf_of_elem[elem[f]] = f

    def lca(a: int, b: int) -> int:
        while depth[a] > depth[b]:
            a = parent[a]
        while depth[b] > depth[a]:
            b = parent[b]
        while a != b:
            a, b = parent[a], parent[b]
        return a

    owner = np.full(n_nodes, -1, dtype=np.int64)
    for e in range(E):
        lf = leaf_of_elem[e]
        for v in conn[e]:
            v = int(v)
            owner[v] = lf if owner[v] < 0 else lca(int(owner[v]), int(lf))
    if (owner < 0).any():
        raise ValueError("node not referenced by any element")
    piv = [[] for _ in range(F)]
    for v in range(n_nodes):
        piv[owner[v]].append(v)
    cbs = [None] * F
    for f in range(F):
        pset = set(piv[f])
        if elem[f] >= 0:
            base = set(int(v) for v in conn[elem[f]])
        else:
            base = set(cbs[left[f]]) | set(cbs[right[f]])
        cbs[f] = sorted(base - pset)
    lists = [sorted(piv[f]) + cbs[f] for f in range(F)]
    npiv = np.array([len(piv[f]) for f in range(F)], dtype=np.int64)
    return parent, left, right, elem, level, npiv, lists


def build_tree(meshes) -> Tree:
    """Nested-dissection tree of a batch of meshes (objects with .conn, .ijk, .n_nodes)."""
    parts = {k: [] for k in ("parent", "left", "right", "elem", "level", "npiv", "mesh")}
    all_lists = []
    f_off = 0
    n_off = 0
    e_off = 0
    for mi, mesh in enumerate(meshes):
        conn = np.asarray(mesh.conn, dtype=np.int64)
        ijk = None if mesh.ijk is None else np.asarray(mesh.ijk)
        parent, left, right, elem, level, npiv, lists = _one_mesh(conn, ijk, mesh.n_nodes)
        shift = lambda a: np.where(a >= 0, a + f_off, -1)
        parts["parent"].append(shift(parent))
        parts["left"].append(shift(left))
        parts["right"].append(shift(right))
        parts["elem"].append(np.where(elem >= 0, elem + e_off, -1))
        parts["level"].append(level)
        parts["npiv"].append(npiv)
        parts["mesh"].append(np.full(parent.shape[0], mi, dtype=np.int64))
        all_lists.extend([[v + n_off for v in lst] for lst in lists])
        f_off += parent.shape[0]
        n_off += mesh.n_nodes
        e_off += conn.shape[0]
    sizes = np.array([len(l) for l in all_lists], dtype=np.int64)
    front_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    front_idx = np.array([v for l in all_lists for v in l], dtype=np.int32)
    cat = lambda k, dt: np.concatenate(parts[k]).astype(dt)
    return Tree(cat("parent", np.int32), cat("left", np.int32), cat("right", np.int32),
                cat("elem", np.int64), cat("mesh", np.int32), cat("level", np.int32),
                cat("npiv", np.int32), front_ptr, front_idx, n_off)


def front_flops(tree: Tree):
    """Algorithmic operation counts: per pivot p of a front of width m (r = m - p remaining),
    the division tasks number r-1 and the multiplication and subtraction tasks (r-1)^2 each
    (Sec. 3: one division per entry right of the pivot, one multiplication and one subtraction
    per entry of the trailing block).  Solve: per pivot one division and 2(r-1) multiply-adds in
    each of the forward and backward sweeps, per right-hand side."""
    fac = 0
    sol = 0
    cb2 = 0
    for f in range(tree.n_fronts):
        m = tree.m(f)
        k = int(tree.npiv[f])
        for p in range(k):
            r = m - p
            fac += (r - 1) + 2 * (r - 1) ** 2
            sol += 1 + 4 * (r - 1)
        cb2 += (m - k) ** 2
    return fac, sol, cb2
