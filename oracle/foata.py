"""Oracle: Foata-normal-form checks of the front-level trace (test infrastructure only).

Sec. 3.3 runs the computation as a sequence of Foata classes: tasks inside one class are
mutually independent and may run in any order, and a class starts only after the previous class
has finished.  At front granularity the only dependency is child -> parent (a front needs its
children's Schur complements, Sec. 2.3), so the Foata normal form is obtained by repeatedly
removing every front whose children have all been removed.  ``fnf_classes`` computes exactly
that peeling; ``check`` verifies a given level array against it and checks independence.
"""
from __future__ import annotations

import numpy as np

from .tree import Tree


def fnf_classes(tree: Tree) -> np.ndarray:
    F = tree.n_fronts
    cls = np.full(F, -1, dtype=np.int64)
    remaining_children = np.zeros(F, dtype=np.int64)
    for f in range(F):
        if tree.parent[f] >= 0:
            remaining_children[tree.parent[f]] += 1
    frontier = [f for f in range(F) if remaining_children[f] == 0]
    c = 0
    while frontier:
        nxt = []
        for f in frontier:
            cls[f] = c
        for f in frontier:
            p = int(tree.parent[f])
            if p >= 0:
                remaining_children[p] -= 1
                if remaining_children[p] == 0:
                    nxt.append(p)
        frontier = nxt
        c += 1
    return cls


def check(tree: Tree, level: np.ndarray) -> list:
    """Returns a list of violated properties (empty when ``level`` is the Foata normal form)."""
    errs = []
    if not np.array_equal(fnf_classes(tree), np.asarray(level)):
        errs.append("levels differ from the Foata normal form of the front trace")
    # independence inside a class: no ancestor relation, disjoint pivot sets
    anc_sets = []
    for f in range(tree.n_fronts):
        s = set()
        p = int(tree.parent[f])
        while p >= 0:
            s.add(p)
            p = int(tree.parent[p])
        anc_sets.append(s)
    for l in range(int(np.max(level)) + 1):
        fs = np.flatnonzero(np.asarray(level) == l)
        fset = set(int(f) for f in fs)
        for f in fs:
            if anc_sets[int(f)] & fset:
                errs.append(f"class {l}: front {int(f)} has an ancestor in the same class")
                break
        piv = np.concatenate([tree.pivots(int(f)) for f in fs]) if len(fs) else np.array([])
        if np.unique(piv).size != piv.size:
            errs.append(f"class {l}: pivot sets overlap")
        for f in fs:
            if l > 0:
                kids = [c for c in (int(tree.left[f]), int(tree.right[f])) if c >= 0]
                if not kids or max(int(level[c]) for c in kids) != l - 1:
                    errs.append(f"class {l}: front {int(f)} has no child in class {l-1}")
                    break
    return errs
