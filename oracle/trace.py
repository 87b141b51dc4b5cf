"""Oracle: the scalar-task trace of the factorization and its Foata normal form (test
infrastructure only, see the package docstring).  Tiny meshes only: the task count grows with
the sum of m^3 over the fronts.

The task alphabet (Sec. 3, eq. alphabet), with z the pivot, x a row and y a column of the
global matrix and f the front eliminating z:
  T1(f, z, y)     division: the entry (z, y) of the pivot row, y after z in the front, by the
                  pivot (z, z);
  T2(f, z, x, y)  multiplication: that quotient times the entry (x, z) of the pivot column;
  T3(f, z, x, y)  subtraction: the product subtracted from the global entry (x, y);
  T4(x, y)        assertion: the global entry (x, y) holds its final value.
Dependencies (Sec. 3.1, J1..J4), each from an earlier to a later task of the trace:
  J1  T4(z, z) -> T1(f, z, y),  T4(z, y) -> T1(f, z, y);
  J2  T1(f, z, y) -> T2(f, z, x, y),  T4(x, z) -> T2(f, z, x, y);
  J3  T2(f, z, x, y) -> T3(f, z, x, y), and every subtraction into the same entry (x, y)
      that comes first -> T3(f, z, x, y);
  J4  every T3 into (x, y) -> T4(x, y).
Reading of "first" in J3 (the paper orders by the global pivot index z, then the front): z is
compared by its position in the elimination order, so the subtractions into one entry form a
chain in the order the factorization issues them.  Every T4 exists, also for entries that no
subtraction touches (Sec. 3.1: an assertion for each global entry).

Foata normal form: every task in the earliest class after all its predecessors (class 1 for a
task without predecessors), i.e. the classes of the longest-path layering of the dependency
graph -- the unique FNF of the trace (Sec. 3.3).  ``typed_classes`` places every task in the
earliest class after its predecessors whose number is congruent to its type
(T4: 1, T1: 2, T2: 3, T3: 0 mod 4), the 4-periodic class structure of Sec. 3.3; it is a valid
schedule by construction.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from .dense import elimination_order
from .tree import Tree

TYPE_RESIDUE = {"T4": 1, "T1": 2, "T2": 3, "T3": 0}


def tasks_and_preds(tree: Tree):
    """(preds, front_of): preds maps each task key to its list of predecessor keys; front_of
    maps the T1..T3 keys to their front.  Keys: ("T1", f, z, y), ("T2", f, z, x, y),
    ("T3", f, z, x, y), ("T4", x, y) with global node ids."""
    order = elimination_order(tree)
    pos = np.empty(len(order), dtype=np.int64)
    pos[order] = np.arange(len(order))
    preds = {}
    front_of = {}
    subs = defaultdict(list)          # (x, y) -> subtraction keys in issue order
    fronts = sorted(range(tree.n_fronts), key=lambda f: (pos[tree.pivots(f)].min()
                                                         if tree.npiv[f] else -1, f))
    for f in fronts:
        idx = [int(v) for v in tree.index_list(f)]
        k = int(tree.npiv[f])
        for p in range(k):
            z = idx[p]
            for j in range(p + 1, len(idx)):
                y = idx[j]
                t1 = ("T1", f, z, y)
                preds[t1] = [("T4", z, z), ("T4", z, y)]
                front_of[t1] = f
                for i in range(p + 1, len(idx)):
                    x = idx[i]
                    t2 = ("T2", f, z, x, y)
                    t3 = ("T3", f, z, x, y)
                    preds[t2] = [t1, ("T4", x, z)]
                    preds[t3] = [t2] + list(subs[(x, y)])
                    front_of[t2] = front_of[t3] = f
                    subs[(x, y)].append(t3)
    for x in range(tree.n):
        for y in range(tree.n):
            preds[("T4", x, y)] = list(subs.get((x, y), []))
    return preds, front_of


def _layer(preds, typed: bool):
    cls = {}

    def c(key):
        if key in cls:
            return cls[key]
        stack = [key]
        while stack:
            kk = stack[-1]
            todo = [q for q in preds[kk] if q not in cls]
            if todo:
                stack.extend(todo)
                continue
            stack.pop()
            if kk in cls:
                continue
            v = 1 + max((cls[q] for q in preds[kk]), default=0)
            if typed:
                want = TYPE_RESIDUE[kk[0]]
                while v % 4 != want:
                    v += 1
            cls[kk] = v
        return cls[key]

    for key in preds:
        c(key)
    return cls


def fnf_classes(preds):
    """Foata class (1-based) of every task: the longest-path layering."""
    return _layer(preds, typed=False)


def typed_classes(preds):
    """Earliest class after the predecessors with the type's residue mod 4."""
    return _layer(preds, typed=True)


def summary(tree: Tree):
    """Counts of the trace: tasks per type, FNF classes, classes holding a single task type,
    typed (4-periodic) classes, and whether the front classes (tree heights) order every
    dependency between tasks of fronts."""
    preds, front_of = tasks_and_preds(tree)
    fnf = fnf_classes(preds)
    typ = typed_classes(preds)
    per_type = defaultdict(int)
    for kk in preds:
        per_type[kk[0]] += 1
    by_class = defaultdict(set)
    for kk, v in fnf.items():
        by_class[v].add(kk[0])
    pure = sum(1 for v in by_class.values() if len(v) == 1)
    level_ok = all(tree.level[front_of[q]] <= tree.level[front_of[kk]]
                   for kk in front_of for q in preds[kk] if q in front_of)
    return {
        "tasks": dict(per_type),
        "fnf_classes": max(fnf.values()),
        "fnf_single_type_classes": pure,
        "typed_classes": max(typ.values()),
        "typed_valid": all(typ[q] < typ[kk] for kk in preds for q in preds[kk]),
        "front_levels_order_dependencies": level_ok,
    }
