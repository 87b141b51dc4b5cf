"""The scalar-task trace of the factorization (the task alphabet and dependencies of Sec. 3, the
Foata normal form of Sec. 3.3): the oracle pinned by closed forms and by an independent
computation of the normal form, and the library's mf_task_trace equal to the oracle.

  * one element: its front is dense and eliminates every node, so the trace is the dense LU of
    an m x m matrix; its Foata normal form has 4(m-1)+1 classes, each of a single task type in
    the order assertion, division, multiplication, subtraction (the 4-periodic structure);
  * task counts: divisions + multiplications + subtractions equal the method's operation count
    (front_flops) and there is one assertion per global entry;
  * the normal form equals the peeling definition (repeatedly take every task whose
    predecessors are all taken), computed without the longest-path recursion;
  * the 4-periodic typed schedule is valid (every dependency goes to a later class) and never
    shorter than the normal form; with more than one element the normal form itself mixes task
    types in some classes (reading recorded with the oracle);
  * the front classes (tree heights) order every dependency between the tasks of two fronts.
Host work only."""
import os

import numpy as np
import pytest

from fixtures import structured_q1, structured_qp
from oracle import trace
from oracle.tree import build_tree, front_flops

lib_mod = pytest.importorskip("paper_2306_08994_amd._lib")


def _peel(preds):
    """Foata classes by peeling: class c = the tasks whose predecessors all lie in classes < c."""
    remaining = {k: len(v) for k, v in preds.items()}
    succ = {k: [] for k in preds}
    for k, v in preds.items():
        for q in v:
            succ[q].append(k)
    frontier = [k for k, c in remaining.items() if c == 0]
    cls, c = {}, 0
    while frontier:
        c += 1
        nxt = []
        for k in frontier:
            cls[k] = c
        for k in frontier:
            for s in succ[k]:
                remaining[s] -= 1
                if remaining[s] == 0:
                    nxt.append(s)
        frontier = nxt
    assert len(cls) == len(preds)
    return cls


@pytest.mark.parametrize("mesh", [structured_q1((1, 1)), structured_q1((1, 1, 1)),
                                  structured_qp((1, 1), 2), structured_qp((1, 1), 3)],
                         ids=["q1-2d", "q1-3d", "q2-2d", "q3-2d"])
def test_one_element_is_dense_lu(mesh):
    tree = build_tree([mesh])
    m = mesh.npe
    preds, _ = trace.tasks_and_preds(tree)
    fnf = trace.fnf_classes(preds)
    assert max(fnf.values()) == 4 * (m - 1) + 1
    for key, c in fnf.items():
        assert c % 4 == trace.TYPE_RESIDUE[key[0]], key
    assert trace.typed_classes(preds) == fnf
    s = trace.summary(tree)
    assert s["fnf_single_type_classes"] == s["fnf_classes"] == s["typed_classes"]


@pytest.mark.parametrize("shape", [(2, 1), (2, 2), (3, 2), (1, 1, 1), (2, 2, 1)])
def test_task_counts(shape):
    mesh = structured_q1(shape)
    tree = build_tree([mesh])
    s = trace.summary(tree)
    fac, _, _ = front_flops(tree)
    t = s["tasks"]
    assert t["T1"] + t["T2"] + t["T3"] == fac
    assert t["T2"] == t["T3"]
    assert t["T4"] == mesh.n_nodes ** 2


@pytest.mark.parametrize("shape", [(2, 1), (2, 2), (3, 2), (2, 1, 1)])
def test_normal_form_is_the_peeling(shape):
    tree = build_tree([structured_q1(shape)])
    preds, _ = trace.tasks_and_preds(tree)
    assert trace.fnf_classes(preds) == _peel(preds)


@pytest.mark.parametrize("shape", [(2, 2), (3, 2), (4, 3), (2, 2, 1)])
def test_typed_schedule_and_front_classes(shape):
    tree = build_tree([structured_q1(shape)])
    s = trace.summary(tree)
    assert s["typed_valid"] and s["typed_classes"] >= s["fnf_classes"]
    assert s["front_levels_order_dependencies"]
    # more than one element: subtractions of different fronts into a shared entry are chained
    # (J3), which shifts some tasks off the 4-periodic pattern in the normal form
    assert s["typed_classes"] > s["fnf_classes"]


def _lib_ready():
    return os.path.exists(lib_mod.LIB_PATH)


@pytest.mark.skipif(not _lib_ready(), reason="libmf.so not built")
@pytest.mark.parametrize("mesh", [structured_q1(s) for s in [(1, 1), (2, 2), (4, 3), (2, 2, 2), (5, 4)]]
                         + [structured_qp((2, 2), 2), structured_qp((2, 1), 3)],
                         ids=["1x1", "2x2", "4x3", "2x2x2", "5x4", "q2", "q3"])
def test_library_trace_equals_oracle(mesh):
    from paper_2306_08994_amd import Plan
    a = Plan([mesh]).task_trace()
    tree = build_tree([mesh])
    o = trace.summary(tree)
    for key in ("tasks", "fnf_classes", "fnf_single_type_classes", "typed_classes",
                "front_levels_order_dependencies"):
        assert a[key] == o[key], key
    preds, _ = trace.tasks_and_preds(tree)
    fnf = trace.fnf_classes(preds)
    hist = np.zeros((max(fnf.values()) + 1, 4), np.int64)
    col = {"T1": 0, "T2": 1, "T3": 2, "T4": 3}
    for key, c in fnf.items():
        hist[c, col[key[0]]] += 1
    np.testing.assert_array_equal(a["hist"], hist)


@pytest.mark.skipif(not _lib_ready(), reason="libmf.so not built")
def test_library_trace_refuses_large_meshes():
    from paper_2306_08994_amd import MFError, Plan
    with pytest.raises(MFError):
        Plan([structured_q1((64, 64))]).task_trace()
