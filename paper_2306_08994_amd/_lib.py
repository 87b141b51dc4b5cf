"""ctypes declarations of libmf's C ABI (include/mf.h).  Loading fails loudly when the library
has not been built: there is no CPU fallback anywhere in this package."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmf.so")

MF_OK, MF_EINVAL, MF_ENOMEM, MF_EZERO_PIVOT, MF_EHIP, MF_ENOCONV, MF_ESTATE = 0, -1, -2, -3, -4, -5, -6
MF_FP64, MF_SCHUR_FP32, MF_SCHUR_BF16 = 0, 1, 2
MF_NOALLOC_SCRATCH_DOUBLES = 8388608     # include/mf.h
ERROR_NAMES = {MF_EINVAL: "MF_EINVAL", MF_ENOMEM: "MF_ENOMEM", MF_EZERO_PIVOT: "MF_EZERO_PIVOT",
               MF_EHIP: "MF_EHIP", MF_ENOCONV: "MF_ENOCONV", MF_ESTATE: "MF_ESTATE"}

EXPORTED = ["mf_analyse", "mf_plan_info", "mf_plan_export_tree", "mf_task_trace", "mf_set_tuning",
            "mf_set_class_tuning", "mf_set_subtree_launch", "mf_subtree_launch_info", "mf_set_chunked_solve",
            "mf_autotune",
            "mf_factor", "mf_solve", "mf_solve_noalloc",
            "mf_residual", "mf_refine", "mf_refine_gmres", "mf_factor_refine", "mf_elem_grad", "mf_export_factors", "mf_profile",
            "mf_profile_report", "mf_destroy", "mf_last_error"]


class MfMesh(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("npe", c_int32), ("n_nodes", c_int64), ("n_elem", c_int64),
                ("conn", POINTER(c_int32)), ("elem_ijk", POINTER(c_int32))]


class MfTraceInfo(ctypes.Structure):
    _fields_ = [("tasks", c_int64 * 4), ("fnf_classes", c_int32),
                ("fnf_single_type_classes", c_int32), ("typed_classes", c_int32),
                ("levels_order_dependencies", c_int32)]


class MfInfo(ctypes.Structure):
    _fields_ = [("n", c_int64), ("n_elem", c_int64), ("n_fronts", c_int64), ("sum_m", c_int64),
                ("sum_mk", c_int64), ("store_doubles", c_int64), ("n_mesh", c_int32),
                ("dim", c_int32), ("npe", c_int32), ("height", c_int32), ("max_m", c_int32),
                ("max_k", c_int32), ("factor_flops", c_double), ("solve_flops_per_rhs", c_double),
                ("sum_cb2", c_double)]


class MFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2306_08994_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    dp = POINTER(c_double)
    sig = {
        "mf_analyse": (c_int32, [c_int32, POINTER(MfMesh), POINTER(c_void_p)]),
        "mf_plan_info": (c_int32, [P, POINTER(MfInfo)]),
        "mf_plan_export_tree": (c_int32, [P, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p]),
        "mf_task_trace": (c_int32, [P, POINTER(MfTraceInfo), c_void_p, c_int64, POINTER(c_int64)]),
        "mf_set_tuning": (c_int32, [P, c_int32, c_int32, c_int32, c_int32, c_int32]),
        "mf_set_class_tuning": (c_int32, [P, c_int32, c_void_p]),
        "mf_set_subtree_launch": (c_int32, [P, c_int32, c_int64]),
        "mf_subtree_launch_info": (c_int32, [P, POINTER(c_int64)]),
        "mf_set_chunked_solve": (c_int32, [P, c_int32]),
        "mf_autotune": (c_int32, [P, c_void_p, c_int32, c_int32, c_void_p, c_char_p, c_int64,
                                  POINTER(c_int64)]),
        "mf_factor": (c_int32, [P, c_void_p, c_int32, c_void_p]),
        "mf_solve": (c_int32, [P, c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
        "mf_solve_noalloc": (c_int32, [P, c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
        "mf_residual": (c_int32, [P, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
        "mf_refine": (c_int32, [P, c_void_p, c_void_p, c_void_p, c_int32, c_double, c_int32,
                                POINTER(c_int32), dp, c_void_p]),
        "mf_refine_gmres": (c_int32, [P, c_void_p, c_void_p, c_void_p, c_int32, c_double, c_int32,
                                      c_int32, POINTER(c_int32), dp, c_void_p]),
        "mf_factor_refine": (c_int32, [P, c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_double,
                                       c_int32, POINTER(c_int32), dp, c_void_p]),
        "mf_elem_grad": (c_int32, [P, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
        "mf_export_factors": (c_int32, [P, c_void_p, c_void_p]),
        "mf_profile": (c_int32, [P, c_int32]),
        "mf_profile_report": (c_int32, [P, c_char_p, c_int64, POINTER(c_int64)]),
        "mf_destroy": (None, [P]),
        "mf_last_error": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != MF_OK:
        raise MFError(rc, load().mf_last_error().decode(errors="replace"))
