"""Python face of libmf: argument marshalling only.  Every step of the factor and solve runs in
the HIP kernels behind the C ABI; torch provides device memory and the current stream."""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np

from . import _lib
from ._lib import MFError, check  # noqa: F401

PRECISIONS = {"fp64": _lib.MF_FP64, "fp32": _lib.MF_SCHUR_FP32, "bf16": _lib.MF_SCHUR_BF16}


def _stream():
    """The current HIP stream of the current device (its raw handle: building a Stream object
    per call costs more than the rest of a call's marshalling)."""
    import torch
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return ctypes.c_void_p(raw(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Analysed elimination tree of one mesh or a batch of meshes (see mf_analyse).

    ``meshes``: objects with ``conn`` (E, npe) and ``ijk`` (E, dim) integer arrays, ``dim`` and
    ``n_nodes`` (``fixtures.Mesh`` satisfies this).  ``ijk`` None: connectivity-only tree."""

    def __init__(self, meshes: Sequence):
        lib = _lib.load()
        self._keep = []
        arr = (_lib.MfMesh * len(meshes))()
        for i, m in enumerate(meshes):
            conn = np.ascontiguousarray(m.conn, dtype=np.int32)
            ijk = None if m.ijk is None else np.ascontiguousarray(m.ijk, dtype=np.int32)
            self._keep += [conn, ijk]
            arr[i].dim = int(m.dim)
            arr[i].npe = int(conn.shape[1])
            arr[i].n_nodes = int(m.n_nodes)
            arr[i].n_elem = int(conn.shape[0])
            arr[i].conn = conn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            arr[i].elem_ijk = (None if ijk is None
                               else ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        h = ctypes.c_void_p()
        check(lib.mf_analyse(len(meshes), arr, ctypes.byref(h)))
        self._h = h
        self._keep = []
        inf = _lib.MfInfo()
        check(lib.mf_plan_info(self._h, ctypes.byref(inf)))
        self.info = {k: getattr(inf, k) for k, _ in _lib.MfInfo._fields_}
        self.n = int(inf.n)
        self.n_elem = int(inf.n_elem)
        self.npe = int(inf.npe)
        self.factor_version = 0     # bumped by every factor call (autograd staleness check)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().mf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- structure ---------------------------------------------------------------------------
    def export_tree(self) -> dict:
        F = int(self.info["n_fronts"])
        out = {"parent": np.empty(F, np.int32), "level": np.empty(F, np.int32),
               "front_ptr": np.empty(F + 1, np.int64),
               "front_idx": np.empty(int(self.info["sum_m"]), np.int32),
               "npiv": np.empty(F, np.int32), "leaf_elem": np.empty(F, np.int64)}
        ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
        check(_lib.load().mf_plan_export_tree(self._h, ptr(out["parent"]), ptr(out["level"]),
                                              ptr(out["front_ptr"]), ptr(out["front_idx"]),
                                              ptr(out["npiv"]), ptr(out["leaf_elem"])))
        return out

    def task_trace(self) -> dict:
        """Scalar-task trace of the factorization and its Foata classes (mf_task_trace): task
        counts, class counts and the per-class histogram hist[c, t] (t: T1, T2, T3, T4)."""
        lib = _lib.load()
        info = _lib.MfTraceInfo()
        need = ctypes.c_int64(0)
        check(lib.mf_task_trace(self._h, ctypes.byref(info), None, 0, ctypes.byref(need)))
        hist = np.zeros(int(need.value), np.int64)
        check(lib.mf_task_trace(self._h, ctypes.byref(info), ctypes.c_void_p(hist.ctypes.data),
                                int(need.value), ctypes.byref(need)))
        return {"tasks": {"T1": int(info.tasks[0]), "T2": int(info.tasks[1]),
                          "T3": int(info.tasks[2]), "T4": int(info.tasks[3])},
                "fnf_classes": int(info.fnf_classes),
                "fnf_single_type_classes": int(info.fnf_single_type_classes),
                "typed_classes": int(info.typed_classes),
                "front_levels_order_dependencies": bool(info.levels_order_dependencies),
                "hist": hist.reshape(-1, 4)}

    def set_tuning(self, small_max_m: int = 0, nb: int = 0, fused_max_m: int = 0, tile: int = 0,
                   persistent: int = 0):
        """See mf_set_tuning: 0 keeps a value; fused_max_m=-1 disables the fused panel route;
        persistent=1 / -1 switches the persistent class launches on / off."""
        self.factor_version += 1
        check(_lib.load().mf_set_tuning(self._h, int(small_max_m), int(nb), int(fused_max_m),
                                        int(tile), int(persistent)))

    def set_class_tuning(self, classes):
        """Per-class schedule (see mf_set_class_tuning): one dict per Foata class with keys
        small_max_m, nb, fused_max_m, tile, persistent (e.g. autotune()["chosen"]["classes"]);
        an empty list drops it."""
        self.factor_version += 1
        if not classes:
            check(_lib.load().mf_set_class_tuning(self._h, 0, None))
            return
        keys = ("small_max_m", "nb", "fused_max_m", "tile", "persistent")
        arr = np.ascontiguousarray([[int(c[k]) for k in keys] for c in classes], dtype=np.int32)
        check(_lib.load().mf_set_class_tuning(self._h, len(classes),
                                              ctypes.c_void_p(arr.ctypes.data)))

    def set_subtree_launch(self, max_classes: int = -1, min_units: int = 2048):
        """Bottom-subtree launches (see mf_set_subtree_launch): at most max_classes leading
        classes as one launch (-1: as the routes allow, 0 / 1: off, the library's default), with
        >= min_units units."""
        self.factor_version += 1
        check(_lib.load().mf_set_subtree_launch(self._h, int(max_classes), int(min_units)))

    def subtree_launch_info(self) -> dict:
        """Classes fused and units of the factorization's and the solves' subtree launches."""
        out = (ctypes.c_int64 * 4)()
        check(_lib.load().mf_subtree_launch_info(self._h, out))
        return {"factor_classes": out[0], "factor_units": out[1], "solve_classes": out[2],
                "solve_units": out[3]}

    def set_chunked_solve(self, min_pivots: int = 512):
        """Chunked triangle solves for classes whose widest front has >= min_pivots pivots
        (see mf_set_chunked_solve; 0 = off)."""
        check(_lib.load().mf_set_chunked_solve(self._h, int(min_pivots)))

    def autotune(self, K, precision: str = "fp64", reps: int = 3) -> dict:
        """Times the relevant schedule candidates on K, keeps the fastest (see mf_autotune)."""
        import json
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        p = _dev_ptr(K, "K", (self.n_elem, self.npe, self.npe))
        self.factor_version += 1
        buf = ctypes.create_string_buffer(1 << 16)
        need = ctypes.c_int64(0)
        check(_lib.load().mf_autotune(self._h, p, PRECISIONS[precision], int(reps), _stream(),
                                      buf, len(buf), ctypes.byref(need)))
        return json.loads(buf.value.decode())

    # -- numerics ----------------------------------------------------------------------------
    def factor(self, K, precision: str = "fp64"):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        p = _dev_ptr(K, "K", (self.n_elem, self.npe, self.npe))
        self.factor_version += 1
        check(_lib.load().mf_factor(self._h, p, PRECISIONS[precision], _stream()))

    def solve(self, b, transpose: bool = False, out=None):
        import torch
        b2 = b if b.dim() == 2 else b.reshape(-1, 1)
        nrhs = int(b2.shape[1])
        pb = _dev_ptr(b2, "b", (self.n, nrhs))
        x = torch.empty_like(b2) if out is None else out.reshape(self.n, nrhs)
        px = _dev_ptr(x, "x", (self.n, nrhs))
        check(_lib.load().mf_solve(self._h, pb, px, nrhs, int(bool(transpose)), _stream()))
        return x.reshape(b.shape)

    def solve_noalloc(self, b, out, transpose: bool = False):
        """mf_solve_noalloc: the solve without any device allocation in the call (the output
        buffer `out` is the caller's); its workspace is the library's static scratch."""
        b2 = b if b.dim() == 2 else b.reshape(-1, 1)
        nrhs = int(b2.shape[1])
        pb = _dev_ptr(b2, "b", (self.n, nrhs))
        x = out.reshape(self.n, nrhs)
        px = _dev_ptr(x, "x", (self.n, nrhs))
        check(_lib.load().mf_solve_noalloc(self._h, pb, px, nrhs, int(bool(transpose)),
                                           _stream()))
        return out

    def residual(self, K, x, b):
        import torch
        b2 = b if b.dim() == 2 else b.reshape(-1, 1)
        nrhs = int(b2.shape[1])
        r = torch.empty_like(b2)
        check(_lib.load().mf_residual(self._h, _dev_ptr(K, "K", (self.n_elem, self.npe, self.npe)),
                                      _dev_ptr(x.reshape(self.n, nrhs), "x"), _dev_ptr(b2, "b"),
                                      _dev_ptr(r, "r"), nrhs, _stream()))
        return r.reshape(b.shape)

    def refine(self, K, b, tol: float = 1e-12, max_it: int = 30, x=None):
        """Solve with FP64 iterative refinement; returns (x, corrections, relres)."""
        import torch
        b2 = b if b.dim() == 2 else b.reshape(-1, 1)
        nrhs = int(b2.shape[1])
        x = torch.empty_like(b2) if x is None else x.reshape(self.n, nrhs)
        its = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        check(_lib.load().mf_refine(self._h, _dev_ptr(K, "K", (self.n_elem, self.npe, self.npe)),
                                    _dev_ptr(b2, "b", (self.n, nrhs)), _dev_ptr(x, "x"), nrhs,
                                    float(tol), int(max_it), ctypes.byref(its), ctypes.byref(rr),
                                    _stream()))
        return x.reshape(b.shape), int(its.value), float(rr.value)

    def refine_gmres(self, K, b, tol: float = 1e-12, max_it: int = 60, restart: int = 20, x=None):
        """Solve with GMRES refinement in FP64 preconditioned by the stored factors (see
        mf_refine_gmres); returns (x, Arnoldi steps, relres)."""
        import torch
        b2 = b if b.dim() == 2 else b.reshape(-1, 1)
        nrhs = int(b2.shape[1])
        x = torch.empty_like(b2) if x is None else x.reshape(self.n, nrhs)
        its = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        check(_lib.load().mf_refine_gmres(
            self._h, _dev_ptr(K, "K", (self.n_elem, self.npe, self.npe)),
            _dev_ptr(b2, "b", (self.n, nrhs)), _dev_ptr(x, "x"), nrhs, float(tol), int(max_it),
            int(restart), ctypes.byref(its), ctypes.byref(rr), _stream()))
        return x.reshape(b.shape), int(its.value), float(rr.value)

    def factor_refine(self, K, b, precision: str = "fp64", tol: float = 1e-12, max_it: int = 30,
                      x=None):
        """factor(K, precision) then refine(K, b) in one call, the first forward sweep overlapped
        with the factorization (see mf_factor_refine); returns (x, corrections, relres)."""
        import torch
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        b2 = b if b.dim() == 2 else b.reshape(-1, 1)
        nrhs = int(b2.shape[1])
        x = torch.empty_like(b2) if x is None else x.reshape(self.n, nrhs)
        its = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        self.factor_version += 1
        check(_lib.load().mf_factor_refine(
            self._h, _dev_ptr(K, "K", (self.n_elem, self.npe, self.npe)), PRECISIONS[precision],
            _dev_ptr(b2, "b", (self.n, nrhs)), _dev_ptr(x, "x"), nrhs, float(tol), int(max_it),
            ctypes.byref(its), ctypes.byref(rr), _stream()))
        return x.reshape(b.shape), int(its.value), float(rr.value)

    def elem_grad(self, lam, u):
        import torch
        lam2 = lam if lam.dim() == 2 else lam.reshape(-1, 1)
        nrhs = int(lam2.shape[1])
        gK = torch.empty((self.n_elem, self.npe, self.npe), dtype=torch.float64, device=lam.device)
        check(_lib.load().mf_elem_grad(self._h, _dev_ptr(lam2, "lam", (self.n, nrhs)),
                                       _dev_ptr(u.reshape(self.n, nrhs), "u"), nrhs,
                                       _dev_ptr(gK, "gK"), _stream()))
        return gK

    def profile(self, enable: bool = True):
        """Start (clearing counters) or stop per-launch event timing of this plan's kernels."""
        check(_lib.load().mf_profile(self._h, int(bool(enable))))

    def profile_report(self) -> dict:
        import json
        lib = _lib.load()
        need = ctypes.c_int64(0)
        check(lib.mf_profile_report(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(int(need.value) + 16)
        check(lib.mf_profile_report(self._h, buf, len(buf), ctypes.byref(need)))
        return json.loads(buf.value.decode())

    def export_factors(self):
        """Per-front (L (m x k), U (k x m)) numpy arrays, fronts in id order."""
        tot = int(self.info["sum_mk"])
        L = np.empty(max(tot, 1))
        U = np.empty(max(tot, 1))
        check(_lib.load().mf_export_factors(self._h, ctypes.c_void_p(L.ctypes.data),
                                            ctypes.c_void_p(U.ctypes.data)))
        t = self.export_tree()
        ms = np.diff(t["front_ptr"])
        ks = t["npiv"]
        Ls, Us, off = [], [], 0
        for m, k in zip(ms, ks):
            m, k = int(m), int(k)
            Ls.append(L[off:off + m * k].reshape(m, k))
            Us.append(U[off:off + m * k].reshape(k, m))
            off += m * k
        return Ls, Us


def analyse(meshes) -> Plan:
    return Plan(meshes)
