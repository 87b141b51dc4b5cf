#!/usr/bin/env python3
"""Benchmark of the multifrontal factor + solve on one MI355X.

Workload of one step: the 2D Q1 reaction-diffusion system on a 256 x 256 element grid (66,049
unknowns, 131,071 fronts, 17 Foata classes), element coefficients lognormal(0, 1), 8
right-hand sides N(0, 1), seed 2.  A step is one FP64 factorization (extend-add, partial LU,
Schur update, class by class) followed by the solve (forward and backward sweeps) and the FP64
residual check, with refinement corrections applied only if the relative residual exceeds
1e-12.  Inputs are resident in HBM before the timed region.

value = algorithmic factor+solve GFLOP/s = (factor flops + nrhs * solve flops per RHS) / step
time, with the operation counts of the method itself (division, multiplication and
subtraction tasks), not dense n^3.

Extra fields: per-kernel event timing of the same step (roofline of the dominant kernel),
the batched and mixed-precision variants, the L2 projection with linear, quadratic and cubic
bases at 299,209 unknowns, and the CPU oracle on the host (cpu_baseline).
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFS = 78.6           # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFS = 157.3
BF16_PEAK_TFS = 2500.0


def _sync():
    import torch
    torch.cuda.synchronize()


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    _sync()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    out = None
    for _ in range(steps):
        out = fn()
    ev1.record()
    _sync()
    wall = (time.perf_counter() - t0) / steps
    return wall, ev0.elapsed_time(ev1) / 1e3 / steps, out


# Source file of each profiled kernel kind (a measured HBM traffic figure is used only while
# the kernel's source is unchanged since the counters were taken).
KIND_SOURCE = {
    "factor_tiny": "factor_kernels.hpp", "factor_small": "factor_kernels.hpp",
    "assemble": "factor_kernels.hpp", "front_panels": "panel_kernels.hpp",
    "panel_lu_trsm": "panel_kernels.hpp", "gemm_panel": "factor_kernels.hpp",
    "gemm_schur": "factor_kernels.hpp", "solve_down_wave": "solve_kernels.hpp",
    "solve_down_block": "solve_kernels.hpp", "solve_up_wave": "solve_kernels.hpp",
    "solve_up_block": "solve_kernels.hpp", "diag_block_inverse": "solve_kernels.hpp",
    "panel_lookahead": "factor_kernels.hpp", "class_tiled": "class_kernels.hpp",
    "factor_subtree": "factor_kernels.hpp", "solve_down_subtree": "solve_kernels.hpp",
    "solve_up_subtree": "solve_kernels.hpp", "solve_chunk": "solve_kernels.hpp",
    "solve_chunk_stage": "solve_kernels.hpp",
}
TRAFFIC_TAG = re.compile(r"<!-- traffic kind=(\S+) source=(\S+) sha256=([0-9a-f]{64}) "
                         r"bytes_per_launch=([0-9.eE+]+) -->")


def measured_traffic(kind):
    """HBM bytes per launch of `kind` from a committed counter summary under profiles/, if the
    kernel's source still hashes to what it was when the counters were taken; else None."""
    src = KIND_SOURCE.get(kind)
    pdir = os.path.join(ROOT, "profiles")
    if not src or not os.path.isdir(pdir):
        return None
    path = os.path.join(ROOT, "paper_2306_08994_amd", "csrc", src)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        for m in TRAFFIC_TAG.finditer(open(os.path.join(pdir, name)).read()):
            if m.group(1) == kind and m.group(2) == src and m.group(3) == digest:
                return float(m.group(4))
    return None


def roofline_of(report):
    """Dominant kernel (largest summed event time) and its achieved fraction of peak."""
    ks = report["kernels"]
    top = max(ks, key=lambda k: k["ms"])
    sec = top["ms"] / 1e3
    traffic = measured_traffic(top["name"])
    if top["name"].startswith("gemm"):
        ach = top["flops"] / sec / 1e12
        return top, {"bound": "mfma", "achieved": ach, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": ach / FP64_PEAK_TFS, "traffic": traffic}
    ach = top["bytes"] / sec / 1e9
    return top, {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": ach / HBM_PEAK_GBS, "traffic": traffic}


CPU_SNIPPET = r"""
import json, sys, time
sys.path.insert(0, %(root)r)
import numpy as np
from fixtures import config_problem
from oracle.tree import build_tree, front_flops
from oracle.factor import factor, global_connectivity
from oracle.solve import solve
from oracle.residual import relres
p = config_problem(2)
tree = build_tree(p.meshes)
conn = global_connectivity(p)
fac_f, sol_f, _ = front_flops(tree)
times = []
for _ in range(%(runs)d):
    t0 = time.perf_counter()
    fac = factor(tree, p.K, conn)
    x = solve(tree, fac, p.b)
    times.append(time.perf_counter() - t0)
t = sorted(times)[len(times) // 2]
print(json.dumps({"sec": t, "flops": fac_f + p.nrhs * sol_f, "relres": relres(p.K, conn, x, p.b)}))
"""


def cpu_baseline(runs=3):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = CPU_SNIPPET % {"root": ROOT, "runs": runs}
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    if res.returncode != 0:
        return {"error": res.stderr[-400:]}
    r = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": r["flops"] / r["sec"] / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"the full step workload (256x256 Q1, 8 RHS): oracle factor + solve, median of "
                      f"{runs} runs, single thread (OMP/OPENBLAS/MKL_NUM_THREADS=1)",
            "ms_per_system": r["sec"] * 1e3, "relres": r["relres"], "host_cpu": host_cpu(),
            "host_nproc": os.cpu_count()}


def host_cpu():
    """The host processor as lscpu names it (model name, family / model / stepping, sockets,
    cores, threads, clock), with /proc/cpuinfo as the fallback."""
    out = {}
    try:
        res = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30)
        for line in res.stdout.splitlines():
            if ":" not in line:
                continue
            k, v = (t.strip() for t in line.split(":", 1))
            if k in ("Model name", "CPU family", "Model", "Stepping", "Socket(s)",
                     "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz",
                     "Hypervisor vendor", "L3 cache"):
                out[k] = v
    except (OSError, subprocess.SubprocessError):
        pass
    if "Model name" not in out:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    out["Model name"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return out


ORACLE_SOLVE_SNIPPET = r"""
import json, sys, time
sys.path.insert(0, %(root)r)
import numpy as np
from fixtures import config_problem
from oracle.tree import build_tree, front_flops
from oracle.factor import factor, global_connectivity
from oracle.solve import solve
from oracle.residual import relres
p = config_problem(%(cfg)d)
tree = build_tree(p.meshes)
conn = global_connectivity(p)
fac_f, sol_f, _ = front_flops(tree)
t0 = time.perf_counter()
fac = factor(tree, p.K, conn)
t1 = time.perf_counter()
x = solve(tree, fac, p.b)
t2 = time.perf_counter()
np.save(%(out)r, x)
print(json.dumps({"sec_factor": t1 - t0, "sec_solve": t2 - t1, "flops": fac_f + p.nrhs * sol_f,
                  "relres": relres(p.K, conn, x, p.b)}))
"""


def oracle_solution(cfg):
    """The oracle's solution of workload `cfg`, computed once on one host thread, and the time
    it took: (x, summary) or (None, {"error": ...})."""
    import tempfile
    import numpy as np
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "x.npy")
        code = ORACLE_SOLVE_SNIPPET % {"root": ROOT, "cfg": cfg, "out": path}
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                             text=True, timeout=900)
        if res.returncode != 0:
            return None, {"error": res.stderr[-400:]}
        r = json.loads(res.stdout.strip().splitlines()[-1])
        x = np.load(path)
    sec = r["sec_factor"] + r["sec_solve"]
    return x, {"value": r["flops"] / sec / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": "one run of the oracle's factor + solve of this workload, single thread",
               "ms_per_system": sec * 1e3, "ms_factor": r["sec_factor"] * 1e3,
               "relres": r["relres"]}


def err_vs(x, xo):
    """max over right-hand sides of ||x - x_O||_2 / ||x_O||_2 (x a device tensor)."""
    import numpy as np
    xh = x.detach().cpu().numpy().reshape(xo.shape[0], -1)
    xo2 = xo.reshape(xo.shape[0], -1)
    return float(np.max(np.linalg.norm(xh - xo2, axis=0) / np.linalg.norm(xo2, axis=0)))


PEAK_TFS = {"fp64": FP64_PEAK_TFS, "fp32": FP32_PEAK_TFS, "bf16": BF16_PEAK_TFS}


def schur_roofline(plan, step, prec):
    """The Schur-complement GEMM launches of one step timed with events: algorithmic flops
    (2 k c^2 per front) over their summed duration, against the MFMA peak of the precision
    they run in."""
    plan.profile(True)
    step()
    _sync()
    rep = plan.profile_report()
    plan.profile(False)
    k = next((k for k in rep["kernels"] if k["name"] == "gemm_schur"), None)
    if k is None:
        return None
    ach = k["flops"] / (k["ms"] / 1e3) / 1e12
    peak = PEAK_TFS[prec]
    return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
            "launches": k["launches"], "ms_per_step": k["ms"],
            "flops_per_launch": k["flops"] / k["launches"],
            "bytes_per_launch": k["bytes"] / k["launches"],
            "attainable_tfs": min(peak, k["flops"] / k["bytes"] * HBM_PEAK_GBS / 1e3)}


CPU_POOL_SNIPPET = r"""
import json, os, sys, time
sys.path.insert(0, %(root)r)
import multiprocessing as mp
import numpy as np
from fixtures import config_problem
from fixtures.mesh import Problem
from oracle.tree import build_tree, front_flops
from oracle.factor import factor, global_connectivity
from oracle.solve import solve
P = config_problem(4)
NO, EO = P.node_offsets, P.elem_offsets

def one(i):
    sub = Problem(P.name, [P.meshes[i]], P.K[EO[i]:EO[i + 1]], P.b[NO[i]:NO[i + 1]],
                  P.coef[EO[i]:EO[i + 1]], [P.S[i]], [P.M[i]])
    tree = build_tree(sub.meshes)
    conn = global_connectivity(sub)
    fac_f, sol_f, _ = front_flops(tree)
    fac = factor(tree, sub.K, conn)
    x = solve(tree, fac, sub.b)
    return fac_f + sub.nrhs * sol_f, x

if __name__ == "__main__":
    workers = %(workers)d
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        res = pool.map(one, range(len(P.meshes)), chunksize=1)
        wall = time.perf_counter() - t0
    np.save(%(out)r, np.concatenate([r[1] for r in res]))
    print(json.dumps({"sec": wall, "flops": sum(r[0] for r in res), "systems": len(P.meshes),
                      "workers": workers}))
"""


def cpu_pool_baseline(workers=16):
    """The 256-mesh batch on the host: the oracle (factor + solve) one mesh per task over a
    process pool of `workers` single-threaded processes; wall clock of the whole batch.
    Returns (the oracle's solution of the batch, summary)."""
    import tempfile
    import numpy as np
    workers = max(1, min(workers, os.cpu_count() or 1))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "x.npy")
        code = CPU_POOL_SNIPPET % {"root": ROOT, "workers": workers, "out": path}
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                             text=True, timeout=900)
        if res.returncode != 0:
            return None, {"error": res.stderr[-400:]}
        r = json.loads(res.stdout.strip().splitlines()[-1])
        x = np.load(path)
    return x, {"value": r["flops"] / r["sec"] / 1e9, "unit": "GFLOP/s", "cores": r["workers"],
               "kind": "oracle",
               "sample": f"the whole batch ({r['systems']} meshes): oracle factor + solve, one "
                         f"mesh per task over {r['workers']} single-threaded processes, wall clock",
               "ms_per_batch": r["sec"] * 1e3}


def tuning_arg(sched):
    """The --tuning value that reproduces a chosen schedule (one group per class if per-class)."""
    def grp(c):
        return ",".join(str(int(c[k])) for k in ("tile", "fused_max_m", "nb", "small_max_m",
                                                 "persistent"))
    if sched.get("mode") == "per_class" and sched.get("classes"):
        return ";".join(grp(c) for c in sched["classes"])
    return grp(sched)


def schedule(plan, K, prec, tuning):
    """The schedule of a run: `tuning` (tile,fused_max_m,nb,small_max_m) if given, else the
    autotuner's choice on this workload and precision; with its --tuning form."""
    sched = given_schedule(plan, tuning) if tuning else plan.autotune(K, prec, reps=2)["chosen"]
    return dict(sched, tuning_arg=tuning_arg(sched))


SUBTREE = None     # --subtree: (max_classes, min_units) of the bottom-subtree launches
CHUNKED = None     # --chunked: min_pivots of the chunked triangle solves


def new_plan(meshes):
    """A plan of the meshes, with the --subtree setting if one was given."""
    from paper_2306_08994_amd import Plan
    plan = Plan(meshes)
    if SUBTREE is not None:
        plan.set_subtree_launch(*SUBTREE)
    if CHUNKED is not None:
        plan.set_chunked_solve(CHUNKED)
    return plan


def given_schedule(plan, tuning):
    """tile,fused_max_m,nb,small_max_m[,persistent] (fused_max_m 0: fused route off;
    persistent 1 / 0: persistent class launches on / off, default on); several such groups
    separated by ';' give one schedule per Foata class, leaves first (the form of the
    autotuner's per-class choice, e.g. to profile exactly that schedule)."""
    groups = [g for g in tuning.split(";") if g.strip()]

    def parse(g):
        v = [int(x) for x in g.split(",")]
        t_, f_, nb_, sm_ = v[:4]
        pers = v[4] if len(v) > 4 else 1
        return {"persistent": pers, "tile": t_, "fused_max_m": f_, "nb": nb_, "small_max_m": sm_}

    if len(groups) > 1:
        cls = [parse(g) for g in groups]
        if len(cls) != plan.info["height"] + 1:
            raise SystemExit(f"--tuning has {len(cls)} class groups, the plan has "
                             f"{plan.info['height'] + 1} Foata classes")
        plan.set_class_tuning([dict(c, persistent=1 if c["persistent"] else 0) for c in cls])
        return {"mode": "per_class", "classes": cls, "given": True}
    c = parse(groups[0])
    plan.set_tuning(c["small_max_m"], c["nb"], c["fused_max_m"] if c["fused_max_m"] > 0 else -1,
                    c["tile"], 1 if c["persistent"] else -1)
    return dict(c, given=True)


def variant_mixed(steps, warmup, precs=("fp64", "fp32", "bf16"), tuning=None, oracle=True):
    """3D Q1 32^3 (35,937 unknowns): FP64 vs FP32- and BF16-Schur factorizations, each refined
    in FP64 to a relative residual <= 1e-12; the error of each against the oracle's solution
    (computed once on the host, timed: the oracle leg of this workload) and against the GPU's
    FP64 solution; the Schur GEMMs' fraction of their precision's MFMA peak."""
    import torch
    from fixtures import config_problem
    xo, oleg = oracle_solution(3) if oracle else (None, None)
    p = config_problem(3)
    plan = new_plan(p.meshes)
    K = torch.from_numpy(p.K).cuda()
    b = torch.from_numpy(p.b).cuda()
    x = torch.empty_like(b)
    flops = plan.info["factor_flops"] + p.nrhs * plan.info["solve_flops_per_rhs"]
    out = {"workload": "3D Q1 32x32x32 reaction-diffusion, k~lognormal(0,1), 1 RHS",
           "n": plan.n, "max_front": plan.info["max_m"]}
    ref = None
    for prec in precs:
        out.setdefault("schedule", {})[prec] = schedule(plan, K, prec, tuning)

        def step():
            return plan.factor_refine(K, b, prec, tol=1e-12, max_it=60, x=x)
        wall, dev, (xs, its, rr) = time_steps(step, steps, warmup)
        xs = xs.clone()
        if ref is None:
            ref = xs
        err = float(torch.linalg.norm(xs - ref) / torch.linalg.norm(ref))
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.factor(K, prec)
        _sync()
        tf = (time.perf_counter() - t0) / steps
        out[prec] = {"ms_per_system": wall * 1e3, "ms_factor": tf * 1e3,
                     "gflops": flops / wall / 1e9, "refine_corrections": its, "relres": rr,
                     "err_vs_oracle": None if xo is None else err_vs(xs, xo),
                     "err_vs_fp64": err, "roofline_schur": schur_roofline(plan, step, prec)}
        if prec != "fp64":
            # the same factorization refined by GMRES (FP64, preconditioned by the factors)
            def step_gmres():
                plan.factor(K, prec)
                return plan.refine_gmres(K, b, tol=1e-12, max_it=60, restart=20, x=x)
            gw, _, (xg, gits, grr) = time_steps(step_gmres, steps, warmup)
            out[prec]["gmres"] = {"ms_per_system": gw * 1e3, "gflops": flops / gw / 1e9,
                                  "arnoldi_steps": gits, "relres": grr,
                                  "err_vs_oracle": None if xo is None else err_vs(xg, xo)}
    if oleg is not None:
        out["cpu_oracle"] = oleg
    if "fp64" in out:
        for prec in precs:
            if prec in out and prec != "fp64":
                out[prec]["speedup_vs_fp64"] = out["fp64"]["ms_per_system"] / out[prec]["ms_per_system"]
                out[prec]["factor_speedup_vs_fp64"] = out["fp64"]["ms_factor"] / out[prec]["ms_factor"]
    return out


def variant_l2(steps, warmup):
    """The paper's own benchmark axis (Sec. 5): the L2 projection M u = b with linear, quadratic
    and cubic bases on a 547 x 547 node lattice (299,209 unknowns, the paper's 3e5 limit), one
    load vector; step = factor + solve + FP64 refinement to relres <= 1e-12."""
    import torch
    from fixtures import l2_workload
    out = {"workload": "2D L2 projection (mass matrix), 299,209 unknowns, 1 RHS, FP64"}
    for deg in (1, 2, 3):
        p = l2_workload(deg)
        plan = new_plan(p.meshes)
        K = torch.from_numpy(p.K).cuda()
        b = torch.from_numpy(p.b).cuda()
        x = torch.empty_like(b)
        inf = plan.info
        flops = inf["factor_flops"] + p.nrhs * inf["solve_flops_per_rhs"]
        sched = plan.autotune(K, reps=2)["chosen"]

        def step():
            return plan.factor_refine(K, b, tol=1e-12, max_it=5, x=x)
        wall, dev, (_, its, rr) = time_steps(step, steps, warmup)
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.factor(K)
        _sync()
        tf = (time.perf_counter() - t0) / steps
        out[f"p{deg}"] = {"elements": list(p.meshes[0].shape), "fronts": inf["n_fronts"],
                          "max_front": inf["max_m"], "factor_flops": inf["factor_flops"],
                          "ms_per_system": wall * 1e3, "ms_factor": tf * 1e3,
                          "gflops": flops / wall / 1e9, "refine_corrections": its,
                          "relres": rr, "schedule": sched}
    return out


def variant_table3(steps, warmup):
    """The 256 x 256 workload with the connectivity-only tree of Table 3 (element fronts sorted
    by lowest node id, joined in adjacent pairs) instead of nested dissection: the same step,
    the tree's own operation count."""
    import torch
    from fixtures import config_problem
    p = config_problem(2)
    p.meshes[0].ijk = None
    plan = new_plan(p.meshes)
    K = torch.from_numpy(p.K).cuda()
    b = torch.from_numpy(p.b).cuda()
    x = torch.empty_like(b)
    inf = plan.info
    flops = inf["factor_flops"] + p.nrhs * inf["solve_flops_per_rhs"]
    sched = plan.autotune(K, reps=2)["chosen"]

    def step():

        return plan.factor_refine(K, b, tol=1e-12, max_it=5, x=x)
    wall, dev, (_, its, rr) = time_steps(step, steps, warmup)
    return {"workload": "2D Q1 256x256 reaction-diffusion, 8 RHS, FP64, tree of Table 3",
            "fronts": inf["n_fronts"], "classes": inf["height"] + 1, "max_front": inf["max_m"],
            "factor_flops": inf["factor_flops"], "ms_per_system": wall * 1e3,
            "gflops": flops / wall / 1e9, "refine_corrections": its, "relres": rr,
            "schedule": sched}


def variant_batched(steps, warmup, precs=("fp64", "fp32"), tuning=None, oracle=True):
    """256 independent 2D advection-diffusion meshes (sides 32..128) in one batch: every class
    of all meshes in one launch sequence; FP64 and FP32-Schur, refined to 1e-12.  The oracle
    solves the batch on the host (one mesh per task over a process pool, timed): the error of
    each variant against it, the whole batch's and the worst mesh's."""
    import numpy as np
    import torch
    from fixtures import config_problem
    xo, pool = cpu_pool_baseline() if oracle else (None, None)
    p = config_problem(4)
    plan = new_plan(p.meshes)
    K = torch.from_numpy(p.K).cuda()
    b = torch.from_numpy(p.b).cuda()
    x = torch.empty_like(b)
    flops = plan.info["factor_flops"] + p.nrhs * plan.info["solve_flops_per_rhs"]
    out = {"workload": "256 2D Q1 advection-diffusion meshes, sides U{32..128}, 1 RHS",
           "n": plan.n, "systems": len(p.meshes), "fronts": plan.info["n_fronts"]}
    ref = None
    for prec in precs:
        out.setdefault("schedule", {})[prec] = schedule(plan, K, prec, tuning)

        def step():
            return plan.factor_refine(K, b, prec, tol=1e-12, max_it=30, x=x)
        wall, dev, (xs, its, rr) = time_steps(step, steps, warmup)
        xs = xs.clone()
        if ref is None:
            ref = xs
        err = float(torch.linalg.norm(xs - ref) / torch.linalg.norm(ref))
        worst = None
        if xo is not None:
            xh = xs.cpu().numpy()
            no = p.node_offsets
            worst = max(float(np.linalg.norm(xh[no[i]:no[i + 1]] - xo[no[i]:no[i + 1]]) /
                              np.linalg.norm(xo[no[i]:no[i + 1]])) for i in range(len(p.meshes)))
        out[prec] = {"ms_per_batch": wall * 1e3, "ms_per_system": wall * 1e3 / len(p.meshes),
                     "gflops": flops / wall / 1e9, "refine_corrections": its, "relres": rr,
                     "err_vs_oracle": None if xo is None else err_vs(xs, xo),
                     "err_vs_oracle_worst_mesh": worst,
                     "err_vs_fp64": err, "roofline_schur": schur_roofline(plan, step, prec)}
    if pool is not None:
        out["cpu_oracle_pool"] = pool
    out["one_mesh_at_a_time"] = unbatched(p, steps=3)
    if "fp64" in out:
        for prec in precs:
            if prec in out and prec != "fp64":
                out[prec]["speedup_vs_fp64"] = out["fp64"]["ms_per_batch"] / out[prec]["ms_per_batch"]
    return out


def unbatched(p, steps=3):
    """The same 256 meshes with one plan per mesh, factored and solved one after another (FP64,
    the same step and schedule defaults): what the batched class launches are compared with."""
    import torch
    NO, EO = p.node_offsets, p.elem_offsets
    plans = []
    for i in range(len(p.meshes)):
        plan = new_plan([p.meshes[i]])
        K = torch.from_numpy(p.K[EO[i]:EO[i + 1]]).cuda()
        b = torch.from_numpy(p.b[NO[i]:NO[i + 1]]).cuda()
        plans.append((plan, K, b, torch.empty_like(b)))

    def step():
        for plan, K, b, x in plans:
            plan.factor_refine(K, b, tol=1e-12, max_it=30, x=x)
    wall, _, _ = time_steps(step, steps, 1)
    return {"ms_per_batch": wall * 1e3, "ms_per_system": wall * 1e3 / len(plans),
            "note": "one plan per mesh, factor_refine called mesh after mesh (FP64)"}


def calibration_copies():
    """Device-to-device copies of known sizes (8 KiB .. 1 GiB, three each, in that order) after
    the measured launches: the HBM counters of a plain copy of each size calibrate the counter
    readings of kernels with few workgroups as well as of ones that fill the chip."""
    import torch
    sizes = [1 << 13, 1 << 16, 1 << 19, 1 << 23, 1 << 30]
    for nbytes in sizes:
        src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        _sync()
        for _ in range(3):
            dst.copy_(src)
        _sync()
        del src, dst
    return sizes


def pmc_probe_variant(variant, prec, tuning):
    """Counter runs of the 3D or the batched workload: the schedule (given or autotuned), one
    profiled factorization to count launches, three plain factorizations, then the calibration
    copies."""
    import torch
    from fixtures import config_problem
    p = config_problem(3 if variant == "mixed" else 4)
    plan = new_plan(p.meshes)
    K = torch.from_numpy(p.K).cuda()
    sched = schedule(plan, K, prec, tuning)
    plan.factor(K, prec)
    plan.profile(True)
    plan.factor(K, prec)
    _sync()
    per = {k["name"]: k["launches"] for k in plan.profile_report()["kernels"]}
    plan.profile(False)
    for _ in range(3):
        plan.factor(K, prec)
    _sync()
    return {"pmc_probe": True, "variant": variant, "precision": prec, "plain_factorizations": 3,
            "launches_per_factorization": per, "schedule": sched,
            "copy_bytes": calibration_copies()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help="tile,fused_max_m,nb,small_max_m[,persistent]: use this schedule instead "
                         "of autotuning (fused_max_m 0 = fused route off; persistent 0 = one launch "
                         "per panel step), e.g. for counter runs, where the "
                         "serialised dispatches distort the autotuner's timings")
    ap.add_argument("--variant", default="all",
                    choices=["all", "main", "mixed", "batched", "l2", "table3"],
                    help="run one workload only and print its JSON (main: the 256x256 step)")
    ap.add_argument("--precs", default=None,
                    help="comma-separated precisions of the mixed / batched variants")
    ap.add_argument("--subtree", default=None,
                    help="max_classes[,min_units] of the bottom-subtree launches (0: per-class "
                         "launches; default: the library's choice)")
    ap.add_argument("--chunked", type=int, default=None,
                    help="min_pivots of the chunked triangle solves (0: off; default: the "
                         "library's choice)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run a few steps and a 1 GiB device copy (HBM counter calibration) only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU subtree mapping is described in the design, not built)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from fixtures import config_problem
    global SUBTREE, CHUNKED
    CHUNKED = args.chunked
    if args.subtree:
        v = [int(x) for x in args.subtree.split(",")]
        SUBTREE = (v[0], v[1] if len(v) > 1 else 2048)

    if args.pmc_probe and args.variant in ("mixed", "batched"):
        print(json.dumps(pmc_probe_variant(args.variant, (args.precs or "fp64").split(",")[0],
                                           args.tuning)))
        return
    if args.variant in ("mixed", "batched", "l2", "table3"):
        kw = {}
        if args.variant in ("mixed", "batched"):
            kw["tuning"] = args.tuning
            kw["oracle"] = not args.no_cpu_baseline
            if args.precs:
                kw["precs"] = tuple(args.precs.split(","))
        fn = {"mixed": variant_mixed, "batched": variant_batched, "l2": variant_l2,
              "table3": variant_table3}[args.variant]
        print(json.dumps({"variant": args.variant, **fn(args.steps, args.warmup, **kw)}))
        return

    dev = torch.device("cuda:0")
    p = config_problem(2)
    t0 = time.perf_counter()
    plan = new_plan(p.meshes)
    t_analyse = time.perf_counter() - t0
    K = torch.from_numpy(p.K).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    x = torch.empty_like(b)
    info = plan.info
    nrhs = p.nrhs
    if args.tuning:
        tuned = {"chosen": given_schedule(plan, args.tuning)}
    else:
        tuned = plan.autotune(K, reps=3)      # schedule chosen on this workload, before timing
    tuned["chosen"]["tuning_arg"] = tuning_arg(tuned["chosen"])

    def step():
        # factorization, the first solve with its forward sweep overlapped, FP64 residual check
        return plan.factor_refine(K, b, tol=1e-12, max_it=5, x=x)

    def step_sequential():
        plan.factor(K)
        return plan.refine(K, b, tol=1e-12, max_it=5, x=x)

    if args.pmc_probe:
        # launches of each kernel kind in one step (a profiled step), then 3 plain steps: the
        # counters of a kind are read from its last 3 x launches dispatches
        plan.profile(True)
        step()
        per_step = {k["name"]: k["launches"] for k in plan.profile_report()["kernels"]}
        plan.profile(False)
        for _ in range(3):
            step()
        copies = calibration_copies()
        print(json.dumps({"pmc_probe": True, "copy_bytes": copies, "plain_steps": 3,
                          "launches_per_step": per_step, "schedule": tuned["chosen"]}))
        return
    t_step, t_dev, (_, its, rr) = time_steps(step, args.steps, args.warmup)
    t_seq, _, _ = time_steps(step_sequential, args.steps, 1)
    t_fac, _, _ = time_steps(lambda: plan.factor(K), args.steps, 1)
    t_sol, _, _ = time_steps(lambda: plan.solve(b, out=x), args.steps, 1)
    flops = info["factor_flops"] + nrhs * info["solve_flops_per_rhs"]

    # per-kernel event timing over the same steps (graphs off while profiling)
    plan.profile(True)
    for _ in range(args.steps):
        step()
    _sync()
    rep = plan.profile_report()
    plan.profile(False)
    top, roof = roofline_of(rep)
    factor_kinds = {"factor_tiny", "factor_small", "assemble", "front_panels", "panel_lu_trsm",
                    "gemm_panel", "gemm_schur", "class_tiled", "panel_lookahead", "factor_subtree"}
    launches = {"factor": sum(k["launches"] for k in rep["kernels"] if k["name"] in factor_kinds),
                "solve_and_inverses": sum(k["launches"] for k in rep["kernels"]
                                          if k["name"] not in factor_kinds)}
    launches = {k: v / args.steps for k, v in launches.items()}

    out = {
        "metric": "factor+solve GFLOP/s at relres<=1e-12 (FP64 multifrontal, 256x256 Q1, 8 RHS)",
        "value": flops / t_step / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D Q1 256x256 reaction-diffusion, k~lognormal(0,1), 8 RHS, FP64, seed 2",
                   "n": info["n"], "fronts": info["n_fronts"], "classes": info["height"] + 1,
                   "nrhs": nrhs, "global_batch": 1, "parallelism": "single GPU"},
        "ms_per_system": t_step * 1e3,
        "ms_factor_then_refine": t_seq * 1e3,
        "ms_factor": t_fac * 1e3, "ms_solve": t_sol * 1e3, "ms_analyse_host": t_analyse * 1e3,
        "relres": rr, "refine_corrections": its, "schedule": tuned["chosen"],
        "roofline": dict(roof, kernel=top["name"],
                         avg_launch_us=top["ms"] * 1e3 / top["launches"],
                         bytes_per_launch=top["bytes"] / top["launches"],
                         flops_per_launch=top["flops"] / top["launches"]),
        "kernels": rep["kernels"],
        "subtree_launch": plan.subtree_launch_info(),
        "launches_per_step": dict(launches, classes=info["height"] + 1,
                                  note="the plan's kernel launches per step; the residual, norm "
                                       "and status-clearing launches (4-5 per step) not included"),
    }
    if not args.no_variants and args.variant == "all":
        vs = args.steps
        out["mixed_precision_3d"] = variant_mixed(vs, 2, oracle=not args.no_cpu_baseline)
        out["batched_256_meshes"] = variant_batched(vs, 2, oracle=not args.no_cpu_baseline)
        out["l2_projection_p123"] = variant_l2(vs, 2)
        out["tree_of_table3"] = variant_table3(vs, 2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
