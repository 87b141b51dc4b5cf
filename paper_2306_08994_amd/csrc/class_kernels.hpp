// class_kernels.hpp -- one persistent launch per Foata class for the fronts on the tiled route.
//
// Inside a class every front is an independent task (Sec. 3.3); inside a front the blocked
// elimination of Table 2 is a chain of phases: the extend-add, then per panel of 32 pivots the
// panel step (diagonal-block LU and the two triangular solves) and the trailing update of the
// fully summed rows and columns, then the Schur update C22 -= L21 U12.  The launch runs the
// class's task list -- extend-add strips, panel chunks, update tiles, Schur tiles, phase after
// phase -- with each task waiting only for the earlier phases of its own front, so fronts
// advance independently and a front's next panel starts as soon as its own update is done,
// instead of one launch (and one chip-wide barrier) per panel step and per kind of work.
//
// Ordering.  Each front has a progress counter: every task adds one when its results are
// stored, and a task of phase P waits until the counter holds the number of tasks of the
// front's phases before P (a count of the plan, `need`).  Workgroups take tasks in list order
// from a ticket counter, and the list is in phase order, so every task a workgroup waits for
// was taken earlier by a workgroup that is running: the launch cannot deadlock, whatever the
// number of workgroups resident at once.  Memory: the producer's stores complete (waitcnt),
// its workgroup synchronises, and one thread releases at device scope (the L2 of the producing
// XCD written back) before the counter increment; the consumer's waiting thread acquires at
// device scope (its L1 and L2 invalidated) before its workgroup's barrier.
//
// Every wait is bounded: after `wait_ticks` of the constant 100 MHz clock, or as soon as
// another workgroup gave up, the workgroup sets the abort word of the status block and
// leaves; every other wait sees the word and leaves too, so the launch always ends, and the
// host reports the abort as an error.
#pragma once

#include "factor_kernels.hpp"

namespace mf {

constexpr int kStatusAbort = 3;     // status word set when a device-side wait gave up
constexpr int kClassNB = 32;        // panel width of the persistent route

// LDS of the persistent launch: the union of the panel step's diagonal block, the GEMM
// staging (FP64 panel updates and the Schur update's precision) and the extend-add maps.
template <int PREC, int TILE>
constexpr size_t class_lds_bytes(int max_m) {
  size_t b = sizeof(double) * (kClassNB * (kClassNB + 1) + kClassNB);
  b = b > sizeof(GemmLds<0, TILE>) ? b : sizeof(GemmLds<0, TILE>);
  b = b > sizeof(GemmLds<PREC, TILE>) ? b : sizeof(GemmLds<PREC, TILE>);
  const size_t maps = (size_t)2 * max_m * sizeof(int);
  return b > maps ? b : maps;
}

// Waits (thread 0) until cnt reaches need; false if this or another workgroup gave up.  Bounded
// by the clock and, should the clock not advance, by the number of polls (each poll is two
// dependent memory round trips, well over 50 ticks).
__device__ inline bool class_wait(const int *cnt, int need, int *status, int64_t wait_ticks) {
  if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  const int64_t max_polls = 1000 + wait_ticks / 50;
  for (int64_t poll = 0;; ++poll) {
    __builtin_amdgcn_s_sleep(1);
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
    if (__hip_atomic_load(status + kStatusAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
    if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > wait_ticks || poll > max_polls) {
      __hip_atomic_store(status + kStatusAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}

template <int PREC, int TILE>
__global__ void __launch_bounds__(256)
k_class_tiled(const ClassTask *__restrict__ tasks, int ntasks, int *__restrict__ tick,
              int *__restrict__ cnt, const WaveRec *__restrict__ wrec, double *__restrict__ store,
              const int32_t *__restrict__ inv_l, const int32_t *__restrict__ inv_r,
              const double *__restrict__ K, int *__restrict__ status, int64_t wait_ticks) {
  extern __shared__ double smem[];
  __shared__ int s_task, s_go, s_prev;
  double(*D)[kClassNB + 1] = reinterpret_cast<double(*)[kClassNB + 1]>(smem);
  double *rd = smem + kClassNB * (kClassNB + 1);
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) s_task = __hip_atomic_fetch_add(tick, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int t = s_task;
    if (t >= ntasks) return;                       // uniform
    const ClassTask tk = tasks[t];
    if (tid == 0) {
      s_go = class_wait(cnt + tk.ci, tk.need, status, wait_ticks);
      // the front's earlier stores, released at device scope by their producers, are visible
      // to this workgroup's loads after the barrier
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!s_go) return;                             // uniform: the launch is being abandoned
    PanelRec pr;
    if (tk.type == kTaskAssemble) {
      assemble_rows(wrec[tk.a], tk.b, tk.c, store, inv_l, inv_r, K, reinterpret_cast<int *>(smem));
    } else if (tk.type == kTaskPanel) {
      pr.store = tk.store;
      pr.m = tk.m;
      pr.k = tk.k;
      pr.p0 = tk.a;
      pr.f = tk.f;
      panel_chunk<kClassNB>(pr, tk.b, store, status, D, rd, tk.c == 1);
    } else {
      GemmTask g;
      g.store = tk.store;
      g.ld = tk.m;
      g.i0 = tk.a;
      g.i1 = tk.b;
      g.j0 = tk.c;
      g.j1 = tk.d;
      g.q0 = tk.e;
      g.q1 = tk.g;
      g.front = tk.f;
      if (tk.type == kTaskSchur)
        gemm_tile<PREC, TILE>(g, store, *reinterpret_cast<GemmLds<PREC, TILE> *>(smem));
      else
        gemm_tile<0, TILE>(g, store, *reinterpret_cast<GemmLds<0, TILE> *>(smem));
    }
    // every thread's stores complete, then one release at device scope and the count
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      // the L2 write-back the release issues must be complete before the count is raised: the
      // wait the fence carries is dropped by the compiler when no other memory operation is
      // outstanding here (every store was waited for above), which let a consumer on another
      // XCD see the count before the producer's results reached memory
      __builtin_amdgcn_s_waitcnt(0);
      s_prev = __hip_atomic_fetch_add(cnt + tk.ci, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // the last chunk of a panel step stores the factored diagonal block, which every chunk
    // read as input (no task of this launch reads it afterwards: the step's update and the
    // later steps work on other blocks)
    if (tk.type == kTaskPanel && tk.c > 1 && s_prev == tk.need + tk.c - 1 && tid < 64)
      store_diag_block<kClassNB>(pr, store, D, tid);
  }
}

}  // namespace mf
