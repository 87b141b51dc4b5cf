// api_core.hpp -- host side of libmf: the device plan (uploaded once per plan), algorithmic
// cost model per launch, optional per-launch event timing, hipGraph capture of the per-class
// launch sequences, and the launch schedules of the factor and the solve.
//
// Scheduling (Sec. 3.3): Foata classes are executed in order, and all fronts of one class are
// independent tasks.  Each class is a handful of launches over the class's front lists (the
// bag of tasks); stream order is the barrier between classes.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mf.h"
#include "common.hpp"
#include "class_kernels.hpp"
#include "factor_kernels.hpp"
#include "trace.hpp"
#include "plan.hpp"
#include "solve_kernels.hpp"

namespace mfapi {

extern thread_local std::string g_err;

inline int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::mfapi::fail(MF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

enum Kind {
  K_TINY, K_SMALL, K_ASSEMBLE, K_FUSED, K_TRSM, K_GEMM_PANEL, K_GEMM_SCHUR,
  K_DOWN_WAVE, K_DOWN_BLOCK, K_UP_WAVE, K_UP_BLOCK, K_DOWN_RECT, K_UP_RECT, K_RESIDUAL,
  K_DIAG_INV, K_CLASS, K_PANEL_LA, K_SUB_FACTOR, K_SUB_DOWN, K_SUB_UP, K_CHUNK_STAGE, K_CHUNK,
  K_OTHER, K_COUNT
};
static const char *const kKindName[K_COUNT] = {
    "factor_tiny", "factor_small", "assemble", "front_panels", "panel_lu_trsm", "gemm_panel",
    "gemm_schur", "solve_down_wave", "solve_down_block", "solve_up_wave", "solve_up_block",
    "solve_down_rect", "solve_up_rect", "residual", "diag_block_inverse", "class_tiled",
    "panel_lookahead", "factor_subtree", "solve_down_subtree", "solve_up_subtree",
    "solve_chunk_stage", "solve_chunk", "other"};

// Algorithmic traffic and work of one launch (bytes that must cross HBM at least once, flops
// of the method's own operation count).
struct Cost {
  double bytes = 0, flops = 0;
};

struct StepDev {
  int64_t prec = 0, n = 0;         // panel records (d_panel) of the step's fronts
  int64_t update = 0, n_update = 0;
  int64_t trsm_items = 0;
  // look-ahead form: the previous panel's update tiles beyond this panel (d_tasks), and the
  // chunks per front of the panel part (the widest front's)
  int64_t prev_update = 0, n_prev_update = 0;
  int32_t la_chunks = 0;
  Cost trsm, upd;
};

struct LevelDev {
  int64_t tiny = 0, n_tiny = 0;
  int32_t tiny_max_m = 0;
  int64_t small = 0, n_small = 0;
  int32_t small_max_m = 0;
  int64_t large = 0, n_large = 0;
  int32_t large_max_m = 0;
  int64_t fused = 0, n_fused = 0;
  int32_t fused_max_m = 0;
  int64_t all = 0, n_all = 0;
  int64_t rall = 0;            // first wave record of the class (records follow `all`)
  int64_t rwup = 0, n_wup = 0; // the class's fronts with pivots in the up sweep's wave records
  int32_t max_m = 0, max_k = 0;
  std::vector<StepDev> steps;
  int64_t schur = 0, n_schur = 0;
  Cost c_tiny, c_small, c_assemble, c_schur, c_fused;
  // persistent launch of the class's tiled fronts: its tasks in d_ctasks, its ticket counter
  int64_t ctask = 0, n_ctask = 0;
  int32_t tick = 0;
  Cost c_class;
  bool lookahead = false;      // panel steps in the look-ahead form
  // solves: fixed (coefficient) bytes, bytes and flops per right-hand side; for the block
  // route split into the triangle (pivot block) and the rectangular (contribution) part
  double down_coef = 0, down_rhs_bytes = 0, down_rhs_flops = 0;
  double up_coef = 0, up_rhs_bytes = 0, up_rhs_flops = 0;
  double tri_coef = 0, tri_down_rhs_bytes = 0, tri_up_rhs_bytes = 0, tri_down_flops = 0,
         tri_up_flops = 0;
  double rect_coef = 0, rect_down_rhs_bytes = 0, rect_up_rhs_bytes = 0, rect_flops = 0;
  // rectangular-part tasks (int4: the front's wave record, first row, rows, 0)
  int64_t rdown = 0, n_rdown = 0, rup = 0, n_rup = 0;
  bool split_down = false, split_up = false;   // rectangular part in its own launch
  // chunked triangle solves (no transposition): stage tasks and, per launch of each sweep,
  // (first, count) of its tasks in d_chunk
  bool chunked = false;
  int64_t cstage = 0, n_cstage = 0;
  std::vector<std::pair<int64_t, int64_t>> csteps_down, csteps_up;
  bool rect_q_down = false, rect_q_up = false; // ... in slabs of 16 rows (quarter form)
};

// Bottom subtrees of the first ncls classes run as one launch (see k_factor_subtree): the wave
// records unit after unit, class after class, and ptr[u * ncls + c] = first record of unit u's
// class c.  ncls = 0: the classes run one launch each.
struct SubtreeDev {
  int32_t ncls = 0;
  int64_t nsub = 0, nrec = 0;
  mf::WaveRec *d_rec = nullptr;
  int32_t *d_ptr = nullptr;
  int32_t max_m = 0, max_k = 0;
  Cost c_factor;                       // factor: the classes' tiny-route cost
  double down_coef = 0, down_rhs_bytes = 0, down_rhs_flops = 0;   // solves: the classes' sums
  double up_coef = 0, up_rhs_bytes = 0, up_rhs_flops = 0;
};

struct ProfRec {
  int kind;
  int cls;          // Foata class of the launch (-1: not a class's launch)
  hipEvent_t a, b;
  Cost cost;
};

struct Profiler {
  bool on = false;
  int cur_class = -1;     // class whose launches are being issued
  std::vector<ProfRec> recs;
  double ms[K_COUNT] = {0};
  double bytes[K_COUNT] = {0};
  double flops[K_COUNT] = {0};
  int64_t launches[K_COUNT] = {0};
};

struct GraphKey {
  const void *p0 = nullptr, *p1 = nullptr;
  int32_t a = -1, b = -1;
  bool operator==(const GraphKey &o) const { return p0 == o.p0 && p1 == o.p1 && a == o.a && b == o.b; }
};

struct Graph {
  hipGraphExec_t exec = nullptr;
  GraphKey key;
};

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

}  // namespace mfapi

struct mf_plan {
  mf::HostPlan hp;
  mf::Tuning tune;                  // schedule of every class without an entry of its own
  std::vector<mf::Tuning> ctune;    // per-class schedule (empty: `tune` for every class)
  std::vector<mf::Tuning> eff;      // the schedule in use, per class (set at upload)
  int device = -1;
  bool uploaded = false;     // schedule (front lists, GEMM tasks) on the device
  bool static_up = false;    // tree arrays and factor storage on the device
  bool factored = false;
  bool use_graphs = true;
  int max_shared = 65536;
  int n_cu = 256;             // compute units of the plan's device
  mf::FrontDesc *d_desc = nullptr;
  int32_t *d_front_idx = nullptr, *d_inv_l = nullptr, *d_inv_r = nullptr, *d_conn = nullptr;
  int64_t *d_nptr = nullptr;
  int32_t *d_nelem = nullptr;
  int32_t *d_lists = nullptr;
  mf::GemmTask *d_tasks = nullptr;
  int4 *d_rect = nullptr;
  int4 *d_chunk = nullptr;    // tasks of the chunked triangle solves
  int32_t chunk_min_k = 512;  // classes with a front of at least this many pivots are chunked
  int64_t chunk_ws_rows = 0;  // workspace rows (after the contribution blocks' sum_c rows)
  mf::PanelRec *d_panel = nullptr;   // panel records of every step, class after class
  mf::WaveRec *d_wrec = nullptr;   // wave records of every class's front list, class after class
  mf::WaveRec *d_wrec_up = nullptr;   // the same without fronts that have no pivots (up sweep)
  double *d_store = nullptr;
  // inverses of the diagonal blocks of the fronts the block solves handle (see k_diag_inverse)
  double *d_dinv = nullptr;
  int64_t *d_dinv_off = nullptr;
  std::vector<int64_t> h_dinv_off;   // host copy (wave records carry it)
  int2 *d_dinv_tasks = nullptr;
  int64_t n_dinv_tasks = 0;
  mfapi::Cost c_dinv;
  int *d_status = nullptr;
  int *d_arrive = nullptr;    // [F] arrival counters of the panel steps
  // persistent class launches: task lists, and [classes] ticket counters followed by one
  // progress counter per tiled front, cleared at the start of every factorization
  mf::ClassTask *d_ctasks = nullptr;
  int *d_ccnt = nullptr;
  int64_t n_ccnt = 0;
  int class_blocks = 0;       // workgroups of a persistent class launch resident at once
  int64_t wait_ticks = 100000000;   // bound of a device-side wait (100 MHz clock ticks)
  int *h_status = nullptr;
  double *d_ycb = nullptr;
  size_t ycb_cap = 0;
  double *d_work = nullptr;
  size_t work_cap = 0;
  double *h_part = nullptr;   // mapped host memory of the final norms (k_norm_publish)
  double *d_hpart = nullptr;  // its device address
  int *d_hstatus = nullptr;   // device address of h_status (mapped host memory)
  int *d_pub_count = nullptr; // workgroups of k_norm_publish done (zero between launches)
  int pub_seq = 0;            // sequence number of the last k_norm_publish
  size_t part_cap = 0;
  double *d_kry = nullptr;    // Krylov workspace of mf_refine_gmres
  size_t kry_cap = 0;
  double *h_kry = nullptr;    // pinned host staging of its dot products and coefficients
  size_t hkry_cap = 0;
  std::vector<mfapi::LevelDev> lv;
  // bottom-subtree launches of the factorization and of the solves, and their settings: at most
  // sub_max_classes classes (-1: as many as the routes allow; off by default: the per-class
  // launches measured faster on the 2D and 3D workloads), units at least sub_min_units
  mfapi::SubtreeDev sub_f, sub_s;
  int32_t sub_max_classes = 0;
  int64_t sub_min_units = 2048;
  mfapi::Profiler prof;
  hipStream_t cap_stream = nullptr;
  // second stream of the overlapped factor + forward solve, and its per-class events
  hipStream_t side_stream = nullptr;
  std::vector<hipEvent_t> lvl_events;
  std::vector<int64_t> dinv_lvl;        // [classes + 1] first diagonal-inverse task per class
  mfapi::Graph g_factor[2], g_solve[4];   // small caches, least recently captured evicted
  int g_factor_next = 0, g_solve_next = 0;

  void drop_graphs() {
    for (auto &g : g_factor) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g = mfapi::Graph();
    }
    for (auto &g : g_solve) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g = mfapi::Graph();
    }
  }

  ~mf_plan() {
    drop_graphs();
    for (auto &r : prof.recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    for (hipEvent_t e : lvl_events) (void)hipEventDestroy(e);
    mfapi::dfree(d_desc);
    mfapi::dfree(d_front_idx);
    mfapi::dfree(d_inv_l);
    mfapi::dfree(d_inv_r);
    mfapi::dfree(d_conn);
    mfapi::dfree(d_nptr);
    mfapi::dfree(d_nelem);
    mfapi::dfree(d_lists);
    mfapi::dfree(d_tasks);
    mfapi::dfree(d_rect);
    mfapi::dfree(d_chunk);
    mfapi::dfree(d_wrec);
    mfapi::dfree(d_wrec_up);
    mfapi::dfree(sub_f.d_rec);
    mfapi::dfree(sub_f.d_ptr);
    mfapi::dfree(sub_s.d_rec);
    mfapi::dfree(sub_s.d_ptr);
    mfapi::dfree(d_panel);
    mfapi::dfree(d_store);
    mfapi::dfree(d_dinv);
    mfapi::dfree(d_dinv_off);
    mfapi::dfree(d_dinv_tasks);
    mfapi::dfree(d_status);
    mfapi::dfree(d_arrive);
    mfapi::dfree(d_ctasks);
    mfapi::dfree(d_ccnt);
    mfapi::dfree(d_ycb);
    mfapi::dfree(d_work);
    if (h_status) (void)hipHostFree(h_status);
    if (h_part) (void)hipHostFree(h_part);
    if (h_kry) (void)hipHostFree(h_kry);
    mfapi::dfree(d_kry);
    mfapi::dfree(d_pub_count);
  }
};
