// plan.hpp -- host-side plan of the multifrontal solver: elimination tree, front index lists,
// extend-add maps, storage offsets and the per-class launch schedule.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mf {

// Per-front record shared by host and device (plain data, 48 bytes).
struct FrontDesc {
  int64_t store;   // offset (doubles) of the front's m x m row-major storage
  int64_t idx;     // offset into front_idx / inv_l / inv_r (prefix sum of m)
  int64_t cbrow;   // offset (rows) into a solve's contribution-block buffer (prefix sum of m-k)
  int32_t m, k;    // width and number of pivots
  int32_t left, right;  // child fronts, -1 for a leaf
  int32_t elem;    // element of a leaf, -1 otherwise
  int32_t level;   // Foata class
};
static_assert(sizeof(FrontDesc) == 48, "FrontDesc layout");

// Per-front record of the one-wave-per-front kernels (the tiny factor route and the wave
// solves), one per entry of a class's front list: everything the wave needs before its first
// gather, so that the record (uniform, scalar loads), then the maps and the sources in one
// round trip, are the whole dependency chain.  96 bytes.
struct WaveRec {
  int64_t store;    // offset (doubles) of the front's m x m storage
  int64_t idx;      // offset into front_idx / inv_l / inv_r
  int64_t cbrow;    // first row of the front's contribution block in a solve's CB buffer
  int64_t src[2];   // extend-add sources: >= 0 offset (doubles) into the store of a child's CB
                    // (its (k, k) entry); < 0: -1 - offset of an element matrix in K
  int64_t ycb[2];   // first CB-buffer row of each child that passes one to the solve, else -1
  int64_t dinv;     // offset of the front's diagonal-block inverses (block solves), else -1
  int32_t f;        // front id
  int32_t m, k;     // width and pivots
  int32_t ld[2];    // leading dimension of each source
  int32_t n[2];     // size of each (square) source, 0 = absent
  int32_t pad;
};
static_assert(sizeof(WaveRec) == 96, "WaveRec layout");

// One tile of a batched GEMM update  C[i0:i1, j0:j1] -= A[i0:i1, q0:q1] * B[q0:q1, j0:j1],
// where A, B and C are all views of the same front storage (row-major, leading dimension ld,
// at offset store), so that the task alone locates its operands.
struct GemmTask {
  int64_t store;
  int32_t ld;
  int32_t i0, i1, j0, j1;
  int32_t q0, q1;
  int32_t front;
};
static_assert(sizeof(GemmTask) == 40, "GemmTask layout");

// One front of a panel step of the tiled route: everything the panel kernel needs in one
// record.  24 bytes.
struct PanelRec {
  int64_t store;    // offset (doubles) of the front's storage
  int32_t m, k;     // width and pivots
  int32_t p0;       // first pivot of the panel
  int32_t f;        // front id
};
static_assert(sizeof(PanelRec) == 24, "PanelRec layout");

// One task of the persistent launch of a class's tiled fronts (see k_class_tiled): a strip of
// the extend-add, a chunk of a panel step, a tile of a panel's trailing update or a tile of the
// Schur update, with the value of its front's progress counter it must wait for.  56 bytes.
enum : int32_t { kTaskAssemble = 0, kTaskPanel = 1, kTaskUpdate = 2, kTaskSchur = 3 };
struct ClassTask {
  int64_t store;    // offset (doubles) of the front's storage
  int32_t type;     // kTask*
  int32_t f;        // front id
  int32_t ci;       // the front's progress counter
  int32_t need;     // counter value (tasks of the front's earlier phases) to wait for
  int32_t m, k;     // width and pivots
  // assemble: wave record, first row, end row; panel: first pivot, chunk, chunks of the step;
  // update / Schur tile: i0, i1, j0, j1, q0, q1 (as GemmTask)
  int32_t a, b, c, d, e, g;
};
static_assert(sizeof(ClassTask) == 56, "ClassTask layout");

// Work of one panel step of the tiled (HBM-resident) path inside one class.
struct PanelStep {
  std::vector<int32_t> fronts;     // fronts that still have pivots at this step
  std::vector<int32_t> p0;         // first pivot of the panel per front
  std::vector<GemmTask> update;    // trailing update restricted to the fully-summed region
  // look-ahead form (panel width 32): the previous panel's trailing update beyond this panel,
  // run by the same launch as this panel (which applies the previous panel's update to its own
  // rows and columns itself); `update` is then empty
  std::vector<GemmTask> prev_update;
  int64_t trsm_items = 0;          // max over fronts of the panel kernel's items (columns, rows)
};

struct LevelSchedule {
  std::vector<int32_t> tiny;       // fronts factored by one wave each, in LDS
  int32_t tiny_max_m = 0;
  std::vector<int32_t> small;      // fronts factored by one workgroup each, in LDS
  int32_t small_max_m = 0;
  std::vector<int32_t> large;      // fronts assembled and factored in HBM
  int32_t large_max_m = 0;
  std::vector<int32_t> fused;      // large fronts whose panels run in one workgroup
  int32_t fused_max_m = 0;
  std::vector<PanelStep> steps;    // panel steps of the large fronts that are not fused
  bool lookahead = false;          // steps in the look-ahead form (see PanelStep)
  std::vector<GemmTask> schur;     // C22 -= L21 U12 tiles of the large fronts
  std::vector<int32_t> all;        // every front of the class that the solve visits
  int32_t max_m = 0, max_k = 0;
};

struct HostPlan {
  int32_t n_mesh = 0, dim = 0, npe = 0;
  int64_t n = 0, n_elem = 0, F = 0;
  std::vector<int32_t> conn;       // [n_elem][npe] global node ids
  std::vector<int32_t> parent, level, npiv, width;
  std::vector<int64_t> leaf_elem;
  std::vector<int64_t> front_ptr;  // [F+1]
  std::vector<int32_t> front_idx;  // [sum m]
  std::vector<int32_t> inv_l, inv_r;  // [sum m] child CB position (leaf: local node in inv_l)
  std::vector<FrontDesc> desc;
  std::vector<int64_t> mesh_front_ptr, mesh_node_ptr;   // [n_mesh+1] first front / node of a mesh
  int32_t height = 0, max_m = 0, max_k = 0;
  int64_t store_doubles = 0, sum_c = 0, sum_mk = 0;
  double factor_flops = 0, solve_flops = 0, sum_cb2 = 0;
  std::vector<LevelSchedule> levels;
};

// Tunables of the schedule (chosen by the autotuner or defaults).
struct Tuning {
  int32_t tiny_max_m = 32;     // fronts up to this width are factored one per wave
  int32_t small_max_m = 128;   // fronts up to this width are factored in LDS
  int32_t nb = 32;             // panel width of the tiled path
  int32_t fused_max_m = 576;   // tiled fronts up to this width run all panels in one workgroup
  int32_t tile = 64;           // GEMM output tile edge
  int32_t persistent = 0;      // tiled fronts of a class in one persistent launch (panel width 32)
};

// Builds the tree and front structure; returns an error message or "" on success.
std::string analyse(int32_t n_mesh, const int32_t *dims, const int32_t *npes,
                    const int64_t *n_nodes, const int64_t *n_elem,
                    const int32_t *const *conns, const int32_t *const *ijks, HostPlan &out);

// (Re)builds the per-class schedule: class l routes and blocks its fronts by t[l] (t holds one
// entry per class, height + 1).
void build_schedule(HostPlan &p, const std::vector<Tuning> &t);

}  // namespace mf
