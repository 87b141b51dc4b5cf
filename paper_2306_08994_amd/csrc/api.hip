// api.hip -- C ABI of libmf (declared in include/mf.h).
#include "api_core.hpp"

#include <chrono>
#include <mutex>

namespace mfapi {

thread_local std::string g_err;

namespace {

template <typename T>
int upload(T *&dst, const std::vector<T> &src) {
  dfree(dst);
  const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  HIPCHK(hipMalloc((void **)&dst, bytes));
  if (!src.empty()) HIPCHK(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return MF_OK;
}

// -- cost model -----------------------------------------------------------------------------
double child_cb_entries(const mf::HostPlan &H, const mf::FrontDesc &d) {
  if (d.elem >= 0) return (double)H.npe * H.npe;
  double s = 0;
  for (int32_t c : {d.left, d.right}) {
    const mf::FrontDesc &x = H.desc[c];
    s += (x.elem >= 0 && x.k == 0) ? (double)H.npe * H.npe : (double)(x.m - x.k) * (x.m - x.k);
  }
  return s;
}

double elim_flops(int32_t m, int32_t k) {
  double f = 0;
  for (int32_t p = 0; p < k; ++p) {
    const double r = (double)(m - p);
    f += (r - 1) + 2 * (r - 1) * (r - 1);
  }
  return f;
}

Cost front_factor_cost(const mf::HostPlan &H, int32_t f) {
  const mf::FrontDesc &d = H.desc[f];
  const double cb = child_cb_entries(H, d);
  Cost c;
  c.bytes = 8.0 * (cb + (double)d.m * d.m);
  c.flops = elim_flops(d.m, d.k) + (d.elem >= 0 ? 0.0 : cb);
  return c;
}

// Length of the union of half-open intervals.
double union_length(std::vector<std::pair<int32_t, int32_t>> v) {
  std::sort(v.begin(), v.end());
  double len = 0;
  int32_t hi = INT32_MIN;
  for (const auto &iv : v) {
    const int32_t lo = std::max(iv.first, hi);
    if (iv.second > lo) len += iv.second - lo;
    hi = std::max(hi, iv.second);
  }
  return len;
}

// Algorithmic cost of a set of GEMM update tiles C -= A B: per front (and inner range), the
// output entries read and written once, and each operand row of A and column of B read once
// over the inner dimension -- not the operand re-reads of the tiling.
Cost gemm_cost(const std::vector<mf::GemmTask> &ts) {
  Cost c;
  std::unordered_map<int64_t, std::vector<size_t>> by_front;
  for (size_t i = 0; i < ts.size(); ++i) by_front[((int64_t)ts[i].front << 20) ^ ts[i].q0].push_back(i);
  for (const auto &kv : by_front) {
    std::vector<std::pair<int32_t, int32_t>> rows, cols;
    double out = 0, nq = 0;
    for (size_t i : kv.second) {
      const mf::GemmTask &t = ts[i];
      const double ni = t.i1 - t.i0, nj = t.j1 - t.j0;
      nq = t.q1 - t.q0;
      c.flops += 2 * ni * nj * nq;
      out += ni * nj;
      rows.emplace_back(t.i0, t.i1);
      cols.emplace_back(t.j0, t.j1);
    }
    c.bytes += 8 * (2 * out + (union_length(rows) + union_length(cols)) * nq);
  }
  return c;
}

void level_costs(const mf::HostPlan &H, const mf::LevelSchedule &S, LevelDev &D, int32_t nb) {
  for (int32_t f : S.tiny) {
    Cost c = front_factor_cost(H, f);
    D.c_tiny.bytes += c.bytes;
    D.c_tiny.flops += c.flops;
  }
  for (int32_t f : S.small) {
    Cost c = front_factor_cost(H, f);
    D.c_small.bytes += c.bytes;
    D.c_small.flops += c.flops;
  }
  for (int32_t f : S.large) {
    const mf::FrontDesc &d = H.desc[f];
    const double cb = child_cb_entries(H, d);
    D.c_assemble.bytes += 8.0 * (cb + (double)d.m * d.m);
    D.c_assemble.flops += cb;
  }
  for (int32_t f : S.fused) {
    // the fully summed rows and columns read and written once; flops of the pivots minus the
    // Schur product left to the GEMM
    const mf::FrontDesc &d = H.desc[f];
    const double m = d.m, k = d.k, c = m - k;
    D.c_fused.bytes += 16.0 * (m * k + k * c);
    D.c_fused.flops += elim_flops(d.m, d.k) - 2.0 * k * c * c;
  }
  for (size_t s = 0; s < S.steps.size(); ++s) {
    const mf::PanelStep &st = S.steps[s];
    StepDev &sd = D.steps[s];
    for (size_t i = 0; i < st.fronts.size(); ++i) {
      const mf::FrontDesc &d = H.desc[st.fronts[i]];
      const double pb = std::min(nb, d.k - st.p0[i]);
      const double rest = d.m - st.p0[i] - pb;
      sd.trsm.bytes += 8 * (2 * pb * pb + 4 * rest * pb);
      sd.trsm.flops += elim_flops((int32_t)pb, (int32_t)pb) + 2 * rest * pb * pb;
      if (S.lookahead && st.p0[i] > 0) {
        // the previous panel's update of this panel's rows and columns: its L and U entries
        // of them read once, 2 nb flops per entry of the panel's rows and columns
        sd.trsm.bytes += 8 * (nb * (2 * rest + 2 * pb));
        sd.trsm.flops += 2.0 * nb * pb * (2 * rest + pb);
      }
    }
    sd.upd = gemm_cost(S.lookahead ? st.prev_update : st.update);
  }
  D.c_schur = gemm_cost(S.schur);
  for (int32_t f : S.all) {
    const mf::FrontDesc &d = H.desc[f];
    const double m = d.m, k = d.k;
    double ch = 0;
    if (d.elem < 0)
      for (int32_t c : {d.left, d.right}) {
        const mf::FrontDesc &x = H.desc[c];
        if (!(x.elem >= 0 && x.k == 0)) ch += x.m - x.k;
      }
    const double c = m - k;
    D.down_coef += 8 * (m * k - k * (k - 1) / 2);
    D.down_rhs_bytes += 8 * (k + ch + (m - k) + k);
    D.up_coef += 8 * (m * k - k * (k - 1) / 2);
    if (d.k > 0) D.up_rhs_bytes += 8 * (m + k);   // a front without pivots has no up-sweep work
    for (int32_t p = 0; p < d.k; ++p) {
      D.down_rhs_flops += 1 + 2 * (m - p - 1);
      D.up_rhs_flops += 2 * (m - p - 1);
      D.tri_down_flops += 1 + 2 * (k - p - 1);
      D.tri_up_flops += 2 * (k - p - 1);
    }
    D.tri_coef += 8 * (k * (k + 1) / 2);
    D.tri_down_rhs_bytes += 8 * 3 * k;                 // b and child values in, y out
    D.tri_up_rhs_bytes += 8 * 2 * k;
    D.rect_coef += 8 * c * k;
    D.rect_down_rhs_bytes += 8 * (k + ch + c);         // y in, child values in, CB out
    D.rect_up_rhs_bytes += 8 * (c + 2 * k);
    D.rect_flops += 2 * c * k;
  }
}


// Appends the tiles of one GEMM launch in an order that keeps tiles sharing operands on one
// XCD.  Workgroups are dispatched to the 8 XCDs round robin (workgroup b on XCD b mod 8), each
// XCD with its own L2: a front's tile grid is cut into 8 blocks of tile rows x tile columns (2 x
// 4, 4 x 2, 1 x 8 or 8 x 1, the closest to square), one per XCD, so each XCD reads a half or a
// quarter of the front's L21 rows and U12 columns instead of all of them; a front of fewer than
// 32 tiles goes whole to the least loaded XCD.  Slot t of the launch (workgroup first + t) gets
// a tile of XCD (first + t) mod 8 while that XCD has tiles left.  Tiles of a launch are
// independent, so the order changes only where they run.
void append_xcd_ordered(std::vector<mf::GemmTask> &out, const std::vector<mf::GemmTask> &ts,
                        int64_t first) {
  constexpr int X = 8;
  if (ts.size() < 2 * X) {
    out.insert(out.end(), ts.begin(), ts.end());
    return;
  }
  std::vector<std::vector<size_t>> q(X);
  std::vector<int64_t> load(X, 0);
  size_t i = 0;
  while (i < ts.size()) {
    size_t j = i;
    while (j < ts.size() && ts[j].front == ts[i].front && ts[j].q0 == ts[i].q0) ++j;
    const size_t n = j - i;
    if (n < 32) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      for (size_t t = i; t < j; ++t) q[x].push_back(t);
      load[x] += (int64_t)n;
    } else {
      std::vector<int32_t> rows, cols;
      for (size_t t = i; t < j; ++t) {
        rows.push_back(ts[t].i0);
        cols.push_back(ts[t].j0);
      }
      std::sort(rows.begin(), rows.end());
      rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      // pa x pb = 8 blocks, pa (tile-row groups) chosen closest to square blocks
      int pa = 1;
      double best = 1e30;
      for (int a : {1, 2, 4, 8}) {
        const double r = ((double)rows.size() / a) / ((double)cols.size() / (X / a));
        const double dev = std::fabs(std::log(r));
        if (dev < best) {
          best = dev;
          pa = a;
        }
      }
      const int pb = X / pa;
      for (size_t t = i; t < j; ++t) {
        const int64_t ri = std::lower_bound(rows.begin(), rows.end(), ts[t].i0) - rows.begin();
        const int64_t ci = std::lower_bound(cols.begin(), cols.end(), ts[t].j0) - cols.begin();
        const int x = (int)(ri * pa / (int64_t)rows.size()) * pb + (int)(ci * pb / (int64_t)cols.size());
        q[x].push_back(t);
        ++load[x];
      }
    }
    i = j;
  }
  std::vector<size_t> head(X, 0);
  for (size_t t = 0; t < ts.size(); ++t) {
    int x = (int)((first + (int64_t)t) % X);
    if (head[x] == q[x].size()) {   // this XCD's tiles are used up: take from the fullest one
      size_t most = 0;
      for (int y = 0; y < X; ++y)
        if (q[y].size() - head[y] > most) {
          most = q[y].size() - head[y];
          x = y;
        }
    }
    out.push_back(ts[q[x][head[x]++]]);
  }
}

}  // namespace

// Classes with fewer rectangular-part slabs of 64 rows than this use slabs of 16 (quarter form).
constexpr int64_t kRectQuarterBelow = 256;

// Launches that put one front per grid row cap the rows here and take the rest grid-stride.
constexpr int64_t kMaxGridY = 65535;

// Fronts of a class whose widest front is above this take the workgroup-per-front block solves.
constexpr int kWaveSolveMaxM = 64;
// Largest (m - k) k of a class from which its rectangular part is a launch of its own.
constexpr int64_t kSplitDownCK = 16384, kSplitUpCK = 8192;

// Bottom subtrees of the first classes as one launch (see k_factor_subtree).  `eligible` is the
// number of leading classes whose every front takes the route the subtree kernels run (the
// tiny factor route, or the wave solves); of those, the most classes (at least two, at most
// P->sub_max_classes) that still give P->sub_min_units units, so that the launch fills the chip
// with units whose per-class front counts are small.  wpos[f]: front f's entry in `wrec`.
int build_subtrees(mf_plan *P, SubtreeDev &S, int32_t eligible,
                   const std::vector<mf::WaveRec> &wrec, const std::vector<int64_t> &wpos) {
  const mf::HostPlan &H = P->hp;
  dfree(S.d_rec);
  dfree(S.d_ptr);
  S = SubtreeDev();
  int32_t lim = eligible;
  if (P->sub_max_classes >= 0) lim = std::min(lim, P->sub_max_classes);
  // units of ncls classes: fronts with a record, class < ncls, parent at or above ncls
  auto is_root = [&](int64_t f, int32_t ncls) {
    if (wpos[f] < 0 || H.level[f] >= ncls) return false;
    const int32_t par = H.parent[f];
    return par < 0 || H.level[par] >= ncls;
  };
  int32_t ncls = 0;
  for (int32_t c = lim; c >= 2 && !ncls; --c) {
    int64_t units = 0;
    for (int64_t f = 0; f < H.F; ++f) units += is_root(f, c) ? 1 : 0;
    if (units >= P->sub_min_units) ncls = c;
  }
  if (!ncls) return MF_OK;
  std::vector<mf::WaveRec> rec;
  std::vector<int32_t> ptr;
  std::vector<std::vector<int32_t>> by_cls(ncls);
  std::vector<int32_t> stack;
  for (int64_t f = 0; f < H.F; ++f) {
    if (!is_root(f, ncls)) continue;
    for (auto &v : by_cls) v.clear();
    stack.assign(1, (int32_t)f);
    while (!stack.empty()) {
      const int32_t g = stack.back();
      stack.pop_back();
      if (wpos[g] >= 0) by_cls[H.level[g]].push_back(g);
      const mf::FrontDesc &d = H.desc[g];
      if (d.left >= 0) stack.push_back(d.left);
      if (d.right >= 0) stack.push_back(d.right);
    }
    for (int32_t c = 0; c < ncls; ++c) {
      ptr.push_back((int32_t)rec.size());
      for (int32_t g : by_cls[c]) rec.push_back(wrec[wpos[g]]);
    }
    ++S.nsub;
  }
  ptr.push_back((int32_t)rec.size());
  S.ncls = ncls;
  S.nrec = (int64_t)rec.size();
  for (int32_t c = 0; c < ncls; ++c) {
    const LevelDev &D = P->lv[c];
    S.max_m = std::max(S.max_m, D.max_m);
    S.max_k = std::max(S.max_k, D.max_k);
    S.c_factor.bytes += D.c_tiny.bytes;
    S.c_factor.flops += D.c_tiny.flops;
    S.down_coef += D.down_coef;
    S.down_rhs_bytes += D.down_rhs_bytes;
    S.down_rhs_flops += D.down_rhs_flops;
    S.up_coef += D.up_coef;
    S.up_rhs_bytes += D.up_rhs_bytes;
    S.up_rhs_flops += D.up_rhs_flops;
  }
  int rc;
  if ((rc = upload(S.d_rec, rec)) || (rc = upload(S.d_ptr, ptr))) return rc;
  return MF_OK;
}

int ensure_uploaded(mf_plan *P) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (P->uploaded) {
    if (dev != P->device)
      return fail(MF_EINVAL, "plan was uploaded to device " + std::to_string(P->device) +
                                 " but the current device is " + std::to_string(dev));
    return MF_OK;
  }
  P->drop_graphs();
  P->device = dev;
  HIPCHK(hipDeviceGetAttribute(&P->max_shared, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  HIPCHK(hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  mf::HostPlan &H = P->hp;
  // widest front whose padded square fits in one workgroup's LDS
  int32_t mm = 1;
  while (mf::small_lds_doubles(mm + 1) * 8 <= P->max_shared) ++mm;
  P->tune.small_max_m = std::min<int32_t>(P->tune.small_max_m, mm);
  // the schedule of each class: its own entry if the autotuner chose one, else the plan's
  P->eff.assign(H.height + 1, P->tune);
  if (P->ctune.size() == P->eff.size()) P->eff = P->ctune;
  bool any_persistent = false;
  for (mf::Tuning &t : P->eff) {
    t.small_max_m = std::min<int32_t>(t.small_max_m, mm);
    any_persistent = any_persistent || t.persistent;
  }
  mf::build_schedule(H, P->eff);
  std::vector<int32_t> lists;
  std::vector<mf::GemmTask> tasks;
  std::vector<mf::PanelRec> panel;
  P->lv.assign(H.levels.size(), LevelDev());
  auto put = [&](const std::vector<int32_t> &v) {
    const int64_t off = (int64_t)lists.size();
    lists.insert(lists.end(), v.begin(), v.end());
    return off;
  };
  for (size_t l = 0; l < H.levels.size(); ++l) {
    const mf::LevelSchedule &S = H.levels[l];
    LevelDev &D = P->lv[l];
    D.tiny = put(S.tiny);
    D.n_tiny = (int64_t)S.tiny.size();
    D.tiny_max_m = S.tiny_max_m;
    D.small = put(S.small);
    D.n_small = (int64_t)S.small.size();
    D.small_max_m = S.small_max_m;
    D.large = put(S.large);
    D.n_large = (int64_t)S.large.size();
    D.large_max_m = S.large_max_m;
    D.fused = put(S.fused);
    D.n_fused = (int64_t)S.fused.size();
    D.fused_max_m = S.fused_max_m;
    D.all = put(S.all);
    D.n_all = (int64_t)S.all.size();
    D.max_m = S.max_m;
    D.max_k = S.max_k;
    for (const mf::PanelStep &st : S.steps) {
      StepDev sd;
      sd.n = (int64_t)st.fronts.size();
      sd.prec = (int64_t)panel.size();
      for (size_t i = 0; i < st.fronts.size(); ++i) {
        const mf::FrontDesc &d = H.desc[st.fronts[i]];
        mf::PanelRec r;
        r.store = d.store;
        r.m = d.m;
        r.k = d.k;
        r.p0 = st.p0[i];
        r.f = st.fronts[i];
        panel.push_back(r);
      }
      for (size_t i = 0; i < st.fronts.size(); ++i) {
        const mf::FrontDesc &d = H.desc[st.fronts[i]];
        sd.la_chunks = std::max(sd.la_chunks,
                                mf::lookahead_chunks(d.m, std::min(st.p0[i] + mf::LA_NB, d.k)));
      }
      sd.update = (int64_t)tasks.size();
      sd.n_update = (int64_t)st.update.size();
      append_xcd_ordered(tasks, st.update, 0);
      sd.prev_update = (int64_t)tasks.size();
      sd.n_prev_update = (int64_t)st.prev_update.size();
      // the update tiles follow the panel's workgroups in the same launch
      append_xcd_ordered(tasks, st.prev_update, sd.n * (int64_t)sd.la_chunks);
      sd.trsm_items = st.trsm_items;
      D.steps.push_back(sd);
    }
    D.lookahead = S.lookahead;
    D.schur = (int64_t)tasks.size();
    D.n_schur = (int64_t)S.schur.size();
    append_xcd_ordered(tasks, S.schur, 0);
    level_costs(H, S, D, P->eff[l].persistent ? mf::kClassNB : P->eff[l].nb);
  }
  // wave records follow the class lists, class after class
  {
    int64_t off = 0;
    for (size_t l = 0; l < H.levels.size(); ++l) {
      P->lv[l].rall = off;
      off += (int64_t)H.levels[l].all.size();
    }
  }
  // rectangular-part tasks of the classes the block solves handle (x: the front's wave record)
  std::vector<int4> rect, chunk;
  P->chunk_ws_rows = 0;
  for (size_t l = 0; l < H.levels.size(); ++l) {
    const mf::LevelSchedule &S = H.levels[l];
    LevelDev &D = P->lv[l];
    if (S.max_m <= kWaveSolveMaxM) continue;
    int32_t kmax = 0, cmax = 0;
    int64_t ckmax = 0;
    for (int32_t f : S.all) {
      const mf::FrontDesc &d = H.desc[f];
      kmax = std::max(kmax, d.k);
      cmax = std::max(cmax, d.m - d.k);
      ckmax = std::max<int64_t>(ckmax, (int64_t)(d.m - d.k) * d.k);
    }
    // a separate launch costs a few dependent memory round trips; it pays once the
    // rectangular part is large (measured on the 256 x 256 grid: from c k = 16K down, 8K up)
    D.split_down = ckmax >= kSplitDownCK;
    D.split_up = ckmax >= kSplitUpCK;
    // chunked triangle solves (k_solve_chunk) for classes with many pivots; their contribution
    // rows then always take the rectangular launches
    D.chunked = P->chunk_min_k > 0 && kmax >= P->chunk_min_k;
    if (D.chunked) D.split_down = D.split_up = ckmax > 0;
    // slabs of 64 rows, or of 16 (the quarter form) where a class has too few slabs of 64 to
    // occupy the chip
    int64_t n64_down = 0, n64_up = 0;
    for (size_t i = 0; i < S.all.size(); ++i) {
      const mf::FrontDesc &d = H.desc[S.all[i]];
      n64_down += (d.m - d.k + mf::kRectRows - 1) / mf::kRectRows;
      if (d.m > d.k) n64_up += (d.k + mf::kRectRows - 1) / mf::kRectRows;
    }
    D.rect_q_down = n64_down < kRectQuarterBelow;
    D.rect_q_up = n64_up < kRectQuarterBelow;
    const int32_t sd = D.rect_q_down ? mf::kRectRowsQ : mf::kRectRows;
    const int32_t su = D.rect_q_up ? mf::kRectRowsQ : mf::kRectRows;
    D.rdown = (int64_t)rect.size();
    if (D.split_down)
      for (size_t i = 0; i < S.all.size(); ++i) {
        const mf::FrontDesc &d = H.desc[S.all[i]];
        const int32_t ri = (int32_t)(D.rall + (int64_t)i);
        for (int32_t r = d.k; r < d.m; r += sd) rect.push_back(make_int4(ri, r, std::min(sd, d.m - r), 0));
      }
    D.n_rdown = (int64_t)rect.size() - D.rdown;
    D.rup = (int64_t)rect.size();
    if (D.split_up)
      for (size_t i = 0; i < S.all.size(); ++i) {
        const mf::FrontDesc &d = H.desc[S.all[i]];
        const int32_t ri = (int32_t)(D.rall + (int64_t)i);
        if (d.m == d.k) continue;
        for (int32_t r = 0; r < d.k; r += su) rect.push_back(make_int4(ri, r, std::min(su, d.k - r), 0));
      }
    D.n_rup = (int64_t)rect.size() - D.rup;
    if (D.chunked) {
      // per front: its pivot rows in the workspace; stage strips; per launch of each sweep the
      // chunk's writer and its tiles (down: rows below the chunk, up: rows above it)
      int32_t wrow = 0, nch = 0;
      std::vector<int32_t> wr(S.all.size());
      std::vector<std::vector<int32_t>> starts(S.all.size());   // first pivot of each chunk
      for (size_t i = 0; i < S.all.size(); ++i) {
        const mf::FrontDesc &d = H.desc[S.all[i]];
        wr[i] = wrow;
        wrow += d.k;
        for (int32_t p0 = 0; p0 < d.k; p0 += mf::chunk_pivots(d.k, p0)) starts[i].push_back(p0);
        nch = std::max(nch, (int32_t)starts[i].size());
      }
      P->chunk_ws_rows = std::max<int64_t>(P->chunk_ws_rows, wrow);
      D.cstage = (int64_t)chunk.size();
      for (size_t i = 0; i < S.all.size(); ++i) {
        const mf::FrontDesc &d = H.desc[S.all[i]];
        const int32_t ri = (int32_t)(D.rall + (int64_t)i);
        for (int32_t r = 0; r < d.k; r += 256) chunk.push_back(make_int4(ri, r, std::min(256, d.k - r), wr[i]));
      }
      D.n_cstage = (int64_t)chunk.size() - D.cstage;
      for (int up = 0; up < 2; ++up) {
        std::vector<std::pair<int64_t, int64_t>> &steps = up ? D.csteps_up : D.csteps_down;
        steps.clear();
        for (int32_t st = 0; st < nch; ++st) {
          const int64_t first = (int64_t)chunk.size();
          for (size_t i = 0; i < S.all.size(); ++i) {
            const mf::FrontDesc &d = H.desc[S.all[i]];
            const int32_t ri = (int32_t)(D.rall + (int64_t)i);
            const int32_t nf = (int32_t)starts[i].size();
            if (st >= nf) continue;
            const int32_t c = up ? nf - 1 - st : st, p0 = starts[i][c];
            const int32_t p1 = p0 + mf::chunk_pivots(d.k, p0);
            chunk.push_back(make_int4(ri, p0, -1, wr[i]));
            const int32_t lo = up ? 0 : p1, hi = up ? p0 : d.k;
            for (int32_t r = lo; r < hi; r += mf::kTileRows) chunk.push_back(make_int4(ri, p0, r, wr[i]));
          }
          steps.emplace_back(first, (int64_t)chunk.size() - first);
        }
      }
    }
  }
  // persistent class launches: per class with tiled fronts, its task list in phase order
  // (extend-add strips, then per panel step the chunks and the update tiles, then the Schur
  // tiles) with the count of earlier-phase tasks of the same front that each task waits for
  std::vector<mf::ClassTask> ctasks;
  int64_t n_counters = 0;
  if (any_persistent) {
    for (size_t l = 0; l < H.levels.size(); ++l) {
      const mf::LevelSchedule &S = H.levels[l];
      LevelDev &D = P->lv[l];
      D.ctask = (int64_t)ctasks.size();
      D.n_ctask = 0;
      if (S.large.empty() || !P->eff[l].persistent) continue;
      std::vector<int32_t> cidx(S.large.size()), done(S.large.size(), 0);
      std::unordered_map<int32_t, int32_t> slot;
      for (size_t i = 0; i < S.large.size(); ++i) {
        cidx[i] = (int32_t)(n_counters++);
        slot[S.large[i]] = (int32_t)i;
      }
      auto base = [&](int32_t f, int32_t type) {
        const mf::FrontDesc &d = H.desc[f];
        mf::ClassTask t;
        std::memset(&t, 0, sizeof t);
        t.store = d.store;
        t.type = type;
        t.f = f;
        t.ci = cidx[slot[f]];
        t.need = done[slot[f]];
        t.m = d.m;
        t.k = d.k;
        return t;
      };
      std::vector<int32_t> phase(S.large.size(), 0);   // tasks of the current phase per front
      auto close_phase = [&]() {
        for (size_t i = 0; i < S.large.size(); ++i) {
          done[i] += phase[i];
          phase[i] = 0;
        }
      };
      for (size_t i = 0; i < S.large.size(); ++i) {
        const int32_t f = S.large[i];
        const int32_t m = H.desc[f].m;
        // strips of about 8K entries (rows in multiples of 4)
        const int32_t rows = std::min(m, std::max(4, ((8192 / std::max(1, m)) + 3) & ~3));
        for (int32_t r = 0; r < m; r += rows) {
          mf::ClassTask t = base(f, mf::kTaskAssemble);
          t.a = (int32_t)(D.rall + D.n_tiny + D.n_small + (int64_t)i);
          t.b = r;
          t.c = std::min(m, r + rows);
          ctasks.push_back(t);
          ++phase[i];
        }
      }
      close_phase();
      for (const mf::PanelStep &st : S.steps) {
        for (size_t i = 0; i < st.fronts.size(); ++i) {
          const int32_t f = st.fronts[i];
          const mf::FrontDesc &d = H.desc[f];
          const int32_t p0 = st.p0[i], pe = std::min(p0 + mf::kClassNB, d.k);
          const int32_t nch = mf::panel_chunks(d.m, pe);
          for (int32_t c = 0; c < nch; ++c) {
            mf::ClassTask t = base(f, mf::kTaskPanel);
            t.a = p0;
            t.b = c;
            t.c = nch;
            ctasks.push_back(t);
            ++phase[slot[f]];
          }
        }
        close_phase();
        for (const mf::GemmTask &g : st.update) {
          mf::ClassTask t = base(g.front, mf::kTaskUpdate);
          t.a = g.i0;
          t.b = g.i1;
          t.c = g.j0;
          t.d = g.j1;
          t.e = g.q0;
          t.g = g.q1;
          ctasks.push_back(t);
          ++phase[slot[g.front]];
        }
        close_phase();
      }
      for (const mf::GemmTask &g : S.schur) {
        mf::ClassTask t = base(g.front, mf::kTaskSchur);
        t.a = g.i0;
        t.b = g.i1;
        t.c = g.j0;
        t.d = g.j1;
        t.e = g.q0;
        t.g = g.q1;
        ctasks.push_back(t);
      }
      D.n_ctask = (int64_t)ctasks.size() - D.ctask;
      D.c_class.bytes = D.c_assemble.bytes + D.c_schur.bytes;
      D.c_class.flops = D.c_assemble.flops + D.c_schur.flops;
      for (const StepDev &sd : D.steps) {
        D.c_class.bytes += sd.trsm.bytes + sd.upd.bytes;
        D.c_class.flops += sd.trsm.flops + sd.upd.flops;
      }
    }
    // ticket counters (one per class) precede the progress counters
    for (size_t l = 0; l < H.levels.size(); ++l) P->lv[l].tick = (int32_t)l;
  }
  int rc;
  if ((rc = upload(P->d_lists, lists)) || (rc = upload(P->d_tasks, tasks)) ||
      (rc = upload(P->d_rect, rect)) || (rc = upload(P->d_chunk, chunk)) ||
      (rc = upload(P->d_panel, panel)) ||
      (rc = upload(P->d_ctasks, ctasks)))
    return rc;
  {
    const int64_t nc = any_persistent ? (int64_t)H.levels.size() + n_counters : 0;
    dfree(P->d_ccnt);
    P->n_ccnt = nc;
    if (hipMalloc((void **)&P->d_ccnt, std::max<int64_t>(1, nc) * sizeof(int)) != hipSuccess)
      return fail(MF_ENOMEM, "cannot allocate the class launches' counters");
  }
  if (!P->static_up) {
    // node -> (element, local node) pairs in ascending element order, for the residual
    std::vector<int64_t> nptr(H.n + 1, 0);
    for (int64_t q = 0; q < H.n_elem * H.npe; ++q) nptr[H.conn[q] + 1]++;
    for (int64_t v = 0; v < H.n; ++v) nptr[v + 1] += nptr[v];
    std::vector<int32_t> nelem(H.n_elem * H.npe);
    {
      std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
      for (int64_t q = 0; q < H.n_elem * H.npe; ++q) nelem[fill[H.conn[q]]++] = (int32_t)q;
    }
    if ((rc = upload(P->d_desc, H.desc)) || (rc = upload(P->d_front_idx, H.front_idx)) ||
        (rc = upload(P->d_inv_l, H.inv_l)) || (rc = upload(P->d_inv_r, H.inv_r)) ||
        (rc = upload(P->d_conn, H.conn)) || (rc = upload(P->d_nptr, nptr)) ||
        (rc = upload(P->d_nelem, nelem)))
      return rc;
    dfree(P->d_store);
    if (hipMalloc((void **)&P->d_store, std::max<int64_t>(1, H.store_doubles) * sizeof(double)) != hipSuccess)
      return fail(MF_ENOMEM, "cannot allocate " + std::to_string(H.store_doubles * 8) +
                                 " bytes of factor storage");
    // diagonal-block inverses for every front of the classes the block solves handle
    std::vector<int64_t> doff(H.desc.size(), -1);
    std::vector<int2> dtasks;
    int64_t dtot = 0;
    constexpr int64_t kPair = 2 * mf::NBS * mf::NBS;
    P->dinv_lvl.assign(H.levels.size() + 1, 0);
    for (size_t l = 0; l < H.levels.size(); ++l) {
      const mf::LevelSchedule &S = H.levels[l];
      P->dinv_lvl[l] = (int64_t)dtasks.size();
      if (S.max_m <= kWaveSolveMaxM) continue;
      for (int32_t f : S.all) {
        const int32_t k = H.desc[f].k;
        if (k <= 0) continue;
        doff[f] = dtot;
        for (int32_t p0 = 0; p0 < k; p0 += mf::NBS) dtasks.push_back(make_int2(f, p0));
        dtot += (int64_t)((k + mf::NBS - 1) / mf::NBS) * kPair;
      }
    }
    P->dinv_lvl[H.levels.size()] = (int64_t)dtasks.size();
    if ((rc = upload(P->d_dinv_off, doff)) || (rc = upload(P->d_dinv_tasks, dtasks))) return rc;
    P->h_dinv_off = doff;
    P->n_dinv_tasks = (int64_t)dtasks.size();
    P->c_dinv.bytes = 8.0 * P->n_dinv_tasks * (mf::NBS * mf::NBS + kPair);
    P->c_dinv.flops = P->n_dinv_tasks * 2.0 * mf::NBS * mf::NBS * mf::NBS / 3.0;
    dfree(P->d_dinv);
    if (hipMalloc((void **)&P->d_dinv, std::max<int64_t>(1, dtot) * sizeof(double)) != hipSuccess)
      return fail(MF_ENOMEM, "cannot allocate " + std::to_string(dtot * 8) +
                                 " bytes of diagonal-block inverses");
    // per-front arrival counters of the panel steps (zero between launches, see k_panel_trsm)
    dfree(P->d_arrive);
    if (hipMalloc((void **)&P->d_arrive, std::max<int64_t>(1, H.F) * sizeof(int)) != hipSuccess)
      return fail(MF_ENOMEM, "cannot allocate the panel arrival counters");
    HIPCHK(hipMemset(P->d_arrive, 0, std::max<int64_t>(1, H.F) * sizeof(int)));
    P->static_up = true;
  }
  // wave records, one per entry of every class's front list (the tiny fronts come first)
  std::vector<mf::WaveRec> wrec;
  wrec.reserve(H.F);
  for (size_t l = 0; l < H.levels.size(); ++l) {
    for (int32_t f : H.levels[l].all) {
      const mf::FrontDesc &d = H.desc[f];
      mf::WaveRec r;
      std::memset(&r, 0, sizeof r);
      r.f = f;
      r.m = d.m;
      r.k = d.k;
      r.store = d.store;
      r.idx = d.idx;
      r.cbrow = d.cbrow;
      r.ycb[0] = r.ycb[1] = -1;
      r.dinv = P->h_dinv_off[f];
      const int64_t e2 = (int64_t)H.npe * H.npe;
      if (d.elem >= 0) {
        r.src[0] = -1 - (int64_t)d.elem * e2;
        r.ld[0] = r.n[0] = H.npe;
      } else {
        const int32_t ch[2] = {d.left, d.right};
        for (int s2 = 0; s2 < 2; ++s2) {
          const mf::FrontDesc &c = H.desc[ch[s2]];
          if (c.elem >= 0 && c.k == 0) {       // pass-through leaf: its element matrix
            r.src[s2] = -1 - (int64_t)c.elem * e2;
            r.ld[s2] = r.n[s2] = H.npe;
          } else {
            r.src[s2] = c.store + (int64_t)c.k * c.m + c.k;
            r.ld[s2] = c.m;
            r.n[s2] = c.m - c.k;
            r.ycb[s2] = c.cbrow;
          }
        }
      }
      wrec.push_back(r);
    }
  }
  if ((rc = upload(P->d_wrec, wrec))) return rc;
  {
    // the up sweep's wave records: a front without pivots computes nothing there (its rows are
    // its ancestors' pivots), and the lower classes hold many of them (element-pair fronts)
    std::vector<mf::WaveRec> wup;
    int64_t w = 0;
    for (size_t l = 0; l < H.levels.size(); ++l) {
      P->lv[l].rwup = (int64_t)wup.size();
      for (size_t i = 0; i < H.levels[l].all.size(); ++i, ++w)
        if (wrec[w].k > 0) wup.push_back(wrec[w]);
      P->lv[l].n_wup = (int64_t)wup.size() - P->lv[l].rwup;
    }
    if ((rc = upload(P->d_wrec_up, wup))) return rc;
  }
  {
    // bottom subtrees: the leading classes on the tiny factor route, and on the wave solves
    std::vector<int64_t> wpos(H.F, -1);
    int64_t w = 0;
    for (const mf::LevelSchedule &S : H.levels)
      for (int32_t f : S.all) wpos[f] = w++;
    int32_t ef = 0, es = 0;
    while (ef < (int32_t)H.levels.size() &&
           H.levels[ef].tiny.size() == H.levels[ef].all.size())
      ++ef;
    while (es < (int32_t)H.levels.size() && H.levels[es].max_m <= kWaveSolveMaxM) ++es;
    if ((rc = build_subtrees(P, P->sub_f, ef, wrec, wpos)) ||
        (rc = build_subtrees(P, P->sub_s, es, wrec, wpos)))
      return rc;
  }
  if (!P->d_status) HIPCHK(hipMalloc((void **)&P->d_status, mf::kStatusWords * sizeof(int)));
  if (!P->h_status) {
    HIPCHK(hipHostMalloc((void **)&P->h_status, mf::kStatusWords * sizeof(int),
                         hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&P->d_hstatus, P->h_status, 0));
  }
  if (!P->cap_stream) HIPCHK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  if (!P->side_stream) HIPCHK(hipStreamCreateWithFlags(&P->side_stream, hipStreamNonBlocking));
  // events that only order the plan's two streams on this device: no system-scope fence (the
  // device-scope release of the recorded work is what the other stream needs; the host never
  // waits on them), which removes a stall of the recording stream at every record
  while (P->lvl_events.size() < H.levels.size() + 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence));
    P->lvl_events.push_back(e);
  }
  // raise the dynamic-LDS limit of the kernels that size LDS per launch (best effort)
  const void *dyn[] = {(const void *)mf::k_factor_tiny<1>, (const void *)mf::k_factor_tiny<4>,
                       (const void *)mf::k_factor_tiny<9>, (const void *)mf::k_factor_tiny<16>,
                       (const void *)mf::k_factor_small<256>,
                       (const void *)mf::k_factor_small<mf::SM_THREADS>,
                       (const void *)mf::k_assemble, (const void *)mf::k_front_panels<32>,
                       (const void *)mf::k_solve_down_wave<false>, (const void *)mf::k_solve_down_wave<true>,
                       (const void *)mf::k_solve_up_wave<false>, (const void *)mf::k_solve_up_wave<true>,
                       (const void *)mf::k_solve_down_block<false, false>,
                       (const void *)mf::k_solve_down_block<true, false>,
                       (const void *)mf::k_solve_down_block<false, true>,
                       (const void *)mf::k_solve_down_block<true, true>,
                       (const void *)mf::k_solve_up_block<false, false>,
                       (const void *)mf::k_solve_up_block<true, false>,
                       (const void *)mf::k_solve_up_block<false, true>,
                       (const void *)mf::k_solve_up_block<true, true>,
                       (const void *)mf::k_factor_subtree<1>, (const void *)mf::k_factor_subtree<4>,
                       (const void *)mf::k_factor_subtree<9>, (const void *)mf::k_factor_subtree<16>,
                       (const void *)mf::k_solve_down_subtree<false>,
                       (const void *)mf::k_solve_down_subtree<true>,
                       (const void *)mf::k_solve_up_subtree<false>,
                       (const void *)mf::k_solve_up_subtree<true>,
                       (const void *)mf::k_solve_chunk<false>, (const void *)mf::k_solve_chunk<true>};
  for (const void *fn : dyn)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, P->max_shared);
  (void)hipGetLastError();
  if (any_persistent) {
    // workgroups of a persistent class launch resident at once (the launch never needs more:
    // it runs any number of tasks, and never waits for a workgroup that has not started)
    int per_cu = 0, cus = 0;
    int32_t mmax = 1;
    for (const LevelDev &D : P->lv) mmax = std::max(mmax, D.large_max_m);
    const size_t lds = mf::class_lds_bytes<2, 64>(mmax) > mf::class_lds_bytes<2, 32>(mmax)
                           ? mf::class_lds_bytes<2, 64>(mmax) : mf::class_lds_bytes<2, 32>(mmax);
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, (const void *)mf::k_class_tiled<0, 64>, 256, lds));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    P->class_blocks = std::max(1, per_cu) * std::max(1, cus);
  }
  P->uploaded = true;
  return MF_OK;
}

// Message of a bad pivot reported by the kernels: the front and pivot, the mesh they belong to,
// the front's id within that mesh and the pivot's node (global id and id within the mesh).
std::string pivot_message(const mf_plan *P, int32_t f, int32_t p) {
  const mf::HostPlan &H = P->hp;
  std::string msg = "zero or non-finite pivot in front " + std::to_string(f) + ", pivot " +
                    std::to_string(p);
  if (f < 0 || f >= H.F) return msg;
  const auto it = std::upper_bound(H.mesh_front_ptr.begin(), H.mesh_front_ptr.end(), (int64_t)f);
  const int64_t mi = (int64_t)(it - H.mesh_front_ptr.begin()) - 1;
  msg += " (mesh " + std::to_string(mi) + ", front " + std::to_string(f - H.mesh_front_ptr[mi]) +
         " of that mesh";
  if (p >= 0 && p < H.desc[f].k) {
    const int32_t v = H.front_idx[H.front_ptr[f] + p];
    msg += ", node " + std::to_string(v) + " = node " + std::to_string(v - H.mesh_node_ptr[mi]) +
           " of that mesh";
  }
  return msg + ")";
}

// Doubles of a solve's contribution-block buffer: the per-front contribution blocks (sum_c rows)
// and the chunked triangle solves' workspace rows, nrhs values per row.
size_t ycb_doubles(const mf_plan *P, int32_t nrhs) {
  return (size_t)std::max<int64_t>(1, P->hp.sum_c + P->chunk_ws_rows) * nrhs;
}

int grow(mf_plan *P, double *&buf, size_t &cap, size_t doubles) {
  if (cap >= doubles && buf) return MF_OK;
  P->drop_graphs();   // captured launches may hold the old pointer
  dfree(buf);
  cap = 0;
  if (hipMalloc((void **)&buf, std::max<size_t>(doubles, 1) * sizeof(double)) != hipSuccess)
    return fail(MF_ENOMEM, "cannot allocate " + std::to_string(doubles * 8) + " bytes of workspace");
  cap = doubles;
  return MF_OK;
}

// -- launches -------------------------------------------------------------------------------
struct Scope {
  mf_plan *P;
  hipStream_t s;
  int kind;
  Cost cost;
  hipEvent_t a = nullptr;
  Scope(mf_plan *P_, int kind_, Cost c, hipStream_t s_) : P(P_), s(s_), kind(kind_), cost(c) {
    if (P->prof.on && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
  }
  ~Scope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    (void)hipEventRecord(b, s);
    P->prof.recs.push_back(ProfRec{kind, P->prof.cur_class, a, b, cost});
  }
};

#define LAUNCH(kind, cost, kern, grid, block, lds, stream, ...)                          \
  do {                                                                                   \
    ::mfapi::Scope sc_(P, kind, cost, stream);                                           \
    hipLaunchKernelGGL(kern, grid, block, lds, stream, __VA_ARGS__);                     \
  } while (0)

// The launches of class l of the factorization.
int factor_level(mf_plan *P, const double *K, int prec, size_t l, hipStream_t s) {
  P->prof.cur_class = (int)l;
  if ((int32_t)l < P->sub_f.ncls) {
    // the bottom-subtree launch runs classes 0..ncls-1 (issued with class 0)
    const mfapi::SubtreeDev &S = P->sub_f;
    if (l == 0) {
      const int m = S.max_m;
      const int ldsw = m * (m | 1) + m;
      const int grid = (int)std::min<int64_t>(S.nsub, 65535);
      const size_t lds = (size_t)4 * ldsw * 8;
      if (m > mf::kTinyMaxM) return fail(MF_EINVAL, "tiny route front wider than the kernel's limit");
#define MF_SUB(U)                                                                                \
  LAUNCH(K_SUB_FACTOR, S.c_factor, mf::k_factor_subtree<U>, dim3(grid), dim3(256), lds, s, S.d_rec, \
         S.d_ptr, (int)S.nsub, S.ncls, P->d_store, P->d_inv_l, P->d_inv_r, K, P->d_status, ldsw, m)
      if (m <= 8) MF_SUB(1);
      else if (m <= 16) MF_SUB(4);
      else if (m <= 24) MF_SUB(9);
      else MF_SUB(16);
#undef MF_SUB
    }
    P->prof.cur_class = -1;
    return MF_OK;
  }
  {
    const LevelDev &D = P->lv[l];
    const mf::Tuning &T = P->eff[l];
    if (D.n_tiny) {
      const int m = D.tiny_max_m;
      const int ldsw = m * (m | 1) + m;           // front + 2m int maps
      const int grid = (int)std::min<int64_t>((D.n_tiny + 3) / 4, 65535);
      const mf::WaveRec *rc0 = P->d_wrec + D.rall;   // the tiny fronts lead the class's list
      if (m > mf::kTinyMaxM) return fail(MF_EINVAL, "tiny route front wider than the kernel's limit");
      if (m <= 8)
        LAUNCH(K_TINY, D.c_tiny, mf::k_factor_tiny<1>, dim3(grid), dim3(256), (size_t)4 * ldsw * 8, s,
               rc0, (int)D.n_tiny, P->d_store, P->d_inv_l, P->d_inv_r, K, P->d_status, ldsw, m);
      else if (m <= 16)
        LAUNCH(K_TINY, D.c_tiny, mf::k_factor_tiny<4>, dim3(grid), dim3(256), (size_t)4 * ldsw * 8, s,
               rc0, (int)D.n_tiny, P->d_store, P->d_inv_l, P->d_inv_r, K, P->d_status, ldsw, m);
      else if (m <= 24)
        LAUNCH(K_TINY, D.c_tiny, mf::k_factor_tiny<9>, dim3(grid), dim3(256), (size_t)4 * ldsw * 8, s,
               rc0, (int)D.n_tiny, P->d_store, P->d_inv_l, P->d_inv_r, K, P->d_status, ldsw, m);
      else
        LAUNCH(K_TINY, D.c_tiny, mf::k_factor_tiny<16>, dim3(grid), dim3(256), (size_t)4 * ldsw * 8, s,
               rc0, (int)D.n_tiny, P->d_store, P->d_inv_l, P->d_inv_r, K, P->d_status, ldsw, m);
    }
    if (D.n_small) {
      const int m = D.small_max_m;
      const size_t lds = (size_t)mf::small_lds_doubles(m) * sizeof(double);
      const int grid = (int)std::min<int64_t>(D.n_small, 16384);
      // more fronts than compute units: smaller workgroups, more of them resident
      if (D.n_small > P->n_cu)
        LAUNCH(K_SMALL, D.c_small, mf::k_factor_small<256>, dim3(grid), dim3(256), lds, s,
               P->d_wrec + D.rall + D.n_tiny, (int)D.n_small, P->d_store, P->d_inv_l, P->d_inv_r,
               K, P->d_status, m);
      else
        LAUNCH(K_SMALL, D.c_small, mf::k_factor_small<mf::SM_THREADS>, dim3(grid),
               dim3(mf::SM_THREADS), lds, s, P->d_wrec + D.rall + D.n_tiny, (int)D.n_small,
               P->d_store, P->d_inv_l, P->d_inv_r, K, P->d_status, m);
    }
    if (D.n_large && D.n_ctask) {
      const size_t lds = T.tile == 32 ? mf::class_lds_bytes<2, 32>(D.large_max_m)
                                            : mf::class_lds_bytes<2, 64>(D.large_max_m);
      const int grid = (int)std::min<int64_t>(D.n_ctask, P->class_blocks);
      const mf::ClassTask *ct = P->d_ctasks + D.ctask;
      int *tick = P->d_ccnt + D.tick;
      int *cnt = P->d_ccnt + P->lv.size();
#define MF_CLASS(PR, TI)                                                                       \
  LAUNCH(K_CLASS, D.c_class, (mf::k_class_tiled<PR, TI>), dim3(grid), dim3(256), lds, s, ct,   \
         (int)D.n_ctask, tick, cnt, P->d_wrec, P->d_store, P->d_inv_l, P->d_inv_r, K,          \
         P->d_status, P->wait_ticks)
      if (T.tile == 32) {
        if (prec == MF_SCHUR_FP32) MF_CLASS(1, 32);
        else if (prec == MF_SCHUR_BF16) MF_CLASS(2, 32);
        else MF_CLASS(0, 32);
      } else {
        if (prec == MF_SCHUR_FP32) MF_CLASS(1, 64);
        else if (prec == MF_SCHUR_BF16) MF_CLASS(2, 64);
        else MF_CLASS(0, 64);
      }
#undef MF_CLASS
    } else if (D.n_large) {
      LAUNCH(K_ASSEMBLE, D.c_assemble, mf::k_assemble,
             dim3((D.large_max_m + 3) / 4, (unsigned)std::min<int64_t>(D.n_large, kMaxGridY)),
             dim3(256), (size_t)2 * D.large_max_m * sizeof(int), s,
             P->d_wrec + D.rall + D.n_tiny + D.n_small, (int)D.n_large, P->d_store, P->d_inv_l,
             P->d_inv_r, K);
      if (D.n_fused) {
        const size_t lds = (size_t)(32 * 33 + 32 + 32 * mf::FP_MAXM) * sizeof(double);
        LAUNCH(K_FUSED, D.c_fused, mf::k_front_panels<32>, dim3((unsigned)D.n_fused),
               dim3(mf::FP_THREADS), lds, s, P->d_desc, P->d_lists + D.fused, (int)D.n_fused,
               P->d_store, P->d_status);
      }
      if (D.lookahead) {
        for (const StepDev &st : D.steps) {
          Cost c;
          c.bytes = st.trsm.bytes + st.upd.bytes;
          c.flops = st.trsm.flops + st.upd.flops;
          const int64_t nblk = st.n * (int64_t)st.la_chunks + st.n_prev_update;
          const mf::PanelRec *pr = P->d_panel + st.prec;
          const mf::GemmTask *t = P->d_tasks + st.prev_update;
          if (T.tile == 32)
            LAUNCH(K_PANEL_LA, c, mf::k_panel_lookahead<32>, dim3((unsigned)nblk), dim3(256), 0, s,
                   pr, (int)st.n, st.la_chunks, t, P->d_store, P->d_status, P->d_arrive);
          else
            LAUNCH(K_PANEL_LA, c, mf::k_panel_lookahead<64>, dim3((unsigned)nblk), dim3(256), 0, s,
                   pr, (int)st.n, st.la_chunks, t, P->d_store, P->d_status, P->d_arrive);
        }
      }
      for (size_t si = 0; si < (D.lookahead ? 0 : D.steps.size()); ++si) {
        const StepDev &st = D.steps[si];
        const dim3 gt((unsigned)std::max<int64_t>(1, (st.trsm_items + 255) / 256),
                      (unsigned)std::min<int64_t>(st.n, kMaxGridY));
        const mf::PanelRec *pr = P->d_panel + st.prec;
        switch (T.nb) {
          case 16:
            LAUNCH(K_TRSM, st.trsm, mf::k_panel_trsm<16>, gt, dim3(256), 0, s, pr, (int)st.n, P->d_store, P->d_status,
                   P->d_arrive);
            break;
          case 64:
            LAUNCH(K_TRSM, st.trsm, mf::k_panel_trsm<64>, gt, dim3(256), 0, s, pr, (int)st.n, P->d_store, P->d_status,
                   P->d_arrive);
            break;
          default:
            LAUNCH(K_TRSM, st.trsm, mf::k_panel_trsm<32>, gt, dim3(256), 0, s, pr, (int)st.n, P->d_store, P->d_status,
                   P->d_arrive);
        }
        if (st.n_update) {
          const dim3 g((unsigned)st.n_update);
          const mf::GemmTask *t = P->d_tasks + st.update;
          if (T.tile == 32)
            LAUNCH(K_GEMM_PANEL, st.upd, (mf::k_gemm_update<0, 32>), g, dim3(256), 0, s, t, P->d_store);
          else
            LAUNCH(K_GEMM_PANEL, st.upd, (mf::k_gemm_update<0, 64>), g, dim3(256), 0, s, t, P->d_store);
        }
      }
      if (D.n_schur) {
        const mf::GemmTask *t = P->d_tasks + D.schur;
        const dim3 g((unsigned)D.n_schur);
        const bool t32 = T.tile == 32;
        if (prec == MF_SCHUR_FP32) {
          if (t32) LAUNCH(K_GEMM_SCHUR, D.c_schur, (mf::k_gemm_update<1, 32>), g, dim3(256), 0, s, t, P->d_store);
          else LAUNCH(K_GEMM_SCHUR, D.c_schur, (mf::k_gemm_update<1, 64>), g, dim3(256), 0, s, t, P->d_store);
        } else if (prec == MF_SCHUR_BF16) {
          if (t32) LAUNCH(K_GEMM_SCHUR, D.c_schur, (mf::k_gemm_update<2, 32>), g, dim3(256), 0, s, t, P->d_store);
          else LAUNCH(K_GEMM_SCHUR, D.c_schur, (mf::k_gemm_update<2, 64>), g, dim3(256), 0, s, t, P->d_store);
        } else {
          if (t32) LAUNCH(K_GEMM_SCHUR, D.c_schur, (mf::k_gemm_update<0, 32>), g, dim3(256), 0, s, t, P->d_store);
          else LAUNCH(K_GEMM_SCHUR, D.c_schur, (mf::k_gemm_update<0, 64>), g, dim3(256), 0, s, t, P->d_store);
        }
      }
    }
  }
  P->prof.cur_class = -1;
  return MF_OK;
}

// Diagonal-block inverses of the tasks [lo, hi) (the tasks are ordered class by class).
void dinv_launch(mf_plan *P, int64_t lo, int64_t hi, hipStream_t s) {
  if (hi <= lo) return;
  Cost c;
  const double frac = (double)(hi - lo) / (double)std::max<int64_t>(1, P->n_dinv_tasks);
  c.bytes = P->c_dinv.bytes * frac;
  c.flops = P->c_dinv.flops * frac;
  const int grid = (int)std::min<int64_t>((hi - lo + 3) / 4, 65535);
  LAUNCH(K_DIAG_INV, c, mf::k_diag_inverse, dim3(grid), dim3(256), 0, s, P->d_desc,
         P->d_dinv_tasks + lo, (int)(hi - lo), P->d_store, P->d_dinv_off, P->d_dinv);
}

// Clears the status block (and the persistent class launches' counters) on s.
void clear_status(mf_plan *P, hipStream_t s) {
  if (P->n_ccnt > 0) {
    const int grid = (int)std::min<int64_t>(1024, (P->n_ccnt + 255) / 256);
    hipLaunchKernelGGL(mf::k_clear_status_counters, dim3(grid), dim3(256), 0, s, P->d_status,
                       P->d_ccnt, P->n_ccnt);
  } else {
    hipLaunchKernelGGL(mf::k_clear_status, dim3(1), dim3(64), 0, s, P->d_status);
  }
}

int launch_factor(mf_plan *P, const double *K, int prec, hipStream_t s) {
  clear_status(P, s);
  int rc;
  for (size_t l = 0; l < P->lv.size(); ++l)
    if ((rc = factor_level(P, K, prec, l, s))) return rc;
  dinv_launch(P, 0, P->n_dinv_tasks, s);
  HIPCHK(hipGetLastError());
  return MF_OK;
}


// Largest power-of-two column chunk (<= nrhs) whose LDS footprint fits.
int chunk(const mf_plan *P, int32_t nrhs, int64_t fixed_doubles, int64_t per_col_doubles) {
  int nc = 1;
  while (nc * 2 <= nrhs && (fixed_doubles + per_col_doubles * nc * 2) * 8 <= P->max_shared) nc *= 2;
  return nc;
}

// The launches of class l of the forward (down) or backward sweep; ycb holds the per-front
// contribution blocks of the right-hand sides ([sum of CB widths][nrhs] doubles).
void solve_level(mf_plan *P, const double *b, double *x, int32_t nrhs, bool trans, bool down,
                 size_t l, hipStream_t s, double *ycb) {
  const int gridcap = 16384;
  {
    {
      if ((int32_t)l < P->sub_s.ncls) {
        // the bottom-subtree launch of the sweep: issued with class 0 (down: the first class
        // of the sweep, up: the last), it runs classes 0..ncls-1
        const mfapi::SubtreeDev &S = P->sub_s;
        if (l != 0) return;
        Cost c;
        c.bytes = (down ? S.down_coef : S.up_coef) + nrhs * (down ? S.down_rhs_bytes : S.up_rhs_bytes);
        c.flops = nrhs * (down ? S.down_rhs_flops : S.up_rhs_flops);
        const int mmax = std::max(1, S.max_m), kmax = std::max(1, S.max_k);
        const int cld = kmax | 1;
        const int64_t cdoubles = (int64_t)mmax * cld + mf::kWaveRows;
        const int nc = chunk(P, nrhs, 4 * cdoubles, 4 * (int64_t)mmax);
        const int ldsw = (int)(mmax * nc + cdoubles);
        const size_t lds = (size_t)4 * ldsw * 8;
        const int grid = (int)std::min<int64_t>(S.nsub, 65535);
        if (down && trans)
          LAUNCH(K_SUB_DOWN, c, mf::k_solve_down_subtree<true>, dim3(grid), dim3(256), lds, s,
                 S.d_rec, S.d_ptr, (int)S.nsub, S.ncls, P->d_store, P->d_front_idx, P->d_inv_l,
                 P->d_inv_r, b, x, ycb, nrhs, nc, mmax, cld, ldsw);
        else if (down)
          LAUNCH(K_SUB_DOWN, c, mf::k_solve_down_subtree<false>, dim3(grid), dim3(256), lds, s,
                 S.d_rec, S.d_ptr, (int)S.nsub, S.ncls, P->d_store, P->d_front_idx, P->d_inv_l,
                 P->d_inv_r, b, x, ycb, nrhs, nc, mmax, cld, ldsw);
        else if (trans)
          LAUNCH(K_SUB_UP, c, mf::k_solve_up_subtree<true>, dim3(grid), dim3(256), lds, s,
                 S.d_rec, S.d_ptr, (int)S.nsub, S.ncls, P->d_store, P->d_front_idx, x, nrhs, nc,
                 mmax, cld, ldsw);
        else
          LAUNCH(K_SUB_UP, c, mf::k_solve_up_subtree<false>, dim3(grid), dim3(256), lds, s,
                 S.d_rec, S.d_ptr, (int)S.nsub, S.ncls, P->d_store, P->d_front_idx, x, nrhs, nc,
                 mmax, cld, ldsw);
        return;
      }
      const LevelDev &D = P->lv[l];
      if (!D.n_all) return;
      Cost c;
      c.bytes = (down ? D.down_coef : D.up_coef) + nrhs * (down ? D.down_rhs_bytes : D.up_rhs_bytes);
      c.flops = nrhs * (down ? D.down_rhs_flops : D.up_rhs_flops);
      const mf::WaveRec *rec = P->d_wrec + D.rall;
      const int n = (int)D.n_all;
      const int mmax = std::max(1, D.max_m), kmax = std::max(1, D.max_k);
      if (D.max_m <= kWaveSolveMaxM) {
        // per wave: W (mmax x nc) + coefficients (mmax rows of kmax) + 64 reciprocals
        const int cld = kmax | 1;
        const int64_t cdoubles = (int64_t)mmax * cld + mf::kWaveRows;
        const int nc = chunk(P, nrhs, 4 * cdoubles, 4 * (int64_t)mmax);
        const int ldsw = (int)(mmax * nc + cdoubles);
        const size_t lds = (size_t)4 * ldsw * 8;
        const int grid = (int)std::min<int64_t>((n + 3) / 4, gridcap);
        const mf::WaveRec *rec_up = P->d_wrec_up + D.rwup;
        const int grid_up = (int)std::min<int64_t>((D.n_wup + 3) / 4, gridcap);
        if (down && trans)
          LAUNCH(K_DOWN_WAVE, c, mf::k_solve_down_wave<true>, dim3(grid), dim3(256), lds, s, rec,
                 n, P->d_store, P->d_front_idx, P->d_inv_l, P->d_inv_r, b, x, ycb, nrhs, nc,
                 mmax, cld, ldsw);
        else if (down)
          LAUNCH(K_DOWN_WAVE, c, mf::k_solve_down_wave<false>, dim3(grid), dim3(256), lds, s, rec,
                 n, P->d_store, P->d_front_idx, P->d_inv_l, P->d_inv_r, b, x, ycb, nrhs, nc,
                 mmax, cld, ldsw);
        else if (D.n_wup == 0)
          return;                               // no front of the class has pivots
        else if (trans)
          LAUNCH(K_UP_WAVE, c, mf::k_solve_up_wave<true>, dim3(grid_up), dim3(256), lds, s,
                 rec_up, (int)D.n_wup, P->d_store, P->d_front_idx, x, nrhs, nc, mmax, cld, ldsw);
        else
          LAUNCH(K_UP_WAVE, c, mf::k_solve_up_wave<false>, dim3(grid_up), dim3(256), lds, s,
                 rec_up, (int)D.n_wup, P->d_store, P->d_front_idx, x, nrhs, nc, mmax, cld, ldsw);
      } else {
        // the pivot block (one workgroup per front, blocks of NBS in sequence) and the
        // rectangular part (many workgroups): down triangle then rect, up rect then triangle
        Cost ct, cr;
        ct.bytes = D.tri_coef + nrhs * (down ? D.tri_down_rhs_bytes : D.tri_up_rhs_bytes);
        ct.flops = nrhs * (down ? D.tri_down_flops : D.tri_up_flops);
        cr.bytes = D.rect_coef + nrhs * (down ? D.rect_down_rhs_bytes : D.rect_up_rhs_bytes);
        cr.flops = nrhs * D.rect_flops;
        const bool split = down ? D.split_down : D.split_up;
        const int rmax = split ? kmax : mmax;
        if (!split) {
          ct.bytes = (down ? D.down_coef : D.up_coef) + nrhs * (down ? D.down_rhs_bytes : D.up_rhs_bytes);
          ct.flops = nrhs * (down ? D.down_rhs_flops : D.up_rhs_flops);
        }
        const int64_t fixed = mf::block_solve_fixed_doubles();
        const int nc = chunk(P, nrhs, fixed, mf::block_solve_col_doubles(rmax));
        const size_t lds = (size_t)(fixed + (int64_t)mf::block_solve_col_doubles(rmax) * nc) * 8;
        const int grid = std::min(n, gridcap);
        const int64_t nt = down ? D.n_rdown : D.n_rup;
        const int4 *rt = P->d_rect + (down ? D.rdown : D.rup);
        const bool rq = down ? D.rect_q_down : D.rect_q_up;
        const size_t rlds = ((size_t)16 * mf::kRectLdv + (rq ? 4 * 64 * 4 : 0)) * 8;
#define MF_DOWN_BLOCK(TR, FU)                                                                   \
  LAUNCH(K_DOWN_BLOCK, ct, (mf::k_solve_down_block<TR, FU>), dim3(grid), dim3(256), lds, s,     \
         rec, n, P->d_store, P->d_front_idx, P->d_inv_l, P->d_inv_r, b, x, ycb,            \
         nrhs, nc, rmax, P->d_dinv)
#define MF_UP_BLOCK(TR, FU)                                                                     \
  LAUNCH(K_UP_BLOCK, ct, (mf::k_solve_up_block<TR, FU>), dim3(grid), dim3(256), lds, s,         \
         rec, n, P->d_store, P->d_front_idx, x, nrhs, nc, rmax, P->d_dinv)
#define MF_RECT_Q(KIND, TR, UP, Q)                                                              \
  LAUNCH(KIND, cr, (mf::k_solve_rect<TR, UP, Q>), dim3((unsigned)nt), dim3(256), rlds, s,       \
         P->d_wrec, rt, P->d_store, P->d_front_idx, P->d_inv_l, P->d_inv_r, x, ycb, nrhs)
#define MF_RECT(KIND, TR, UP)                                                                   \
  do {                                                                                          \
    if (rq) MF_RECT_Q(KIND, TR, UP, true);                                                      \
    else MF_RECT_Q(KIND, TR, UP, false);                                                        \
  } while (0)
        if (!trans && D.chunked) {
          // chunked triangle: stage the pivot rows, one launch per chunk; the contribution rows
          // by the rectangular launches (after the triangle going down, before it going up)
          double *wsp = ycb + P->hp.sum_c * (int64_t)nrhs;
          const int ncc = chunk(P, nrhs, mf::chunk_solve_fixed_doubles(), mf::chunk_solve_col_doubles());
          const size_t clds =
              (size_t)(mf::chunk_solve_fixed_doubles() + (int64_t)mf::chunk_solve_col_doubles() * ncc) * 8;
          const int4 *stk = P->d_chunk + D.cstage;
          const unsigned nst = (unsigned)D.n_cstage;
          Cost cst, cc = ct;
          const double sum_k = D.tri_down_rhs_bytes / 24.0;    // pivots of the class
          cst.bytes = 16.0 * nrhs * sum_k;                      // pivot rows in and out
          const double nsteps = (double)std::max<size_t>(1, D.csteps_down.size());
          cc.bytes /= nsteps;                                   // the triangle's cost per launch
          cc.flops /= nsteps;
          if (down) {
            LAUNCH(K_CHUNK_STAGE, cst, mf::k_solve_chunk_stage<false>, dim3(nst), dim3(256), 0, s,
                   P->d_wrec, stk, P->d_front_idx, P->d_inv_l, P->d_inv_r, b, x, ycb, wsp, nrhs);
            for (const auto &st : D.csteps_down)
              LAUNCH(K_CHUNK, cc, mf::k_solve_chunk<false>, dim3((unsigned)st.second), dim3(256), clds,
                     s, P->d_wrec, P->d_chunk + st.first, P->d_store, P->d_front_idx, x, wsp, nrhs,
                     ncc, P->d_dinv);
            if (nt) MF_RECT(K_DOWN_RECT, false, false);
          } else {
            if (nt) MF_RECT(K_UP_RECT, false, true);
            LAUNCH(K_CHUNK_STAGE, cst, mf::k_solve_chunk_stage<true>, dim3(nst), dim3(256), 0, s,
                   P->d_wrec, stk, P->d_front_idx, P->d_inv_l, P->d_inv_r, b, x, ycb, wsp, nrhs);
            for (const auto &st : D.csteps_up)
              LAUNCH(K_CHUNK, cc, mf::k_solve_chunk<true>, dim3((unsigned)st.second), dim3(256), clds,
                     s, P->d_wrec, P->d_chunk + st.first, P->d_store, P->d_front_idx, x, wsp, nrhs,
                     ncc, P->d_dinv);
          }
        } else if (down) {
          if (split) {
            if (trans) MF_DOWN_BLOCK(true, false); else MF_DOWN_BLOCK(false, false);
            if (nt) {
              if (trans) MF_RECT(K_DOWN_RECT, true, false); else MF_RECT(K_DOWN_RECT, false, false);
            }
          } else {
            if (trans) MF_DOWN_BLOCK(true, true); else MF_DOWN_BLOCK(false, true);
          }
        } else {
          if (split) {
            if (nt) {
              if (trans) MF_RECT(K_UP_RECT, true, true); else MF_RECT(K_UP_RECT, false, true);
            }
            if (trans) MF_UP_BLOCK(true, false); else MF_UP_BLOCK(false, false);
          } else {
            if (trans) MF_UP_BLOCK(true, true); else MF_UP_BLOCK(false, true);
          }
        }
#undef MF_DOWN_BLOCK
#undef MF_UP_BLOCK
#undef MF_RECT
#undef MF_RECT_Q
      }
    }
  }
}

int launch_solve(mf_plan *P, const double *b, double *x, int32_t nrhs, bool trans, hipStream_t s,
                 double *ycb) {
  for (size_t l = 0; l < P->lv.size(); ++l) solve_level(P, b, x, nrhs, trans, true, l, s, ycb);
  for (size_t l = P->lv.size(); l-- > 0;) solve_level(P, b, x, nrhs, trans, false, l, s, ycb);
  HIPCHK(hipGetLastError());
  return MF_OK;
}

// Factorization and the solve of A x = b with the forward sweep overlapped: class l of the
// forward sweep needs only classes <= l of the factorization (and their diagonal-block
// inverses), so it runs on a second stream as soon as they are done, while the latency-bound
// upper classes of the factorization occupy a fraction of the chip; the backward sweep follows
// on s once both streams have joined.  The same kernels in the same per-class order as
// launch_factor then launch_solve, so the results are identical.
// Spacing of the second stream's joins among the classes below the first class with tiled
// fronts (0: it starts at that class), and whether each join's forward-sweep work is issued
// right after the factorization up to it (else after the whole factorization).  Measured on
// the 256 x 256 workload: joins every 2 or 3 lower classes make the step 3-5 % slower (the
// lower classes' forward sweep then competes with their factorization, which fills the chip,
// and every join stalls the caller's stream); interleaved issue is within noise.
constexpr int kSideStride = 0;
constexpr bool kSideInterleave = false;

int launch_factor_solve(mf_plan *P, const double *K, int prec, const double *b, double *x,
                        int32_t nrhs, hipStream_t s, bool cleared = false) {
  hipStream_t side = P->side_stream;
  const size_t L = P->lv.size();
  if (!cleared) clear_status(P, s);
  int rc;
  // The second stream's class l needs the factorization of classes <= l.  It joins the
  // caller's stream at "sync" classes: every class from the first one with tiled fronts (from
  // there the factorization is latency-bound and leaves most of the chip to the forward sweep),
  // and every kSideStride-th class below it, so that the lower classes' forward sweep overlaps
  // the factorization of the middle classes instead of queueing behind the upper ones.  Each
  // join costs an event record (a stall of a few microseconds on the caller's stream) and a
  // wait, so the lower classes join in groups.
  size_t start = 0;
  while (start + 1 < L && P->lv[start].n_large == 0) ++start;
  std::vector<char> sync(L, 0);
  for (size_t l = start; l < L; ++l) sync[l] = 1;
  if (kSideStride > 0)
    for (size_t l = kSideStride - 1; l < start; l += kSideStride) sync[l] = 1;
  sync[L - 1] = 1;
  // a bottom-subtree forward sweep (issued with class 0) runs its classes 0..ncls-1 at once:
  // it may start only after the factorization of all of them
  if (P->sub_s.ncls > 1) {
    for (size_t l = 0; l + 1 < (size_t)P->sub_s.ncls && l < L; ++l) sync[l] = 0;
    sync[std::min(L, (size_t)P->sub_s.ncls) - 1] = 1;
  }
  size_t next_side = 0;   // first class of the forward sweep not yet issued
  auto issue_side = [&](size_t upto) -> int {   // classes next_side .. upto behind event[upto]
    HIPCHK(hipStreamWaitEvent(side, P->lvl_events[upto], 0));
    for (; next_side <= upto; ++next_side) {
      dinv_launch(P, P->dinv_lvl[next_side], P->dinv_lvl[next_side + 1], side);
      solve_level(P, b, x, nrhs, false, true, next_side, side, P->d_ycb);
    }
    return MF_OK;
  };
  for (size_t l = 0; l < L; ++l) {
    if ((rc = factor_level(P, K, prec, l, s))) return rc;
    if (!sync[l]) continue;
    HIPCHK(hipEventRecord(P->lvl_events[l], s));
    if (kSideInterleave && (rc = issue_side(l))) return rc;
  }
  if (!kSideInterleave)
    for (size_t l = 0; l < L; ++l)
      if (sync[l] && (rc = issue_side(l))) return rc;
  HIPCHK(hipEventRecord(P->lvl_events[L], side));
  HIPCHK(hipStreamWaitEvent(s, P->lvl_events[L], 0));
  for (size_t l = L; l-- > 0;) solve_level(P, b, x, nrhs, false, false, l, s, P->d_ycb);
  HIPCHK(hipGetLastError());
  return MF_OK;
}

// Runs `launch` on `s`, through a cached hipGraph when graphs are enabled and profiling is off.
// The graph is captured on the plan's private stream (the caller's stream may be the null
// stream, which cannot be captured) and replayed on `s`.
template <typename F>
int run_graphed(mf_plan *P, Graph *cache, int n_cache, int &next, const GraphKey &key,
                hipStream_t s, F &&launch) {
  if (!P->use_graphs || P->prof.on) return launch(s);
  int slot = -1;
  for (int i = 0; i < n_cache; ++i)
    if (cache[i].exec && cache[i].key == key) slot = i;
  if (slot < 0) {
    slot = next;
    next = (next + 1) % n_cache;
  }
  Graph &g = cache[slot];
  if (!(g.exec && g.key == key)) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = Graph();
    HIPCHK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch(P->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(P->cap_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(MF_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      g.exec = nullptr;
      return fail(MF_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    }
    g.key = key;
  }
  HIPCHK(hipGraphLaunch(g.exec, s));
  return MF_OK;
}

// Column 2-norms in the refinement loop, one host synchronisation per iteration.  The tail of
// the refinement workspace holds per-block column sums of squares: the residual's (computed by
// the residual kernel itself when nrhs divides 256, else by k_colsq_partial over kNormRows rows
// per block), then those of b (kNormRows rows per block).
constexpr int64_t kNormRows = 512;   // rows per partial sum of k_colsq_partial

struct NormLayout {
  bool fused;                        // residual kernel writes the residual's partial sums
  int64_t r_blocks, b_blocks;
  size_t r_parts, b_parts;           // doubles of each partial-sum array
};

NormLayout norm_layout(int64_t n, int32_t nrhs) {
  NormLayout L;
  L.fused = 256 % nrhs == 0;
  L.r_blocks = L.fused ? std::max<int64_t>(1, (n * nrhs + 255) / 256)
                       : std::max<int64_t>(1, (n + kNormRows - 1) / kNormRows);
  L.b_blocks = std::max<int64_t>(1, (n + kNormRows - 1) / kNormRows);
  L.r_parts = (size_t)L.r_blocks * nrhs;
  L.b_parts = (size_t)L.b_blocks * nrhs;
  return L;
}

// The residual's column norms rn (and b's, bn, if want_b) from their partial sums: summed on
// the device and written, with the factorization's status words if with_status (into
// h_status), to mapped host memory by one small kernel, whose last workgroup then writes a
// sequence number there.  The host spins on that number for up to kSpinMicros (a wake-up from
// a stream synchronization costs tens of microseconds per refinement step), checking the stream
// for errors now and then, and falls back to a synchronization after that.
constexpr double kSpinMicros = 2000.0;

int read_norms(mf_plan *P, const NormLayout &L, const double *dpart, int32_t nrhs, hipStream_t s,
               bool want_b, std::vector<double> &rn, std::vector<double> &bn,
               bool with_status = false) {
  const size_t need = 2 * (size_t)nrhs + 1;   // the sums, then the sequence number
  if (P->part_cap < need) {
    if (P->h_part) (void)hipHostFree(P->h_part);
    P->h_part = nullptr;
    P->d_hpart = nullptr;
    P->part_cap = 0;
    HIPCHK(hipHostMalloc((void **)&P->h_part, need * sizeof(double),
                         hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&P->d_hpart, P->h_part, 0));
    P->part_cap = need;
  }
  if (!P->d_pub_count) {
    HIPCHK(hipMalloc((void **)&P->d_pub_count, sizeof(int)));
    HIPCHK(hipMemset(P->d_pub_count, 0, sizeof(int)));
  }
  int *hseq = reinterpret_cast<int *>(P->h_part + 2 * (size_t)nrhs);
  int *dseq = reinterpret_cast<int *>(P->d_hpart + 2 * (size_t)nrhs);
  if (P->pub_seq == INT32_MAX) P->pub_seq = 0;
  const int seq = ++P->pub_seq;
  __atomic_store_n(hseq, 0, __ATOMIC_RELAXED);   // no stale value can match (seq >= 1)
  const double *bpart = dpart + L.r_parts;
  const int grid = nrhs * (want_b ? 2 : 1);
  hipLaunchKernelGGL(mf::k_norm_publish, dim3(grid), dim3(256), 0, s, dpart, L.r_blocks, bpart,
                     want_b ? L.b_blocks : (int64_t)0, nrhs,
                     with_status ? (const int *)P->d_status : (const int *)nullptr, P->d_hpart,
                     P->d_hstatus, P->d_pub_count, dseq, seq);
  HIPCHK(hipGetLastError());
  const auto t0 = std::chrono::steady_clock::now();
  for (int64_t spins = 1;; ++spins) {
    if (__atomic_load_n(hseq, __ATOMIC_ACQUIRE) == seq) break;
    if (spins % 1024) continue;
    const hipError_t e = hipStreamQuery(s);
    if (e == hipSuccess) {
      if (__atomic_load_n(hseq, __ATOMIC_ACQUIRE) == seq) break;
      return fail(MF_EHIP, "the norm kernel completed without publishing its results");
    }
    if (e != hipErrorNotReady) return fail(MF_EHIP, std::string("hipStreamQuery: ") + hipGetErrorString(e));
    if (std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() >
        kSpinMicros) {
      HIPCHK(hipStreamSynchronize(s));
      if (__atomic_load_n(hseq, __ATOMIC_ACQUIRE) != seq)
        return fail(MF_EHIP, "the norm kernel completed without publishing its results");
      break;
    }
  }
  rn.assign(nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c) rn[c] = std::sqrt(P->h_part[c]);
  if (want_b) {
    bn.assign(nrhs, 0.0);
    for (int c = 0; c < nrhs; ++c) bn[c] = std::sqrt(P->h_part[nrhs + c]);
  }
  return MF_OK;
}

}  // namespace mfapi

// Scratch of the allocation-free solve (mf_solve_noalloc): the per-front contribution blocks of
// the right-hand sides.  One copy per GPU the library runs on, held until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host the name is only a stand-in
// for the symbol): the device address is taken once per device with hipGetSymbolAddress.
static __device__ __align__(256) double scratch[MF_NOALLOC_SCRATCH_DOUBLES];

namespace mfapi {
namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device, looked up on the first call per device.
int scratch_address(double **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return fail(MF_EINVAL, "device " + std::to_string(dev) + " beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return MF_OK;
}
}  // namespace
}  // namespace mfapi

using namespace mfapi;

extern "C" {

const char *mf_last_error(void) { return g_err.c_str(); }

int mf_analyse(int32_t n_mesh, const mf_mesh *meshes, mf_plan **out) {
  if (!out) return fail(MF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_mesh < 1 || !meshes) return fail(MF_EINVAL, "need n_mesh >= 1 and a mesh array");
  std::vector<int32_t> dims(n_mesh), npes(n_mesh);
  std::vector<int64_t> nn(n_mesh), ne(n_mesh);
  std::vector<const int32_t *> conns(n_mesh), ijks(n_mesh);
  for (int32_t i = 0; i < n_mesh; ++i) {
    dims[i] = meshes[i].dim;
    npes[i] = meshes[i].npe;
    nn[i] = meshes[i].n_nodes;
    ne[i] = meshes[i].n_elem;
    conns[i] = meshes[i].conn;
    ijks[i] = meshes[i].elem_ijk;
  }
  mf_plan *P = new (std::nothrow) mf_plan();
  if (!P) return fail(MF_ENOMEM, "cannot allocate plan");
  std::string err;
  try {
    err = mf::analyse(n_mesh, dims.data(), npes.data(), nn.data(), ne.data(), conns.data(),
                      ijks.data(), P->hp);
  } catch (const std::bad_alloc &) {
    delete P;
    return fail(MF_ENOMEM, "host allocation failed during analysis");
  }
  if (!err.empty()) {
    delete P;
    return fail(MF_EINVAL, err);
  }
  // MF_GRAPHS=0 in the environment: launch sequences run eagerly instead of as captured graphs
  const char *g = std::getenv("MF_GRAPHS");
  P->use_graphs = !(g && std::strcmp(g, "0") == 0);
  // MF_WAIT_LIMIT_US: bound of every device-side wait of the persistent class launches
  // (default one second; a launch whose wait exceeds it is abandoned and reported)
  if (const char *w = std::getenv("MF_WAIT_LIMIT_US")) {
    const long long us = std::atoll(w);
    if (us >= 0) P->wait_ticks = us * 100;   // the wait clock runs at 100 MHz
  }
  *out = P;
  return MF_OK;
}

int mf_plan_info(const mf_plan *P, mf_info *o) {
  if (!P || !o) return fail(MF_EINVAL, "null argument");
  const mf::HostPlan &H = P->hp;
  o->n = H.n;
  o->n_elem = H.n_elem;
  o->n_fronts = H.F;
  o->sum_m = (int64_t)H.front_idx.size();
  o->sum_mk = H.sum_mk;
  o->store_doubles = H.store_doubles;
  o->n_mesh = H.n_mesh;
  o->dim = H.dim;
  o->npe = H.npe;
  o->height = H.height;
  o->max_m = H.max_m;
  o->max_k = H.max_k;
  o->factor_flops = H.factor_flops;
  o->solve_flops_per_rhs = H.solve_flops;
  o->sum_cb2 = H.sum_cb2;
  return MF_OK;
}

int mf_plan_export_tree(const mf_plan *P, int32_t *parent, int32_t *level, int64_t *front_ptr,
                        int32_t *front_idx, int32_t *npiv, int64_t *leaf_elem) {
  if (!P) return fail(MF_EINVAL, "null plan");
  const mf::HostPlan &H = P->hp;
  if (parent) std::memcpy(parent, H.parent.data(), H.F * sizeof(int32_t));
  if (level) std::memcpy(level, H.level.data(), H.F * sizeof(int32_t));
  if (front_ptr) std::memcpy(front_ptr, H.front_ptr.data(), (H.F + 1) * sizeof(int64_t));
  if (front_idx) std::memcpy(front_idx, H.front_idx.data(), H.front_idx.size() * sizeof(int32_t));
  if (npiv) std::memcpy(npiv, H.npiv.data(), H.F * sizeof(int32_t));
  if (leaf_elem) std::memcpy(leaf_elem, H.leaf_elem.data(), H.F * sizeof(int64_t));
  return MF_OK;
}

int mf_task_trace(const mf_plan *P, mf_trace_info *out, int64_t *hist, int64_t cap,
                  int64_t *needed) {
  if (!P || !out) return fail(MF_EINVAL, "null plan or output");
  mf::TraceSummary t;
  std::vector<int64_t> h;
  const std::string err = mf::task_trace(P->hp, t, h);
  if (!err.empty()) return fail(MF_EINVAL, err);
  for (int i = 0; i < 4; ++i) out->tasks[i] = t.tasks[i];
  out->fnf_classes = t.fnf_classes;
  out->fnf_single_type_classes = t.fnf_single_type_classes;
  out->typed_classes = t.typed_classes;
  out->levels_order_dependencies = t.levels_order_dependencies;
  if (needed) *needed = (int64_t)h.size();
  if (hist && cap > 0) std::memcpy(hist, h.data(), std::min<int64_t>(cap, (int64_t)h.size()) * sizeof(int64_t));
  return MF_OK;
}

int mf_set_tuning(mf_plan *P, int32_t small_max_m, int32_t nb, int32_t fused_max_m, int32_t tile,
                  int32_t persistent) {
  if (!P) return fail(MF_EINVAL, "null plan");
  if (persistent < -1 || persistent > 1) return fail(MF_EINVAL, "persistent must be -1, 0 or 1");
  if (tile != 0 && tile != 32 && tile != 64) return fail(MF_EINVAL, "tile must be 32 or 64");
  if (small_max_m < 0) return fail(MF_EINVAL, "small_max_m must be >= 0");
  if (nb != 0 && nb != 16 && nb != 32 && nb != 64) return fail(MF_EINVAL, "nb must be 16, 32 or 64");
  if (fused_max_m < -1) return fail(MF_EINVAL, "fused_max_m must be >= -1");
  if (tile > 0) P->tune.tile = tile;
  if (persistent) P->tune.persistent = persistent > 0;
  if (small_max_m > 0) P->tune.small_max_m = small_max_m;
  if (nb > 0) P->tune.nb = nb;
  if (fused_max_m == -1) P->tune.fused_max_m = 0;
  else if (fused_max_m > 0) P->tune.fused_max_m = std::min(fused_max_m, mf::FP_MAXM);
  P->ctune.clear();         // one schedule for every class again
  P->uploaded = false;      // the schedule is rebuilt at the next device call
  P->factored = false;
  P->drop_graphs();
  return MF_OK;
}

int mf_set_subtree_launch(mf_plan *P, int32_t max_classes, int64_t min_units) {
  if (!P) return fail(MF_EINVAL, "null plan");
  if (max_classes < -1) return fail(MF_EINVAL, "max_classes must be >= -1");
  if (min_units < 1) return fail(MF_EINVAL, "min_units must be >= 1");
  P->sub_max_classes = max_classes;
  P->sub_min_units = min_units;
  P->uploaded = false;
  P->factored = false;
  P->drop_graphs();
  return MF_OK;
}

int mf_set_chunked_solve(mf_plan *P, int32_t min_pivots) {
  if (!P) return fail(MF_EINVAL, "null plan");
  if (min_pivots < 0) return fail(MF_EINVAL, "min_pivots must be >= 0");
  P->chunk_min_k = min_pivots;
  P->uploaded = false;      // the solve schedule is rebuilt at the next device call
  P->drop_graphs();
  return MF_OK;
}

int mf_subtree_launch_info(mf_plan *P, int64_t *out) {
  if (!P || !out) return fail(MF_EINVAL, "null argument");
  const int rc = ensure_uploaded(P);
  if (rc) return rc;
  out[0] = P->sub_f.ncls;
  out[1] = P->sub_f.nsub;
  out[2] = P->sub_s.ncls;
  out[3] = P->sub_s.nsub;
  return MF_OK;
}

int mf_set_class_tuning(mf_plan *P, int32_t n_class, const int32_t *params) {
  if (!P) return fail(MF_EINVAL, "null plan");
  const int32_t nc = P->hp.height + 1;
  if (n_class == 0) {
    P->ctune.clear();
  } else {
    if (n_class != nc || !params)
      return fail(MF_EINVAL, "expected " + std::to_string(nc) + " classes of 5 values");
    std::vector<mf::Tuning> ct(nc, P->tune);
    for (int32_t l = 0; l < nc; ++l) {
      const int32_t *q = params + 5 * l;
      const int32_t smax = q[0], nb = q[1], fused = q[2], tile = q[3], pers = q[4];
      if (smax < 1) return fail(MF_EINVAL, "small_max_m must be >= 1 (class " + std::to_string(l) + ")");
      if (nb != 16 && nb != 32 && nb != 64) return fail(MF_EINVAL, "nb must be 16, 32 or 64");
      if (fused < 0) return fail(MF_EINVAL, "fused_max_m must be >= 0");
      if (tile != 32 && tile != 64) return fail(MF_EINVAL, "tile must be 32 or 64");
      if (pers != 0 && pers != 1) return fail(MF_EINVAL, "persistent must be 0 or 1");
      ct[l].small_max_m = smax;
      ct[l].nb = nb;
      ct[l].fused_max_m = std::min(fused, mf::FP_MAXM);
      ct[l].tile = tile;
      ct[l].persistent = pers;
    }
    P->ctune = ct;
  }
  P->uploaded = false;
  P->factored = false;
  P->drop_graphs();
  return MF_OK;
}

int mf_factor(mf_plan *P, const double *elem_mats, int32_t precision, void *hip_stream) {
  if (!P || !elem_mats) return fail(MF_EINVAL, "null plan or element matrices");
  if (precision != MF_FP64 && precision != MF_SCHUR_FP32 && precision != MF_SCHUR_BF16)
    return fail(MF_EINVAL, "unknown precision " + std::to_string(precision));
  int rc = ensure_uploaded(P);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  P->factored = false;
  GraphKey key;
  key.p0 = elem_mats;
  key.a = precision;
  rc = run_graphed(P, P->g_factor, 2, P->g_factor_next, key, s,
                   [&](hipStream_t st) { return launch_factor(P, elem_mats, precision, st); });
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(P->h_status, P->d_status, mf::kStatusWords * sizeof(int),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (P->h_status[mf::kStatusAbort])
    return fail(MF_EHIP, "a device-side wait of the factorization exceeded its limit; the "
                         "launch was abandoned and the plan holds no valid factor");
  if (P->h_status[0]) return fail(MF_EZERO_PIVOT, pivot_message(P, P->h_status[1], P->h_status[2]));
  P->factored = true;
  return MF_OK;
}

int mf_solve(mf_plan *P, const double *b, double *x, int32_t nrhs, int32_t transpose,
             void *hip_stream) {
  if (!P || !b || !x) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1) return fail(MF_EINVAL, "nrhs must be >= 1");
  if (transpose != 0 && transpose != 1) return fail(MF_EINVAL, "transpose must be 0 or 1");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  int rc;
  if ((rc = grow(P, P->d_ycb, P->ycb_cap, ycb_doubles(P, nrhs))))
    return rc;
  GraphKey key;
  key.p0 = b;
  key.p1 = x;
  key.a = nrhs;
  key.b = transpose;
  return run_graphed(P, P->g_solve, 4, P->g_solve_next, key, (hipStream_t)hip_stream,
                     [&](hipStream_t st) { return launch_solve(P, b, x, nrhs, transpose != 0, st, P->d_ycb); });
}

int mf_solve_noalloc(mf_plan *P, const double *b, double *x, int32_t nrhs, int32_t transpose,
                     void *hip_stream) {
  if (!P || !b || !x) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1) return fail(MF_EINVAL, "nrhs must be >= 1");
  if (transpose != 0 && transpose != 1) return fail(MF_EINVAL, "transpose must be 0 or 1");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  const int64_t need = (int64_t)ycb_doubles(P, nrhs);
  if (need > (int64_t)MF_NOALLOC_SCRATCH_DOUBLES)
    return fail(MF_EINVAL, "mf_solve_noalloc needs " + std::to_string(need) +
                               " doubles of scratch ((sum of contribution-block widths " +
                               std::to_string(P->hp.sum_c) + " + chunked-solve rows " +
                               std::to_string(P->chunk_ws_rows) + ") x nrhs " +
                               std::to_string(nrhs) + "), above its limit of " +
                               std::to_string((int64_t)MF_NOALLOC_SCRATCH_DOUBLES));
  double *ycb = nullptr;
  int rc;
  if ((rc = scratch_address(&ycb))) return rc;
  // the same kernels as mf_solve, launched eagerly (no graph: instantiating one allocates), and
  // without the per-launch timing events of a profiled plan
  const bool prof = P->prof.on;
  P->prof.on = false;
  rc = launch_solve(P, b, x, nrhs, transpose != 0, (hipStream_t)hip_stream, ycb);
  P->prof.on = prof;
  return rc;
}

int mf_residual(mf_plan *P, const double *elem_mats, const double *x, const double *b,
                double *r, int32_t nrhs, void *hip_stream) {
  if (!P || !elem_mats || !x || !b || !r) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1) return fail(MF_EINVAL, "nrhs must be >= 1");
  int rc = ensure_uploaded(P);
  if (rc) return rc;
  const mf::HostPlan &H = P->hp;
  const int64_t tot = H.n * nrhs;
  hipLaunchKernelGGL(mf::k_residual, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     (hipStream_t)hip_stream, P->d_nptr, P->d_nelem, P->d_conn, elem_mats, H.npe,
                     H.n, x, b, r, nrhs, (double *)nullptr);
  HIPCHK(hipGetLastError());
  return MF_OK;
}

// The refinement loop from x = the direct solution: residual, norms, corrections.
// check_status: the factorization's pivot status is published to h_status with the first
// residual's norms and checked after that synchronization (no separate wait for it).
static int refine_loop(mf_plan *P, const double *elem_mats, const double *b, double *x,
                       int32_t nrhs, double tol, int32_t max_it, int32_t *its, double *relres,
                       void *hip_stream, bool check_status = false, bool b_ready = false) {
  hipStream_t s = (hipStream_t)hip_stream;
  const mf::HostPlan &H = P->hp;
  const int64_t n = H.n;
  const size_t nn = (size_t)n * nrhs;
  const NormLayout NL = norm_layout(n, nrhs);
  int rc;
  if ((rc = grow(P, P->d_work, P->work_cap, 2 * nn + NL.r_parts + NL.b_parts))) return rc;
  double *r = P->d_work, *dx = P->d_work + nn;
  double *rpart = P->d_work + 2 * nn, *bpart = rpart + NL.r_parts;
  std::vector<double> bn, rn;
  double rr = 0.0;
  for (int32_t it = 0;; ++it) {
    hipLaunchKernelGGL(mf::k_residual, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                       P->d_nptr, P->d_nelem, P->d_conn, elem_mats, H.npe, n, x, b, r, nrhs,
                       NL.fused ? rpart : (double *)nullptr);
    if (!NL.fused)
      hipLaunchKernelGGL(mf::k_colsq_partial, dim3((unsigned)NL.r_blocks), dim3(256), 0, s, r, n,
                         nrhs, kNormRows, rpart);
    if (it == 0 && !b_ready)
      hipLaunchKernelGGL(mf::k_colsq_partial, dim3((unsigned)NL.b_blocks), dim3(256), 0, s, b, n,
                         nrhs, kNormRows, bpart);
    HIPCHK(hipGetLastError());
    if ((rc = read_norms(P, NL, rpart, nrhs, s, it == 0, rn, bn, check_status && it == 0)))
      return rc;
    if (check_status && it == 0 && P->h_status[mf::kStatusAbort]) {
      P->factored = false;
      return fail(MF_EHIP, "a device-side wait of the factorization exceeded its limit; the "
                           "launch was abandoned and the plan holds no valid factor");
    }
    if (check_status && it == 0 && P->h_status[0]) {
      P->factored = false;
      return fail(MF_EZERO_PIVOT, pivot_message(P, P->h_status[1], P->h_status[2]));
    }
    rr = 0.0;
    for (int c = 0; c < nrhs; ++c) {
      const double q = bn[c] > 0 ? rn[c] / bn[c] : (rn[c] > 0 ? INFINITY : 0.0);
      rr = std::max(rr, std::isnan(q) ? INFINITY : q);
    }
    if (its) *its = it;
    if (relres) *relres = rr;
    if (rr <= tol) return MF_OK;
    if (it >= max_it) break;
    if ((rc = mf_solve(P, r, dx, nrhs, 0, hip_stream))) return rc;
    hipLaunchKernelGGL(mf::k_axpy, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, x, dx,
                       (int64_t)nn);
    HIPCHK(hipGetLastError());
  }
  char buf[160];
  std::snprintf(buf, sizeof buf, "refinement stopped after %d corrections at relres %.3e > tol %.3e",
                max_it, rr, tol);
  return fail(MF_ENOCONV, buf);
}

int mf_refine(mf_plan *P, const double *elem_mats, const double *b, double *x,
              int32_t nrhs, double tol, int32_t max_it, int32_t *its, double *relres,
              void *hip_stream) {
  if (!P || !elem_mats || !b || !x) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1 || max_it < 0 || !(tol >= 0)) return fail(MF_EINVAL, "bad nrhs, max_it or tol");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  int rc;
  if ((rc = mf_solve(P, b, x, nrhs, 0, hip_stream))) return rc;
  return refine_loop(P, elem_mats, b, x, nrhs, tol, max_it, its, relres, hip_stream);
}

int mf_refine_gmres(mf_plan *P, const double *elem_mats, const double *b, double *x,
                    int32_t nrhs, double tol, int32_t max_it, int32_t restart, int32_t *its,
                    double *relres, void *hip_stream) {
  if (!P || !elem_mats || !b || !x) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1 || max_it < 0 || !(tol >= 0)) return fail(MF_EINVAL, "bad nrhs, max_it or tol");
  if (restart < 1 || restart > 64) return fail(MF_EINVAL, "restart must be in 1..64");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  hipStream_t s = (hipStream_t)hip_stream;
  const mf::HostPlan &H = P->hp;
  const int64_t n = H.n;
  const int m = restart;
  const size_t nn = (size_t)n * nrhs;
  const NormLayout NL = norm_layout(n, nrhs);
  const int64_t dblocks = std::max<int64_t>(1, (n + kNormRows - 1) / kNormRows);
  const size_t ndots = (size_t)dblocks * (m + 1) * nrhs;
  const size_t total = (size_t)(2 * m + 3) * nn + ndots + NL.r_parts + NL.b_parts + (size_t)(m + 1) * nrhs;
  int rc;
  if ((rc = grow(P, P->d_kry, P->kry_cap, total))) return rc;
  if ((rc = grow(P, P->d_ycb, P->ycb_cap, ycb_doubles(P, nrhs)))) return rc;
  const size_t hneed = std::max(ndots, (size_t)(m + 1) * nrhs) + (size_t)(m + 1) * nrhs;
  if (P->hkry_cap < hneed) {
    if (P->h_kry) (void)hipHostFree(P->h_kry);
    P->h_kry = nullptr;
    P->hkry_cap = 0;
    HIPCHK(hipHostMalloc((void **)&P->h_kry, hneed * sizeof(double), hipHostMallocDefault));
    P->hkry_cap = hneed;
  }
  double *V = P->d_kry;                       // m + 1 basis blocks
  double *Z = V + (size_t)(m + 1) * nn;       // m preconditioned basis blocks
  double *t = Z + (size_t)m * nn;             // -A z
  double *zero = t + nn;
  double *dpart = zero + nn;
  double *rpart = dpart + ndots, *bpart = rpart + NL.r_parts;
  double *coef = bpart + NL.b_parts;
  double *h_dots = P->h_kry, *h_coef = P->h_kry + std::max(ndots, (size_t)(m + 1) * nrhs);
  HIPCHK(hipMemsetAsync(zero, 0, nn * sizeof(double), s));
  const unsigned gblocks = (unsigned)((nn + 255) / 256);
  auto upload = [&](size_t count) -> int {
    HIPCHK(hipMemcpyAsync(coef, h_coef, count * sizeof(double), hipMemcpyHostToDevice, s));
    return MF_OK;
  };
  // sums of the partial column dots of t with V_0 .. V_{nv-1}: d[i * nrhs + c]
  auto dots = [&](int nv, std::vector<double> &d) -> int {
    hipLaunchKernelGGL(mf::k_coldots_partial, dim3((unsigned)dblocks, (unsigned)nv), dim3(256), 0, s,
                       V, (int64_t)nn, t, n, nrhs, kNormRows, dpart);
    HIPCHK(hipGetLastError());
    const size_t cnt = (size_t)dblocks * nv * nrhs;
    HIPCHK(hipMemcpyAsync(h_dots, dpart, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    d.assign((size_t)nv * nrhs, 0.0);
    for (int64_t bl = 0; bl < dblocks; ++bl)
      for (size_t q = 0; q < (size_t)nv * nrhs; ++q) d[q] += h_dots[bl * nv * nrhs + q];
    return MF_OK;
  };
  // x0 = M^-1 b with the stored (possibly narrow-Schur) factors
  if ((rc = launch_solve(P, b, x, nrhs, false, s, P->d_ycb))) return rc;
  std::vector<double> bn, rn, d, Hm, cs, sn, g, y;
  double rr = INFINITY;
  int32_t done_its = 0;
  for (int outer = 0;; ++outer) {
    // the true FP64 residual r = b - A x, into V_0, and its column norms
    hipLaunchKernelGGL(mf::k_residual, dim3(gblocks), dim3(256), 0, s, P->d_nptr, P->d_nelem,
                       P->d_conn, elem_mats, H.npe, n, x, b, V, nrhs,
                       NL.fused ? rpart : (double *)nullptr);
    if (!NL.fused)
      hipLaunchKernelGGL(mf::k_colsq_partial, dim3((unsigned)NL.r_blocks), dim3(256), 0, s, V, n,
                         nrhs, kNormRows, rpart);
    if (outer == 0)
      hipLaunchKernelGGL(mf::k_colsq_partial, dim3((unsigned)NL.b_blocks), dim3(256), 0, s, b, n,
                         nrhs, kNormRows, bpart);
    HIPCHK(hipGetLastError());
    if ((rc = read_norms(P, NL, rpart, nrhs, s, outer == 0, rn, bn))) return rc;
    rr = 0.0;
    for (int c = 0; c < nrhs; ++c) {
      const double q = bn[c] > 0 ? rn[c] / bn[c] : (rn[c] > 0 ? INFINITY : 0.0);
      rr = std::max(rr, std::isnan(q) ? INFINITY : q);
    }
    if (its) *its = done_its;
    if (relres) *relres = rr;
    if (rr <= tol) return MF_OK;
    if (done_its >= max_it || !std::isfinite(rr)) break;
    // V_0 = r / ||r|| per column; Givens-rotated Hessenberg H (column-major per column c)
    for (int c = 0; c < nrhs; ++c) h_coef[c] = rn[c] > 0 ? 1.0 / rn[c] : 0.0;
    if ((rc = upload((size_t)nrhs))) return rc;
    hipLaunchKernelGGL(mf::k_scale_cols, dim3(gblocks), dim3(256), 0, s, V, V, coef, n, nrhs);
    Hm.assign((size_t)(m + 1) * m * nrhs, 0.0);
    cs.assign((size_t)m * nrhs, 1.0);
    sn.assign((size_t)m * nrhs, 0.0);
    g.assign((size_t)(m + 1) * nrhs, 0.0);
    for (int c = 0; c < nrhs; ++c) g[c] = rn[c];
    auto h = [&](int i, int j, int c) -> double & { return Hm[((size_t)j * (m + 1) + i) * nrhs + c]; };
    int j = 0;
    while (j < m && done_its < max_it) {
      double *Vj = V + (size_t)j * nn, *Zj = Z + (size_t)j * nn;
      if ((rc = launch_solve(P, Vj, Zj, nrhs, false, s, P->d_ycb))) return rc;
      hipLaunchKernelGGL(mf::k_residual, dim3(gblocks), dim3(256), 0, s, P->d_nptr, P->d_nelem,
                         P->d_conn, elem_mats, H.npe, n, Zj, zero, t, nrhs, (double *)nullptr);
      HIPCHK(hipGetLastError());
      // w = A z_j = -t, orthogonalised against V_0 .. V_j by classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2; ++pass) {
        if ((rc = dots(j + 1, d))) return rc;       // d_i = <t, V_i> = -<w, V_i>
        for (int i = 0; i <= j; ++i)
          for (int c = 0; c < nrhs; ++c) {
            h(i, j, c) -= d[(size_t)i * nrhs + c];
            h_coef[(size_t)i * nrhs + c] = -d[(size_t)i * nrhs + c];
          }
        if ((rc = upload((size_t)(j + 1) * nrhs))) return rc;
        hipLaunchKernelGGL(mf::k_combine, dim3(gblocks), dim3(256), 0, s, t, V, (int64_t)nn, j + 1,
                           coef, n, nrhs);
      }
      hipLaunchKernelGGL(mf::k_colsq_partial, dim3((unsigned)NL.b_blocks), dim3(256), 0, s, t, n,
                         nrhs, kNormRows, dpart);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(h_dots, dpart, (size_t)NL.b_blocks * nrhs * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      std::vector<double> wn(nrhs, 0.0);
      for (int64_t bl = 0; bl < NL.b_blocks; ++bl)
        for (int c = 0; c < nrhs; ++c) wn[c] += h_dots[bl * nrhs + c];
      double est = 0.0;
      for (int c = 0; c < nrhs; ++c) {
        wn[c] = std::sqrt(wn[c]);
        h(j + 1, j, c) = wn[c];
        h_coef[c] = wn[c] > 0 ? -1.0 / wn[c] : 0.0;       // V_{j+1} = w / ||w|| = -t / ||t||
        // the column's earlier rotations, then a new one that zeroes h(j+1, j)
        for (int i = 0; i < j; ++i) {
          const double a = h(i, j, c), bb = h(i + 1, j, c);
          const double ci = cs[(size_t)i * nrhs + c], si = sn[(size_t)i * nrhs + c];
          h(i, j, c) = ci * a + si * bb;
          h(i + 1, j, c) = -si * a + ci * bb;
        }
        const double a = h(j, j, c), bb = h(j + 1, j, c), r = std::hypot(a, bb);
        const double cj = r > 0 ? a / r : 1.0, sj = r > 0 ? bb / r : 0.0;
        cs[(size_t)j * nrhs + c] = cj;
        sn[(size_t)j * nrhs + c] = sj;
        h(j, j, c) = r;
        h(j + 1, j, c) = 0.0;
        const double gj = g[(size_t)j * nrhs + c];
        g[(size_t)j * nrhs + c] = cj * gj;
        g[(size_t)(j + 1) * nrhs + c] = -sj * gj;
        const double q = bn[c] > 0 ? std::fabs(g[(size_t)(j + 1) * nrhs + c]) / bn[c] : 0.0;
        est = std::max(est, q);
      }
      if ((rc = upload((size_t)nrhs))) return rc;
      hipLaunchKernelGGL(mf::k_scale_cols, dim3(gblocks), dim3(256), 0, s, V + (size_t)(j + 1) * nn,
                         t, coef, n, nrhs);
      HIPCHK(hipGetLastError());
      ++j;
      ++done_its;
      if (est <= 0.5 * tol) break;                       // the least-squares residual suffices
    }
    // y = R^-1 g per column (back substitution), then x += Z y
    y.assign((size_t)j * nrhs, 0.0);
    for (int c = 0; c < nrhs; ++c)
      for (int i = j - 1; i >= 0; --i) {
        double v = g[(size_t)i * nrhs + c];
        for (int k = i + 1; k < j; ++k) v -= h(i, k, c) * y[(size_t)k * nrhs + c];
        const double dg = h(i, i, c);
        y[(size_t)i * nrhs + c] = dg != 0.0 ? v / dg : 0.0;
      }
    std::memcpy(h_coef, y.data(), y.size() * sizeof(double));
    if ((rc = upload(y.size()))) return rc;
    hipLaunchKernelGGL(mf::k_combine, dim3(gblocks), dim3(256), 0, s, x, Z, (int64_t)nn, j, coef, n,
                       nrhs);
    HIPCHK(hipGetLastError());
  }
  char buf[160];
  std::snprintf(buf, sizeof buf, "GMRES refinement stopped after %d preconditioned steps at relres %.3e > tol %.3e",
                done_its, rr, tol);
  return fail(MF_ENOCONV, buf);
}

int mf_factor_refine(mf_plan *P, const double *elem_mats, int32_t precision, const double *b,
                     double *x, int32_t nrhs, double tol, int32_t max_it, int32_t *its,
                     double *relres, void *hip_stream) {
  if (!P || !elem_mats || !b || !x) return fail(MF_EINVAL, "null argument");
  if (precision != MF_FP64 && precision != MF_SCHUR_FP32 && precision != MF_SCHUR_BF16)
    return fail(MF_EINVAL, "unknown precision " + std::to_string(precision));
  if (nrhs < 1 || max_it < 0 || !(tol >= 0)) return fail(MF_EINVAL, "bad nrhs, max_it or tol");
  int rc = ensure_uploaded(P);
  if (rc) return rc;
  if ((rc = grow(P, P->d_ycb, P->ycb_cap, ycb_doubles(P, nrhs))))
    return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  P->factored = false;
  // launched eagerly: the two streams overlap only when each launch is issued to its own
  // stream (a captured graph of the same fork/join replays its branches one after the other
  // on this platform -- measured: no overlap, 3 % slower than the sequential calls)
  {
    // the norms of b do not depend on the factorization: their partial sums run first, on the
    // caller's stream, in the launch that also clears the status words and counters (the first
    // launches of a step find the device idle while the host issues them; a second stream
    // would need an event and a wait, two more host calls)
    const int64_t n = P->hp.n;
    const size_t nn = (size_t)n * nrhs;
    const NormLayout NL = norm_layout(n, nrhs);
    if ((rc = grow(P, P->d_work, P->work_cap, 2 * nn + NL.r_parts + NL.b_parts))) return rc;
    hipLaunchKernelGGL(mf::k_refine_prologue, dim3((unsigned)NL.b_blocks), dim3(256), 0, s, b, n,
                       nrhs, kNormRows, P->d_work + 2 * nn + NL.r_parts, P->d_status, P->d_ccnt,
                       P->n_ccnt);
    HIPCHK(hipGetLastError());
  }
  if ((rc = launch_factor_solve(P, elem_mats, precision, b, x, nrhs, s, true))) return rc;
  // the pivot status travels with the first residual's norms (k_norm_publish): one
  // synchronization for both
  P->factored = true;     // withdrawn by refine_loop if the status reports a bad pivot
  return refine_loop(P, elem_mats, b, x, nrhs, tol, max_it, its, relres, hip_stream, true, true);
}

int mf_elem_grad(mf_plan *P, const double *lam, const double *u, int32_t nrhs, double *gK,
                 void *hip_stream) {
  if (!P || !lam || !u || !gK) return fail(MF_EINVAL, "null argument");
  if (nrhs < 1) return fail(MF_EINVAL, "nrhs must be >= 1");
  int rc = ensure_uploaded(P);
  if (rc) return rc;
  const mf::HostPlan &H = P->hp;
  const int64_t tot = H.n_elem * H.npe * H.npe;
  hipLaunchKernelGGL(mf::k_elem_grad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     (hipStream_t)hip_stream, P->d_conn, H.n_elem, H.npe, lam, u, nrhs, gK);
  HIPCHK(hipGetLastError());
  return MF_OK;
}

int mf_export_factors(const mf_plan *P, double *L, double *U) {
  if (!P || !L || !U) return fail(MF_EINVAL, "null argument");
  if (!P->factored) return fail(MF_ESTATE, "no valid factorization: call mf_factor first");
  const mf::HostPlan &H = P->hp;
  std::vector<double> st;
  try {
    st.resize(H.store_doubles);
  } catch (const std::bad_alloc &) {
    return fail(MF_ENOMEM, "cannot allocate host copy of the factors");
  }
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(st.data(), P->d_store, H.store_doubles * sizeof(double), hipMemcpyDeviceToHost));
  int64_t off = 0;
  for (int64_t f = 0; f < H.F; ++f) {
    const mf::FrontDesc &d = H.desc[f];
    const double *Fm = st.data() + d.store;
    double *Lf = L + off, *Uf = U + off;
    for (int32_t i = 0; i < d.m; ++i)
      for (int32_t p = 0; p < d.k; ++p) {
        Lf[(int64_t)i * d.k + p] = i >= p ? Fm[(int64_t)i * d.m + p] : 0.0;
        Uf[(int64_t)p * d.m + i] = i > p ? Fm[(int64_t)p * d.m + i] : (i == p ? 1.0 : 0.0);
      }
    off += (int64_t)d.m * d.k;
  }
  return MF_OK;
}

int mf_autotune(mf_plan *P, const double *elem_mats, int32_t precision, int32_t reps,
                void *hip_stream, char *report, int64_t cap, int64_t *needed) {
  if (!P || !elem_mats) return fail(MF_EINVAL, "null plan or element matrices");
  if (reps < 1) return fail(MF_EINVAL, "reps must be >= 1");
  int rc = ensure_uploaded(P);
  if (rc) return rc;
  // what the workload contains decides which knobs can matter
  bool mid = false, wide = false;
  for (int64_t f = 0; f < P->hp.F; ++f) {
    const int32_t m = P->hp.desc[f].m;
    if (m > 64 && m <= 128) mid = true;
    if (m > 128) wide = true;
  }
  std::vector<mf::Tuning> cands;
  const mf::Tuning base = P->tune;
  for (int32_t pers : {1, 0})
    for (int32_t tile : {64, 32})
      for (int32_t fused : {mf::FP_MAXM, 0})
        for (int32_t nb : {32, 64})
          for (int32_t smax : {128, 64}) {
            // the persistent route has no fused form and a fixed panel width
            if (pers && (fused != mf::FP_MAXM || nb != 32)) continue;
            if (!wide && (tile != 64 || fused != mf::FP_MAXM || nb != 32)) continue;
            if (fused == mf::FP_MAXM && nb != 32 && P->hp.max_m <= mf::FP_MAXM) continue;
            if (!mid && smax != 128) continue;
            mf::Tuning t = base;
            t.persistent = pers;
            t.tile = tile;
            t.fused_max_m = pers ? 0 : fused;
            t.nb = nb;
            t.small_max_m = smax;
            cands.push_back(t);
          }
  const size_t ncls = P->hp.levels.size();
  // host-clock median of `reps` factorizations under the plan's current schedule
  auto timed = [&](double &med) -> int {
    int r;
    P->uploaded = false;
    P->factored = false;
    if ((r = mf_factor(P, elem_mats, precision, hip_stream))) return r;   // warm-up + capture
    std::vector<double> ts;
    for (int32_t i = 0; i < reps; ++i) {
      const auto t0 = std::chrono::steady_clock::now();
      if ((r = mf_factor(P, elem_mats, precision, hip_stream))) return r;
      ts.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    std::sort(ts.begin(), ts.end());
    med = ts[ts.size() / 2];
    return MF_OK;
  };
  // per candidate: the whole factorization (host clock), then each class's launches timed with
  // device events on the stream they run on (summed over the class, averaged over reps)
  std::vector<double> tglob(cands.size());
  std::vector<std::vector<double>> tcls(cands.size(), std::vector<double>(ncls, 0.0));
  const Profiler saved = P->prof;
  P->prof = Profiler();
  for (size_t c = 0; c < cands.size(); ++c) {
    P->tune = cands[c];
    P->ctune.clear();
    if ((rc = timed(tglob[c]))) return rc;
    P->prof.on = true;
    for (int32_t i = 0; i < reps; ++i)
      if ((rc = mf_factor(P, elem_mats, precision, hip_stream))) return rc;
    for (auto &r : P->prof.recs) {
      float ms = 0;
      HIPCHK(hipEventSynchronize(r.b));
      HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
      if (r.cls >= 0 && (size_t)r.cls < ncls) tcls[c][r.cls] += ms / reps;
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    P->prof = Profiler();
  }
  P->prof = saved;
  size_t cb = 0;
  for (size_t c = 1; c < cands.size(); ++c)
    if (tglob[c] < tglob[cb]) cb = c;
  // each class takes the candidate under which its own launches were fastest
  std::vector<size_t> pick(ncls, cb);
  for (size_t l = 0; l < ncls; ++l)
    for (size_t c = 0; c < cands.size(); ++c)
      if (tcls[c][l] < tcls[pick[l]][l]) pick[l] = c;
  P->tune = cands[cb];
  P->ctune.assign(ncls, cands[cb]);
  for (size_t l = 0; l < ncls; ++l) P->ctune[l] = cands[pick[l]];
  double tmix = 0;
  if ((rc = timed(tmix))) return rc;
  const bool per_class = tmix < tglob[cb];
  if (!per_class) P->ctune.clear();
  P->uploaded = false;
  P->factored = false;
  if ((rc = mf_factor(P, elem_mats, precision, hip_stream))) return rc;
  auto tune_js = [](const mf::Tuning &t) {
    char b[160];
    std::snprintf(b, sizeof b, "\"persistent\": %d, \"tile\": %d, \"fused_max_m\": %d, \"nb\": %d, "
                               "\"small_max_m\": %d", t.persistent, t.tile, t.fused_max_m, t.nb,
                  t.small_max_m);
    return std::string(b);
  };
  std::string js = "{\"candidates\": [";
  for (size_t c = 0; c < cands.size(); ++c) {
    char b[64];
    std::snprintf(b, sizeof b, ", \"ms\": %.4f, \"class_ms\": [", tglob[c]);
    js += (c ? ", {" : "{") + tune_js(cands[c]) + b;
    for (size_t l = 0; l < ncls; ++l) {
      std::snprintf(b, sizeof b, "%s%.4f", l ? ", " : "", tcls[c][l]);
      js += b;
    }
    js += "]}";
  }
  js += "], \"chosen\": {\"mode\": \"";
  js += per_class ? "per_class" : "global";
  {
    char b[160];
    std::snprintf(b, sizeof b, "\", \"ms\": %.4f, \"best_global_ms\": %.4f, \"per_class_ms\": %.4f, ",
                  per_class ? tmix : tglob[cb], tglob[cb], tmix);
    js += b;
  }
  js += tune_js(cands[cb]) + ", \"classes\": [";
  for (size_t l = 0; l < ncls; ++l) {
    char b[48];
    std::snprintf(b, sizeof b, ", \"class_ms\": %.4f}", tcls[pick[l]][l]);
    js += (l ? ", {" : "{") + tune_js(cands[pick[l]]) + b;
  }
  js += "]}}";
  if (needed) *needed = (int64_t)js.size() + 1;
  if (report && cap > 0) {
    const size_t n = std::min<size_t>((size_t)cap - 1, js.size());
    std::memcpy(report, js.data(), n);
    report[n] = 0;
  }
  return MF_OK;
}

int mf_profile(mf_plan *P, int32_t enable) {
  if (!P) return fail(MF_EINVAL, "null plan");
  for (auto &r : P->prof.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  P->prof = Profiler();
  P->prof.on = enable != 0;
  return MF_OK;
}

int mf_profile_report(mf_plan *P, char *buf, int64_t cap, int64_t *needed) {
  if (!P) return fail(MF_EINVAL, "null plan");
  Profiler &pr = P->prof;
  for (auto &r : pr.recs) {
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    pr.ms[r.kind] += ms;
    pr.bytes[r.kind] += r.cost.bytes;
    pr.flops[r.kind] += r.cost.flops;
    pr.launches[r.kind] += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  pr.recs.clear();
  std::string js = "{\"kernels\": [";
  bool first = true;
  for (int k = 0; k < K_COUNT; ++k) {
    if (!pr.launches[k]) continue;
    char line[256];
    std::snprintf(line, sizeof line,
                  "%s{\"name\": \"%s\", \"launches\": %lld, \"ms\": %.6f, \"bytes\": %.6e, \"flops\": %.6e}",
                  first ? "" : ", ", kKindName[k], (long long)pr.launches[k], pr.ms[k], pr.bytes[k],
                  pr.flops[k]);
    js += line;
    first = false;
  }
  js += "]}";
  if (needed) *needed = (int64_t)js.size() + 1;
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>((size_t)cap - 1, js.size());
    std::memcpy(buf, js.data(), n);
    buf[n] = 0;
  }
  return MF_OK;
}

void mf_destroy(mf_plan *P) { delete P; }

}  // extern "C"
