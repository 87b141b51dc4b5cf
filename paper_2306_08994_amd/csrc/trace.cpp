// trace.cpp -- the scalar-task trace of the factorization and its Foata classes (host).
//
// The tasks of Sec. 3 (division T1, multiplication T2, subtraction T3 per pivot and front
// entry, assertion T4 per global entry) with the dependencies J1..J4, scheduled in Foata normal
// form (Sec. 3.3): every task in the earliest class after all of its predecessors.  The
// dependencies are never materialised: tasks are visited in the order of the paper's sequential
// algorithm (Table 2: class by class, the fronts of a class in order, pivots in order), and
// every predecessor of a task is either an assertion of an entry whose subtractions are all
// issued already (the pivot row and column entries are final when their pivot is reached) or
// the previous subtraction into the same entry, so one running class per global entry carries
// the whole chain of J3 and J4.
// Alongside the Foata classes the same pass places every task in the earliest class after its
// predecessors that is congruent to its type (T4: 1, T1: 2, T2: 3, T3: 0 mod 4), the
// 4-periodic structure of Sec. 3.3, which is a valid schedule by construction.
#include "trace.hpp"

#include <algorithm>
#include <string>
#include <vector>

namespace mf {

namespace {
inline int32_t typed(int32_t v, int residue) {
  while (v % 4 != residue) ++v;
  return v;
}
}  // namespace

std::string task_trace(const HostPlan &H, TraceSummary &out, std::vector<int64_t> &hist) {
  out = TraceSummary();
  hist.clear();
  if (H.n > kTraceMaxN) return "the scalar trace is for meshes of at most " + std::to_string(kTraceMaxN) + " unknowns";
  double tasks = (double)H.n * H.n;
  for (int64_t f = 0; f < H.F; ++f) {
    const int64_t m = H.front_ptr[f + 1] - H.front_ptr[f];
    for (int64_t p = 0; p < H.npiv[f]; ++p) {
      const double r = (double)(m - p - 1);
      tasks += r + 2 * r * r;
    }
  }
  if (tasks > kTraceMaxTasks) return "the scalar trace would hold more than 5e7 tasks";
  const int64_t n = H.n;
  // per global entry: class of its last subtraction (0 if none), in the Foata and the typed
  // schedules, and the front that issued it (for the front-class check)
  std::vector<int32_t> last(n * n, 0), last_t(n * n, 0), last_f(n * n, -1);
  auto c4 = [&](int64_t e) { return last[e] + 1; };
  auto c4t = [&](int64_t e) { return typed(last_t[e] + 1, 1); };
  auto bump = [&](int32_t cls, int type) {
    const size_t need = (size_t)cls * 4 + 4;
    if (hist.size() < need) hist.resize(need, 0);
    hist[(size_t)cls * 4 + type] += 1;
  };
  out.levels_order_dependencies = 1;
  std::vector<int32_t> c1(H.max_m), c1t(H.max_m);
  std::vector<int64_t> order(H.F);
  for (int64_t f = 0; f < H.F; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return H.level[a] < H.level[b]; });
  for (const int64_t f : order) {
    const int32_t *idx = H.front_idx.data() + H.front_ptr[f];
    const int64_t m = H.front_ptr[f + 1] - H.front_ptr[f];
    for (int64_t p = 0; p < H.npiv[f]; ++p) {
      const int64_t z = idx[p];
      for (int64_t j = p + 1; j < m; ++j) {   // T1(f, z, y): J1
        const int64_t y = idx[j];
        c1[j] = 1 + std::max(c4(z * n + z), c4(z * n + y));
        c1t[j] = typed(1 + std::max(c4t(z * n + z), c4t(z * n + y)), 2);
        bump(c1[j], 0);
        out.tasks[0] += 1;
      }
      for (int64_t i = p + 1; i < m; ++i) {
        const int64_t x = idx[i];
        const int32_t a4 = c4(x * n + z), a4t = c4t(x * n + z);
        for (int64_t j = p + 1; j < m; ++j) {
          const int64_t y = idx[j], e = x * n + y;
          const int32_t k2 = 1 + std::max(c1[j], a4);                 // T2: J2
          const int32_t k2t = typed(1 + std::max(c1t[j], a4t), 3);
          const int32_t k3 = 1 + std::max(k2, last[e]);              // T3: J3
          const int32_t k3t = typed(1 + std::max(k2t, last_t[e]), 0);
          bump(k2, 1);
          bump(k3, 2);
          if (last_f[e] >= 0 && H.level[last_f[e]] > H.level[f]) out.levels_order_dependencies = 0;
          last[e] = k3;
          last_t[e] = k3t;
          last_f[e] = (int32_t)f;
          out.tasks[1] += 1;
          out.tasks[2] += 1;
        }
      }
    }
  }
  for (int64_t e = 0; e < n * n; ++e) {      // T4(x, y): J4
    bump(c4(e), 3);
    out.tasks[3] += 1;
    out.typed_classes = std::max(out.typed_classes, c4t(e));
    out.fnf_classes = std::max(out.fnf_classes, c4(e));
  }
  for (int64_t e = 0; e < n * n; ++e) out.typed_classes = std::max(out.typed_classes, last_t[e]);
  const int32_t ncls = (int32_t)(hist.size() / 4) - 1;   // classes 1..ncls
  out.fnf_classes = std::max(out.fnf_classes, ncls);
  for (int32_t c = 1; c <= ncls; ++c) {
    int types = 0;
    for (int t = 0; t < 4; ++t) types += hist[(size_t)c * 4 + t] > 0;
    out.fnf_single_type_classes += types == 1;
  }
  return "";
}

}  // namespace mf
