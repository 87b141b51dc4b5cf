// trace.hpp -- scalar-task trace of the factorization (host analysis of tiny meshes).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

namespace mf {

constexpr int64_t kTraceMaxN = 4096;
constexpr double kTraceMaxTasks = 5e7;

struct TraceSummary {
  int64_t tasks[4] = {0, 0, 0, 0};       // T1 divisions, T2 multiplications, T3 subtractions, T4 assertions
  int32_t fnf_classes = 0;               // classes of the Foata normal form
  int32_t fnf_single_type_classes = 0;   // of those, classes holding a single task type
  int32_t typed_classes = 0;             // classes of the 4-periodic typed schedule
  int32_t levels_order_dependencies = 0; // 1 if every dependency between two fronts' tasks
                                         // goes from a lower or equal front class
};

// Fills `out` and hist[c * 4 + t] = number of tasks of type t (T1, T2, T3, T4) in Foata class c
// (c >= 1; hist has 4 (classes + 1) entries).  Returns an error message or "".
std::string task_trace(const HostPlan &H, TraceSummary &out, std::vector<int64_t> &hist);

}  // namespace mf
