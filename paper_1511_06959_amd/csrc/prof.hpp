// prof.hpp -- event-pair instrumentation of kernel launches, grouped by kernel class.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "../../include/adjns.h"

namespace adjns {

struct ProfState {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[ADJ_PROF_NCLASS];
  size_t used[ADJ_PROF_NCLASS] = {};
};

ProfState& prof_state();

// While profiling is enabled, brackets the launches made during its lifetime with a pair of
// events recorded on the launch stream.
struct ProfScope {
  int cls;
  hipStream_t st;
  bool active;
  ProfScope(int c, hipStream_t s) : cls(c), st(s), active(prof_state().on) {
    if (!active) return;
    ProfState& P = prof_state();
    auto& v = P.ev[cls];
    if (P.used[cls] == v.size()) {
      std::pair<hipEvent_t, hipEvent_t> p;
      if (hipEventCreate(&p.first) != hipSuccess) {
        active = false;
        return;
      }
      if (hipEventCreate(&p.second) != hipSuccess) {
        (void)hipEventDestroy(p.first);
        active = false;
        return;
      }
      v.push_back(p);
    }
    (void)hipEventRecord(v[P.used[cls]].first, st);
  }
  ~ProfScope() {
    if (!active) return;
    ProfState& P = prof_state();
    (void)hipEventRecord(P.ev[cls][P.used[cls]].second, st);
    ++P.used[cls];
  }
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;
};

}  // namespace adjns
