// prof.hpp -- event-pair instrumentation of kernel launches, grouped by kernel class.
#pragma once
#include <hip/hip_ext.h>
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
// events recorded on the launch stream.  A scope made with `single` times exactly one kernel: the
// launch takes the pair (launch_events) and hands it to hipExtLaunchKernel, which stamps the
// kernel's own start and end, so that no host-side gap between launches enters the duration.
struct ProfScope {
  int cls;
  hipStream_t st;
  bool active, single, taken = false;
  ProfScope(int c, hipStream_t s, bool one_kernel = false)
      : cls(c), st(s), active(prof_state().on), single(one_kernel) {
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
    if (!single) (void)hipEventRecord(v[P.used[cls]].first, st);
  }
  bool launch_events(hipEvent_t& start, hipEvent_t& stop) {
    if (!active || !single || taken) return false;
    ProfState& P = prof_state();
    start = P.ev[cls][P.used[cls]].first;
    stop = P.ev[cls][P.used[cls]].second;
    taken = true;
    return true;
  }
  ~ProfScope() {
    if (!active) return;
    ProfState& P = prof_state();
    if (!single) {
      (void)hipEventRecord(P.ev[cls][P.used[cls]].second, st);
      ++P.used[cls];
    } else if (taken) {
      ++P.used[cls];
    }
  }
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;
};

// One kernel launch, timed by the scope's events when profiling is on.
template <typename K, typename... A>
inline void timed_launch(ProfScope& ps, K kernel, dim3 grid, dim3 block, hipStream_t st, A... args) {
  hipEvent_t e0, e1;
  if (ps.launch_events(e0, e1))
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

}  // namespace adjns
