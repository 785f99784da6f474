// Kernel timing probes: when a probe is enabled, every launch of its kernel
// class is bracketed by a pair of HIP events on the launch stream, and the
// summed elapsed device time can be read back.  Used to measure the achieved
// bandwidth of individual kernels inside a running workload.
#include <vector>

#include "internal.h"

namespace ibs {

namespace {
struct ProbeState {
  bool on[PR_COUNT] = {};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[PR_COUNT];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
};
ProbeState g_probe;
}  // namespace

int probe_begin(int id, hipStream_t s) {
  if (id < 0 || id >= PR_COUNT || !g_probe.on[id]) return -1;
  std::pair<hipEvent_t, hipEvent_t> e;
  if (!g_probe.pool.empty()) {
    e = g_probe.pool.back();
    g_probe.pool.pop_back();
  } else {
    if (hipEventCreate(&e.first) != hipSuccess) return -1;
    if (hipEventCreate(&e.second) != hipSuccess) return -1;
  }
  hipEventRecord(e.first, s);
  g_probe.ev[id].push_back(e);
  return (int)g_probe.ev[id].size() - 1;
}

void probe_end(int id, int slot, hipStream_t s) {
  if (slot < 0) return;
  hipEventRecord(g_probe.ev[id][slot].second, s);
}

void probe_enable(int id, bool on) {
  if (id >= 0 && id < PR_COUNT) g_probe.on[id] = on;
}

// Sum of the recorded launch durations (ms); waits for the events.
hipError_t probe_read(int id, long long *count, double *ms, bool reset) {
  *count = 0;
  *ms = 0.0;
  if (id < 0 || id >= PR_COUNT) return hipErrorInvalidValue;
  double tot = 0.0;
  for (auto &e : g_probe.ev[id]) {
    hipError_t r = hipEventSynchronize(e.second);
    if (r != hipSuccess) return r;
    float t = 0.f;
    r = hipEventElapsedTime(&t, e.first, e.second);
    if (r != hipSuccess) return r;
    tot += t;
  }
  *count = (long long)g_probe.ev[id].size();
  *ms = tot;
  if (reset) {
    for (auto &e : g_probe.ev[id]) g_probe.pool.push_back(e);
    g_probe.ev[id].clear();
  }
  return hipSuccess;
}

}  // namespace ibs
