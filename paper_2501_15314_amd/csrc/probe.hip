// Kernel timing probes: when a probe is enabled on a handle, every launch of
// its kernel class made by that handle is bracketed by a pair of HIP events
// on the launch stream, and the summed elapsed device time can be read back.
// Used to measure the achieved bandwidth of individual kernels inside a
// running workload.  Each handle owns its probe state; the entry points of
// the C ABI bind it to the calling thread for the duration of the call, so
// handles on different threads never share probe state.
#include <vector>

#include "internal.h"

namespace ibs {

struct ProbeState {
  bool on[PR_COUNT] = {};
  long long points = 0, band_cells = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[PR_COUNT];
  std::vector<double> bytes[PR_COUNT];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
};

namespace {
thread_local ProbeState *t_probe = nullptr;
// the event pair of a probed launch made through hipExtLaunchKernel, between
// ProbeExt's constructor and the launch that takes it
thread_local std::pair<hipEvent_t, hipEvent_t> t_ext = {nullptr, nullptr};
}  // namespace

ProbeState *probe_new() { return new ProbeState(); }

void probe_free(ProbeState *ps) {
  if (!ps) return;
  for (int id = 0; id < PR_COUNT; ++id)
    for (auto &e : ps->ev[id]) ps->pool.push_back(e);
  for (auto &e : ps->pool) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  delete ps;
}

ProbeState *probe_bind(ProbeState *ps) {
  ProbeState *prev = t_probe;
  t_probe = ps;
  return prev;
}

void probe_set_points(ProbeState *ps, long long K, long long band_cells) {
  if (ps) {
    ps->points = K;
    ps->band_cells = band_cells;
  }
}

long long probe_points() { return t_probe ? t_probe->points : 0; }
long long probe_band_cells() { return t_probe ? t_probe->band_cells : 0; }

static int probe_slot(ProbeState *ps, int id, double bytes) {
  std::pair<hipEvent_t, hipEvent_t> e;
  if (!ps->pool.empty()) {
    e = ps->pool.back();
    ps->pool.pop_back();
  } else {
    if (hipEventCreate(&e.first) != hipSuccess) return -1;
    if (hipEventCreate(&e.second) != hipSuccess) {
      hipEventDestroy(e.first);
      return -1;
    }
  }
  ps->ev[id].push_back(e);
  ps->bytes[id].push_back(bytes);
  return (int)ps->ev[id].size() - 1;
}

int probe_begin(int id, hipStream_t s, double bytes) {
  ProbeState *ps = t_probe;
  if (!ps || id < 0 || id >= PR_COUNT || !ps->on[id]) return -1;
  const int slot = probe_slot(ps, id, bytes);
  if (slot >= 0) hipEventRecord(ps->ev[id][slot].first, s);
  return slot;
}

// A probe whose events the runtime stamps with the kernel's own start and
// end: the launch inside the scope is made with hipExtLaunchKernel and takes
// the pair through probe_ext_take, so short kernels are timed without the
// dispatch latency that events recorded around the launch add.
int probe_ext_begin(int id, double bytes) {
  ProbeState *ps = t_probe;
  t_ext = {nullptr, nullptr};
  if (!ps || id < 0 || id >= PR_COUNT || !ps->on[id]) return -1;
  const int slot = probe_slot(ps, id, bytes);
  if (slot >= 0) t_ext = ps->ev[id][slot];
  return slot;
}
void probe_ext_take(hipEvent_t *start, hipEvent_t *stop) {
  *start = t_ext.first;
  *stop = t_ext.second;
  t_ext = {nullptr, nullptr};
}
void probe_ext_end(int id, int slot, hipStream_t s) {
  ProbeState *ps = t_probe;
  if (slot < 0 || !ps) return;
  if (t_ext.first) {
    // no launch took the pair: record it here (an empty interval)
    hipEventRecord(t_ext.first, s);
    hipEventRecord(t_ext.second, s);
    t_ext = {nullptr, nullptr};
  }
}

void probe_end(int id, int slot, hipStream_t s) {
  ProbeState *ps = t_probe;
  if (slot < 0 || !ps) return;
  hipEventRecord(ps->ev[id][slot].second, s);
}

void probe_enable(ProbeState *ps, int id, bool on) {
  if (ps && id >= 0 && id < PR_COUNT) ps->on[id] = on;
}

// Sum of the recorded launch durations (ms); waits for the events.
hipError_t probe_read(ProbeState *ps, int id, long long *count, double *ms, double *bytes, bool reset) {
  *count = 0;
  *ms = 0.0;
  *bytes = 0.0;
  if (!ps || id < 0 || id >= PR_COUNT) return hipErrorInvalidValue;
  double tot = 0.0;
  for (auto &e : ps->ev[id]) {
    hipError_t r = hipEventSynchronize(e.second);
    if (r != hipSuccess) return r;
    float t = 0.f;
    r = hipEventElapsedTime(&t, e.first, e.second);
    if (r != hipSuccess) return r;
    tot += t;
  }
  *count = (long long)ps->ev[id].size();
  *ms = tot;
  for (double b : ps->bytes[id]) *bytes += b;
  if (reset) {
    for (auto &e : ps->ev[id]) ps->pool.push_back(e);
    ps->ev[id].clear();
    ps->bytes[id].clear();
  }
  return hipSuccess;
}

}  // namespace ibs
