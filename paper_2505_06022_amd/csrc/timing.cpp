// Per-kernel launch timing with HIP events recorded on each launch's own
// stream (measurement support; off unless enabled).
#include <mutex>
#include <utility>
#include <vector>

#include "ccl_internal.h"

namespace ccl {
namespace {

constexpr size_t kMaxRecords = 1 << 20;

struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;                     // free pairs
  std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[CCL_KERNEL_KINDS];   // recorded
};

Timing &timing() {
  static Timing *t = new Timing();
  return *t;
}

}  // namespace

TimedLaunch::TimedLaunch(int kind, hipStream_t s) : kind_(kind), stream_(s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  Timing &t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  if (!t.on || kind < 0 || kind >= CCL_KERNEL_KINDS || t.rec[kind].size() >= kMaxRecords) return;
  if (t.pool.empty()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return;
    }
    t.pool.emplace_back(a, b);
  }
  ev_ = t.pool.back();
  t.pool.pop_back();
  if (hipEventRecord(ev_.first, s) != hipSuccess) {
    t.pool.push_back(ev_);
    return;
  }
  active_ = true;
}

TimedLaunch::~TimedLaunch() {
  if (!active_) return;
  Timing &t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  if (hipEventRecord(ev_.second, stream_) != hipSuccess) {
    t.pool.push_back(ev_);
    return;
  }
  t.rec[kind_].push_back(ev_);
}

}  // namespace ccl

using namespace ccl;

extern "C" ccl_status ccl_timing_enable(int32_t on) {
  clear_error();
  Timing &t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  for (auto &r : t.rec) {
    for (auto &e : r) t.pool.push_back(e);
    r.clear();
  }
  t.on = on != 0;
  return CCL_OK;
}

extern "C" ccl_status ccl_timing_query(int32_t kernel, int64_t *launches, double *total_ms) {
  clear_error();
  if (!launches || !total_ms) return fail(CCL_E_INVALID, "NULL argument");
  if (kernel < 0 || kernel >= CCL_KERNEL_KINDS) return fail(CCL_E_INVALID, "kernel=%d", kernel);
  Timing &t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  double sum = 0.0;
  for (auto &e : t.rec[kernel]) {
    ccl_status st = hip_check(hipEventSynchronize(e.second), "hipEventSynchronize");
    if (st != CCL_OK) return st;
    float ms = 0.0f;
    st = hip_check(hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
    if (st != CCL_OK) return st;
    sum += ms;
  }
  *launches = static_cast<int64_t>(t.rec[kernel].size());
  *total_ms = sum;
  return CCL_OK;
}
