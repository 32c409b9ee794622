// Stage timing with HIP events (pauli_profile_enable / pauli_profile_read).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.h"

namespace pauli {

namespace {
struct Pending {
  int stage;
  hipEvent_t a, b;
  double bytes;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
double g_ms[PAULI_STAGE_COUNT];
int64_t g_launches[PAULI_STAGE_COUNT];
double g_bytes[PAULI_STAGE_COUNT];

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  PAULI_HIP(hipEventCreate(&e));
  return e;
}

void flush_locked() {
  for (auto& p : g_pending) {
    PAULI_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    PAULI_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    g_ms[p.stage] += ms;
    g_launches[p.stage] += 1;
    g_bytes[p.stage] += p.bytes;
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}
}  // namespace

thread_local int g_no_events = 0;
NoEvents::NoEvents() { ++g_no_events; }
NoEvents::~NoEvents() { --g_no_events; }

StageScope::StageScope(int st, hipStream_t str, double by) : stage(st), s(str), bytes(by) {
  // a call that allocates nothing creates no events, nor does a capture
  if (workspace_active() || g_no_events) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  a = take_event();
  PAULI_HIP(hipEventRecord(a, s));
}

void StageScope::stop() {
  if (!a || b) return;
  std::lock_guard<std::mutex> lk(g_mu);
  b = take_event();
  if (hipEventRecord(b, s) != hipSuccess) {
    (void)hipGetLastError();
    g_pool.push_back(b);
    g_pool.push_back(a);
    a = b = nullptr;
  }
}

StageScope::~StageScope() {
  if (!a) return;
  try {
    stop();
  } catch (...) {
    return;
  }
  if (!a || !b) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back({stage, a, b, bytes});
}

}  // namespace pauli

using namespace pauli;

extern "C" {

pauli_status_t pauli_profile_enable(int32_t on) {
  try {
    std::lock_guard<std::mutex> lk(g_mu);
    flush_locked();
    for (int i = 0; i < PAULI_STAGE_COUNT; ++i) {
      g_ms[i] = 0;
      g_launches[i] = 0;
      g_bytes[i] = 0;
    }
    g_on = on != 0;
    return PAULI_OK;
  } catch (...) {
    return PAULI_ERR_DEVICE;
  }
}

pauli_status_t pauli_profile_read(int32_t stage, double* total_ms, int64_t* launches,
                                  double* bytes) {
  if (stage < 0 || stage >= PAULI_STAGE_COUNT) {
    set_error("unknown stage");
    return PAULI_ERR_INVALID;
  }
  try {
    std::lock_guard<std::mutex> lk(g_mu);
    flush_locked();
    if (total_ms) *total_ms = g_ms[stage];
    if (launches) *launches = g_launches[stage];
    if (bytes) *bytes = g_bytes[stage];
    return PAULI_OK;
  } catch (...) {
    return PAULI_ERR_DEVICE;
  }
}

}  // extern "C"
