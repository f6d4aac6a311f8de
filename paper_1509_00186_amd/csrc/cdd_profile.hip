// Opt-in stage timing with HIP events recorded on the caller's stream.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "cdd_internal.h"

namespace cdd {

namespace {
std::atomic<int> g_on{0};
std::atomic<unsigned> g_mask{(1u << CDD_NSTAGES) - 1u};  // stages timed while on
std::mutex g_mu;
struct Rec {
  int stage;
  hipEvent_t a, b;
};
std::vector<Rec> g_recs;
}  // namespace

bool profiling() { return g_on.load(std::memory_order_relaxed) != 0; }

int stage_begin(int stage, void* stream, void** token) {
  *token = nullptr;
  if (!profiling() || !((g_mask.load(std::memory_order_relaxed) >> stage) & 1u)) return 0;
  hipEvent_t a;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return (int)e;
  e = hipEventRecord(a, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    return (int)e;
  }
  *token = (void*)a;
  return 0;
}

int stage_end(int stage, void* stream, void* token) {
  if (!token) return 0;
  hipEvent_t a = (hipEvent_t)token, b;
  hipError_t e = hipEventCreate(&b);
  if (e != hipSuccess) return (int)e;
  e = hipEventRecord(b, (hipStream_t)stream);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_mu);
  g_recs.push_back({stage, a, b});
  return 0;
}

}  // namespace cdd

extern "C" {

cdd_status cdd_profile_enable(int32_t on) {
  cdd::g_on.store(on ? 1 : 0);
  return CDD_OK;
}

cdd_status cdd_profile_select(uint32_t stage_mask) {
  if (stage_mask == 0 || (stage_mask >> CDD_NSTAGES) != 0)
    return cdd::fail(CDD_EINVAL, "stage_mask 0x%x must select stages among the %d", stage_mask,
                     CDD_NSTAGES);
  cdd::g_mask.store(stage_mask);
  return CDD_OK;
}

cdd_status cdd_profile_read(cdd_profile* out) {
  if (!out) return cdd::fail(CDD_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof *out);
  std::vector<cdd::Rec> recs;
  {
    std::lock_guard<std::mutex> lk(cdd::g_mu);
    recs.swap(cdd::g_recs);
  }
  cdd_status st = CDD_OK;
  for (auto& r : recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && st == CDD_OK)
      st = cdd::fail(CDD_EDEVICE, "event timing: %s", hipGetErrorString(e));
    if (r.stage >= 0 && r.stage < CDD_NSTAGES) {
      out->ms[r.stage] += ms;
      out->count[r.stage] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  return st;
}

}  // extern "C"
