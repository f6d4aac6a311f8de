// Entry point that allocates nothing: cdd_dedisperse with its workspace in a
// static device array instead of caller- or library-allocated memory.
//
// Every launch of the call goes on the caller's stream (no auxiliary
// streams or events) and the twiddle tables come from the library's static
// table pool, so a call issues kernel launches and, on its first call on a
// device, one symbol lookup and the table uploads -- never a device
// allocation.  Each GPU holds its own copy of the array, from the first use
// of the library on it until the process ends.  All calls on one GPU share
// that copy: calls that overlap in time on one GPU (on different streams, or
// from several threads) race on it and must be serialised by the caller.
// Every word a call reads is first written by the same call, so nothing has
// to start at zero.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "cdd_internal.h"

namespace cdd {

constexpr size_t kScratchBytes = (size_t)CDD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_ptr;  // device -> its copy of scratch

// This device's address of the array (looked up once per device, with the
// device current).  The array's name is a host-side stand-in, never passed on.
static int scratch_of(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return 0;
  }
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  if (ptr == nullptr || ((uintptr_t)ptr & 255u) != 0) return (int)hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = (char*)ptr;
  *out = (char*)ptr;
  return 0;
}

}  // namespace cdd

using namespace cdd;

extern "C" cdd_status cdd_dedisperse_noalloc(const void* voltages, int32_t dtype, int64_t nsamp,
                                             int32_t nchan, double f_centre_mhz, double bw_mhz,
                                             double dm, int32_t fft_len, int32_t n_int,
                                             float* intensity, int32_t* coverage,
                                             float* chan_intensity, void* volt_out,
                                             const cdd_opts* opts, void* stream) {
  try {
    if (!voltages) return fail(CDD_EINVAL, "voltages is NULL");
    if (!intensity) return fail(CDD_EINVAL, "intensity is NULL");
    if (opts && (opts->npol > 1 || opts->time_chunks > 1))
      return fail(CDD_ENOTSUP, "cdd_dedisperse_noalloc takes one polarisation and one time "
                               "chunk (npol %d, time_chunks %d)", opts->npol, opts->time_chunks);
    if (opts && (opts->npol < 0 || opts->time_chunks < 0))
      return fail(CDD_EINVAL, "npol and time_chunks must be >= 0");
    BeamPlan p;
    cdd_status s = make_plan(dtype, nsamp, nchan, f_centre_mhz, bw_mhz, &dm, 1, fft_len, n_int,
                             opts, &p);
    if (s != CDD_OK) return s;
    if (!block_supported(p.N) && !large_supported(p.N))
      return fail(CDD_ENOTSUP, "fft_len %d is not supported by the library", p.N);
    const WsLayout lay = ws_layout(p, 1, true, true);
    if (lay.total > kScratchBytes)
      return fail(CDD_EINVAL,
                  "this call needs %zu bytes of scratch; cdd_dedisperse_noalloc holds %zu "
                  "(use cdd_dedisperse with a workspace)", lay.total, kScratchBytes);
    char* ws = nullptr;
    const int e = scratch_of(&ws);
    if (e) return device_fail("static scratch lookup", e);
    DmTile tile;
    tile.ndm = 1;
    tile.dm[0] = dm;
    s = run_tile(p, voltages, tile, nullptr, ws, lay, chan_intensity, volt_out, intensity,
                 coverage, p.t_int, stream, false);
    if (s == CDD_OK) clear_error();
    return s;
  } catch (const std::bad_alloc&) {
    return fail(CDD_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
}
