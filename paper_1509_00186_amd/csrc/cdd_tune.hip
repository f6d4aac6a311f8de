// Autotuner: transform length, block-kernel schedule and DM tile per beam shape.
//
// For a beam (channels, band, DM trials, integration) every valid
// combination of N in [n_min, n_max] (powers of two up to 16384, with the
// overlap shorter than N), schedule and DM tile is timed on the device in
// the form a plan runs it: a beam with one DM trial builds its chirp table
// and runs the one-workgroup-per-block kernel over it; a beam with several
// runs the persistent batched kernel (each schedule that kernel is compiled
// for) over a tile of 16, 32 or 64 trials (no more than the beam has), on
// a seeded random int8 record of the beam's channel count.  Two sweeps, the
// best time of each candidate kept (the first sweep also brings the device
// clocks up).  The score is input samples x DM trials per second, which
// weighs the work per block against the overlap discarded per block
// (M = N - L).  Results are cached in memory per device and shape, and in a
// text file when CDD_TUNE_CACHE names one.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cdd_internal.h"

namespace cdd {
namespace {

std::mutex g_tune_mu;
std::map<std::string, cdd_tune_result> g_tune;
bool g_file_loaded = false;

std::string shape_key(int dev, int32_t dtype, int32_t nchan, double fc, double bw,
                      const double* dms, int32_t ndm, int32_t n_int, int32_t n_min,
                      int32_t n_max) {
  hipDeviceProp_t prop;
  char arch[64] = "gpu";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
      if (*c == ':' || *c == ' ') *c = '_';
  }
  double dlo = dms[0], dhi = dms[0];
  for (int i = 1; i < ndm; ++i) {
    dlo = std::fmin(dlo, dms[i]);
    dhi = std::fmax(dhi, dms[i]);
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "v2|%s|t%d|c%d|f%.6f|b%.6f|dm%.4f:%.4f:%d|i%d|n%d:%d", arch, dtype,
                nchan, fc, bw, dlo, dhi, ndm, n_int, n_min, n_max);
  return buf;
}

void load_file() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  const char* path = std::getenv("CDD_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[256];
  cdd_tune_result r;
  while (std::fscanf(f, "%255s %d %d %d %lf %lf", key, &r.fft_len, &r.kernel_variant,
                     &r.dm_tile, &r.ms, &r.msamples_per_s) == 6)
    g_tune[key] = r;
  std::fclose(f);
}

void append_file(const std::string& key, const cdd_tune_result& r) {
  const char* path = std::getenv("CDD_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %.6f %.3f\n", key.c_str(), r.fft_len, r.kernel_variant,
               r.dm_tile, r.ms, r.msamples_per_s);
  std::fclose(f);
}

__global__ void fill_random_i8(unsigned short* x, int64_t n, unsigned seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  unsigned h = (unsigned)i * 2654435761u ^ seed;
  h ^= h >> 13;
  h *= 0x5bd1e995u;
  h ^= h >> 15;
  // two signed bytes of moderate amplitude
  const int a = (int)(h & 63) - 32, b = (int)((h >> 8) & 63) - 32;
  x[i] = (unsigned short)((a & 0xff) | ((b & 0xff) << 8));
}

}  // namespace
}  // namespace cdd

using namespace cdd;

extern "C" cdd_status cdd_autotune(int32_t dtype, int32_t nchan, double f_centre_mhz,
                                   double bw_mhz, const double* host_dms, int32_t ndm,
                                   int32_t n_int, int32_t n_min, int32_t n_max,
                                   cdd_tune_result* best) {
  if (!best || !host_dms || ndm < 1) return fail(CDD_EINVAL, "NULL argument or no DM");
  if (dtype != CDD_CI8) return fail(CDD_ENOTSUP, "the autotuner times int8 records");
  if (n_min <= 0) n_min = 1 << 11;
  if (n_max <= 0) n_max = 1 << 14;
  n_max = std::min(n_max, 16384);
  if (n_min > n_max) return fail(CDD_EINVAL, "n_min > n_max");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CDD_EDEVICE, "%s", hipGetErrorString(e));
  const std::string key =
      shape_key(dev, dtype, nchan, f_centre_mhz, bw_mhz, host_dms, ndm, n_int, n_min, n_max);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_file();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *best = it->second;
      clear_error();
      return CDD_OK;
    }
  }
  // synthetic record: eight blocks of the longest candidate, at most 256 MiB
  const int64_t cap_samples = std::max<int64_t>(1, ((int64_t)256 << 20) / (2LL * nchan));
  // (a multiple of 64, so the record is its own channel-major layout)
  const int64_t T =
      std::max<int64_t>(64, std::min<int64_t>((int64_t)8 * n_max, cap_samples) / 64 * 64);
  const int max_tile = std::min<int>(ndm, kMaxDmTile);
  std::vector<int> tiles;
  if (ndm == 1) {
    tiles.push_back(1);
  } else {
    for (int t : {16, 32, 64}) {
      const int tt = std::min(t, max_tile);
      if (tiles.empty() || tiles.back() != tt) tiles.push_back(tt);
    }
  }
  unsigned short* x = nullptr;
  float* P = nullptr;
  void* H = nullptr;         // chirp table when there is one DM trial
  void* dev_tab = nullptr;   // launch table and work counter
  hipStream_t st = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  cdd_tune_result win{};
  win.msamples_per_s = -1;
  cdd_status status = CDD_OK;
  std::vector<char> host_tab(batch_table_bytes(1));
  do {
    if ((e = hipMalloc(&x, (size_t)T * nchan * 2)) != hipSuccess) break;
    if ((e = hipMalloc(&P, (size_t)max_tile * nchan * (T / n_int + 1) * 4)) != hipSuccess)
      break;
    if (ndm == 1 && (e = hipMalloc(&H, (size_t)nchan * n_max * 8)) != hipSuccess) break;
    if ((e = hipMalloc(&dev_tab, 512 + batch_table_bytes(1))) != hipSuccess) break;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) break;
    if ((e = hipEventCreate(&a)) != hipSuccess) break;
    if ((e = hipEventCreate(&b)) != hipSuccess) break;
    const int64_t n = T * nchan;
    hipLaunchKernelGGL(fill_random_i8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n,
                       0x9e3779b9u);
    unsigned int* counter = (unsigned int*)dev_tab;
    void* tab = (char*)dev_tab + 512;
    std::vector<float> best_ms;
    for (int sweep = 0; sweep < 2 && e == hipSuccess; ++sweep) {
      int ci = 0;
      for (int N = n_min; N <= n_max && e == hipSuccess; N *= 2) {
        cdd_opts o{};
        BeamPlan p;
        if (make_plan(dtype, T, nchan, f_centre_mhz, bw_mhz, host_dms, ndm, N, n_int, &o, &p) !=
            CDD_OK)
          continue;  // DM too large for this N
        for (int v = 0; v < block_variants(N) && e == hipSuccess; ++v) {
          if (ndm == 1 ? v != 0 : !batch_variant_ok(N, v)) continue;
          p.variant = v;
          for (int tile_n : tiles) {
            BatchBeam bb;
            bb.p = &p;
            bb.xt = x;
            bb.dms.ndm = tile_n;
            for (int i = 0; i < tile_n; ++i) bb.dms.dm[i] = host_dms[(int64_t)i * ndm / tile_n];
            bb.P = P;
            bb.co = offline_coords(p);
            const void* h = H;
            LaunchDesc d;
            int err = prepare_launch(ndm == 1 ? kLaunchTables : kLaunchBatch, &bb, &h, 1,
                                     host_tab.data(), &d);
            // one execution as the plan runs it: the table build with one DM,
            // then the launch (the host table is the same every time)
            auto run = [&]() -> int {
              int r = 0;
              if (H) r = launch_chirp_table(p, bb.dms.dm[0], H, st);
              return r ? r : enqueue_launch(d, host_tab.data(), tab, counter, st);
            };
            if (!err) err = run();  // warm-up (and the twiddle tables)
            if (!err && (e = hipStreamSynchronize(st)) != hipSuccess) break;
            (void)hipEventRecord(a, st);
            for (int r = 0; r < 2 && !err; ++r) err = run();
            (void)hipEventRecord(b, st);
            if (err) {
              e = (hipError_t)err;
              break;
            }
            if ((e = hipEventSynchronize(b)) != hipSuccess) break;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, a, b);
            ms /= 2.0f;
            if (sweep == 0) {
              best_ms.push_back(ms);
            } else {
              ms = std::min(ms, best_ms[ci]);
              const double rate = (double)nchan * T * tile_n / (ms * 1e-3) / 1e6;
              if (rate > win.msamples_per_s) {
                win.fft_len = N;
                win.kernel_variant = v;
                win.dm_tile = tile_n;
                win.ms = ms;
                win.msamples_per_s = rate;
              }
            }
            ++ci;
          }
        }
      }
    }
  } while (false);
  if (e != hipSuccess)
    status = fail(e == hipErrorOutOfMemory ? CDD_ENOMEM : CDD_EDEVICE, "autotune: %s",
                  hipGetErrorString(e));
  else if (win.msamples_per_s < 0)
    status = fail(CDD_EINVAL, "no transform length in [%d, %d] fits this DM", n_min, n_max);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (st) (void)hipStreamDestroy(st);
  if (x) (void)hipFree(x);
  if (P) (void)hipFree(P);
  if (H) (void)hipFree(H);
  if (dev_tab) (void)hipFree(dev_tab);
  if (status != CDD_OK) return status;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = win;
    append_file(key, win);
  }
  *best = win;
  clear_error();
  return CDD_OK;
}
