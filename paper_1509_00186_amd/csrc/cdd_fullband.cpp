// Full-band mode (the paper's unchannelised pipeline): plan and entry points.
//
// The recorded beam holds real-FFT spectra (Sec. 2.3: 8-bit outputs of a
// 2 nchan-point FFT of the real sampled voltage).  Their inverse transforms
// laid end to end give back the real series at 2 bw samples per microsecond
// (Sec. 3.1, the inverse transform routine), which is dedispersed as one
// band by overlap-save with the filter of Eq. 3 about the band's lower edge
// (Sec. 2.1 writes the real-sampled band from its lower edge f_o), then
// detected (y^2) and integrated.
//
// Plan rules (Sec. 2.2, 2.3), in real samples: the filter about the lower
// edge delays every higher frequency to the lower edge's arrival, so its
// impulse response reaches forward by the dispersion time across the band
// (backward for DM < 0); L = the power of two >= that reach (>= 2), raised
// until n_int divides N - L; nfront = front + (L - front - back) / 2, moved
// down to a multiple of 32 if that stays >= front, else to an even value;
// N (if not given) = max(smallest power of two > twice the
// dispersion samples, 2L, 2^16).  Everything stays even so that blocks start
// on sample pairs.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "cdd_fullband.h"

namespace cdd {

#pragma clang fp contract(off)

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

static cdd_status make_fullband_plan(int64_t nspec, int32_t nchan, double f_centre, double bw,
                                     double dm, int32_t fft_len, int32_t n_int,
                                     const cdd_opts* opts, FullbandPlan* out) {
  FullbandPlan f;
  if (nspec < 1) return fail(CDD_EINVAL, "nspec must be >= 1 (got %lld)", (long long)nspec);
  if (!gsb_supported(nchan))
    return fail(CDD_EINVAL, "nchan must be a power of two in [128, 2048] (got %d)", nchan);
  if (n_int < 2 || n_int % 2)
    return fail(CDD_EINVAL, "n_int must be even and >= 2 (got %d)", n_int);
  if (!std::isfinite(f_centre) || !std::isfinite(bw) || !std::isfinite(dm))
    return fail(CDD_EINVAL, "frequencies and DM must be finite");
  if (!(bw > 0)) return fail(CDD_EINVAL, "bw must be > 0 (got %g)", bw);
  if (!(f_centre - bw / 2.0 > 0))
    return fail(CDD_EINVAL, "band must lie above 0 MHz (f_centre - bw/2 = %g)",
                f_centre - bw / 2.0);
  if (nspec > ((int64_t)1 << 40) / nchan)
    return fail(CDD_EINVAL, "record too long (%lld records)", (long long)nspec);
  f.nspec = nspec;
  f.nchan = nchan;
  f.nsamp = nspec * 2 * nchan;
  if (n_int > f.nsamp)
    return fail(CDD_EINVAL, "n_int (%d) exceeds the %lld real samples", n_int,
                (long long)f.nsamp);
  f.n_int = n_int;
  f.bw = bw;
  f.f_lo = f_centre - bw / 2.0;
  f.dm = dm;
  if (opts) {
    if (opts->dm_const != 0) {
      if (!std::isfinite(opts->dm_const) || opts->dm_const <= 0)
        return fail(CDD_EINVAL, "dm_const must be finite and > 0");
      f.dconst = opts->dm_const;
    }
    if (opts->phase_mode == CDD_PHASE_FP32)
      return fail(CDD_ENOTSUP, "the full-band mode evaluates the chirp phase in FP64 only");
    if (opts->phase_mode != CDD_PHASE_FP64_REDUCED)
      return fail(CDD_EINVAL, "unknown phase_mode %d", opts->phase_mode);
    if (opts->taper < CDD_TAPER_NONE || opts->taper > CDD_TAPER_WELCH)
      return fail(CDD_EINVAL, "unknown taper %d", opts->taper);
    f.taper = opts->taper;
    if (opts->npol > 1 || opts->kernel_variant != 0 || opts->time_chunks > 1)
      return fail(CDD_ENOTSUP, "npol, kernel_variant and time_chunks do not apply to the "
                  "full-band mode");
  }
  const double f_hi = f.f_lo + bw;
  const double reach = f.dconst * std::fabs(dm) * (1.0 / (f.f_lo * f.f_lo) - 1.0 / (f_hi * f_hi)) *
                       (2.0 * bw);
  if (!(reach < 1e9))
    return fail(CDD_EINVAL, "dispersion too large (%g samples across the band)", reach);
  f.front = dm >= 0 ? (int32_t)std::ceil(reach) : 0;
  f.back = dm >= 0 ? 0 : (int32_t)std::ceil(reach);

  const bool expl = opts && opts->explicit_plan;
  const int64_t want_n = expl ? opts->fft_len : fft_len;
  if (want_n != 0 && (!is_pow2(want_n) || want_n < kMinFullband || want_n > kMaxFullband))
    return fail(CDD_EINVAL, "fft_len %lld must be a power of two in [%d, %d] real points",
                (long long)want_n, kMinFullband, kMaxFullband);
  if (expl) {
    if (want_n == 0) return fail(CDD_EINVAL, "explicit_plan needs fft_len");
    f.N = (int32_t)want_n;
    f.L = opts->overlap;
    f.nfront = opts->nfront;
    if (f.L < 2 || f.L >= f.N || f.L % 2 || f.nfront % 2)
      return fail(CDD_EINVAL, "overlap %d must be even in [2, fft_len) and nfront %d even",
                  f.L, f.nfront);
    if ((f.N - f.L) % n_int != 0)
      return fail(CDD_EINVAL, "fft_len - overlap (%d) must be a multiple of n_int (%d)",
                  f.N - f.L, n_int);
    if (f.L < f.front + f.back)
      return fail(CDD_EINVAL, "overlap %d shorter than the impulse response (%d); "
                  "DM too large for this overlap", f.L, f.front + f.back);
    if (f.nfront < f.front || f.nfront > f.L - f.back)
      return fail(CDD_EINVAL, "nfront %d outside [%d, %d]", f.nfront, f.front, f.L - f.back);
  } else {
    int64_t L = 2;
    while (L < (int64_t)f.front + f.back) L *= 2;
    int64_t N = want_n;
    if (N == 0) {
      int64_t r = 1;
      while (!((double)r > 2.0 * reach)) r *= 2;
      N = std::max<int64_t>(std::max<int64_t>(r, 2 * L), kMinFullband);
      if (N > kMaxFullband)
        return fail(CDD_ENOTSUP, "DM too large: the length rule asks for %lld real points, "
                    "the library transforms at most %d", (long long)N, kMaxFullband);
    }
    while (L < N && (N - L) % n_int != 0) ++L;
    if (L >= N)
      return fail(CDD_EINVAL, "DM too large for fft_len %lld; need N > %lld", (long long)N,
                  (long long)L);
    f.N = (int32_t)N;
    f.L = (int32_t)L;
    // centred, then moved down to a multiple of 32 real samples (16 sample
    // pairs: whole 128-byte runs of the packed series) where the margin
    // allows, else to an even value
    int32_t nf = f.front + (f.L - f.front - f.back) / 2;
    if (nf - nf % 32 >= f.front)
      nf -= nf % 32;
    else if (nf % 2)
      nf = nf + 1 <= f.L - f.back ? nf + 1 : nf - 1;
    f.nfront = nf;
    if (f.nfront < f.front || f.nfront > f.L - f.back || f.nfront % 2)
      return fail(CDD_EINTERNAL, "plan rule broke its invariant (nfront %d)", f.nfront);
  }
  f.M = f.N - f.L;
  f.nblocks = (f.nsamp + f.M - 1) / f.M;
  f.t_int = f.nsamp / n_int;
  *out = f;
  return CDD_OK;
}

struct FullbandWs {
  size_t x_off = 0, s_off = 0, pb_off = 0, h_off = 0, total = 0;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static FullbandWs fullband_ws(const FullbandPlan& f) {
  FullbandWs w;
  size_t off = 0;
  w.x_off = off;
  off = align256(off + (size_t)f.nsamp * sizeof(float));
  w.s_off = off;
  off = align256(off + (size_t)fullband_chunk_blocks(f) * (size_t)(f.N / 2) * 8);
  w.pb_off = off;
  off = align256(off + std::max((size_t)(f.nsamp / 2) * sizeof(float),
                                 large_partial_bytes(f.N / 2, fullband_chunk_blocks(f))));
  w.h_off = off;
  off = align256(off + (size_t)(f.N / 2 + 1) * 8);
  w.total = off;
  return w;
}

static cdd_status device_error(const char* what, int err) {
  return fail(CDD_EDEVICE, "%s: %s", what, hip_error_string(err));
}

}  // namespace cdd

using namespace cdd;

extern "C" cdd_status cdd_gsb_inverse(const void* spectra, int64_t nspec, int32_t nchan,
                                      float* series, void* stream) {
  if (!spectra || !series) return fail(CDD_EINVAL, "spectra or series is NULL");
  if (((uintptr_t)spectra & 3u) || ((uintptr_t)series & 7u))
    return fail(CDD_EINVAL, "spectra must be 4-byte and series 8-byte aligned");
  if (nspec < 1) return fail(CDD_EINVAL, "nspec must be >= 1 (got %lld)", (long long)nspec);
  if (!gsb_supported(nchan))
    return fail(CDD_EINVAL, "nchan must be a power of two in [128, 2048] (got %d)", nchan);
  void* tok = nullptr;
  int e = stage_begin(kStageTranspose, stream, &tok);
  if (!e) e = launch_gsb_inverse(spectra, nspec, nchan, series, stream);
  if (!e) e = stage_end(kStageTranspose, stream, tok);
  if (e) return device_error("inverse-transform launch", e);
  clear_error();
  return CDD_OK;
}

extern "C" cdd_status cdd_fullband_query(int64_t nspec, int32_t nchan, double f_centre_mhz,
                                         double bw_mhz, double dm, int32_t fft_len,
                                         int32_t n_int, const cdd_opts* opts,
                                         cdd_fullband_info* info) {
  if (!info) return fail(CDD_EINVAL, "info is NULL");
  FullbandPlan f;
  cdd_status s = make_fullband_plan(nspec, nchan, f_centre_mhz, bw_mhz, dm, fft_len, n_int,
                                    opts, &f);
  if (s != CDD_OK) return s;
  std::memset(info, 0, sizeof *info);
  info->fft_len = f.N;
  info->overlap = f.L;
  info->nfront = f.nfront;
  info->step = f.M;
  info->nsamp = f.nsamp;
  info->nblocks = f.nblocks;
  info->t_int = f.t_int;
  info->front = f.front;
  info->back = f.back;
  info->ws_bytes = fullband_ws(f).total;
  clear_error();
  return CDD_OK;
}

extern "C" cdd_status cdd_fullband_dedisperse(const void* spectra, int64_t nspec, int32_t nchan,
                                              double f_centre_mhz, double bw_mhz, double dm,
                                              int32_t fft_len, int32_t n_int, float* intensity,
                                              float* volt_out, const cdd_opts* opts,
                                              void* workspace, size_t ws_bytes, void* stream) {
  try {
    if (!spectra || !intensity) return fail(CDD_EINVAL, "spectra or intensity is NULL");
    if ((uintptr_t)spectra & 3u) return fail(CDD_EINVAL, "spectra must be 4-byte aligned");
    if (volt_out && ((uintptr_t)volt_out & 7u))
      return fail(CDD_EINVAL, "volt_out must be 8-byte aligned");
    FullbandPlan f;
    cdd_status s = make_fullband_plan(nspec, nchan, f_centre_mhz, bw_mhz, dm, fft_len, n_int,
                                      opts, &f);
    if (s != CDD_OK) return s;
    const FullbandWs lay = fullband_ws(f);
    if (!workspace || ws_bytes < lay.total)
      return fail(CDD_EINVAL, "workspace too small: need %zu bytes, got %zu", lay.total,
                  workspace ? ws_bytes : (size_t)0);
    if ((uintptr_t)workspace & 255u)
      return fail(CDD_EINVAL, "workspace must be 256-byte aligned");
    char* ws = (char*)workspace;
    float* x = (float*)(ws + lay.x_off);
    void* tok = nullptr;
    int e = stage_begin(kStageTranspose, stream, &tok);
    if (!e) e = launch_gsb_inverse(spectra, nspec, nchan, x, stream);
    if (!e) e = stage_end(kStageTranspose, stream, tok);
    if (e) return device_error("inverse-transform launch", e);
    e = stage_begin(kStageBlock, stream, &tok);
    if (!e) e = launch_fullband(f, x, ws + lay.s_off, (float*)(ws + lay.pb_off), ws + lay.h_off,
                                intensity, volt_out, stream);
    if (!e) e = stage_end(kStageBlock, stream, tok);
    if (e) return device_error("full-band transform launch", e);
    clear_error();
    return CDD_OK;
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
}
