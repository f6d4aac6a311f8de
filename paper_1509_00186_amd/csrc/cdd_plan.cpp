// Planner: validation, overlap-save geometry and channel delays (host, FP64).
//
// Rules (De & Gupta, Sec. 2.2 and 2.3):
//  * the dedispersing filter of channel c delays offset f by the group delay
//    D*DM*(1/f_c^2 - 1/(f_c+f)^2) us; at the channel edges this gives how far
//    the impulse response reaches forward ("front", corrupting the start of
//    each block) and backward ("back", corrupting its end), in samples;
//  * overlap L covers front + back, rounded up to a power of two, then raised
//    until the step M = N - L is a multiple of the integration length;
//  * the kept window starts at nfront = front + (L - front - back) / 2;
//  * N, unless given, is the smallest power of two above twice the widest
//    channel's dispersion time in samples, and at least 2L and 256.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "cdd_internal.h"

namespace cdd {

namespace {
thread_local std::string g_err = "";
}

cdd_status fail(cdd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = std::string(cdd_status_str(s)) + ": " + buf;
  return s;
}

void clear_error() { g_err.clear(); }

// The delay and geometry arithmetic below must round exactly as written:
// keep the compiler from fusing multiply-adds.
#pragma clang fp contract(off)

double channel_centre(const BeamPlan& p, int c) {
  return (p.f_centre - p.bw / 2.0) + ((double)c + 0.5) * p.df;
}

static double group_delay_samples(double dconst, double dm, double f0, double f,
                                  double df) {
  return dconst * dm * (1.0 / (f0 * f0) - 1.0 / ((f0 + f) * (f0 + f))) * df;
}

int64_t channel_delay(const BeamPlan& p, double dm, int c) {
  double fc = channel_centre(p, c);
  double fref = channel_centre(p, dm >= 0 ? p.nchan - 1 : 0);
  double x = p.dconst * dm * (1.0 / (fc * fc) - 1.0 / (fref * fref)) * p.df /
             (double)p.n_int;
  return (int64_t)std::floor(x + 0.5);
}

static bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

cdd_status make_plan(int32_t dtype, int64_t nsamp, int32_t nchan,
                     double f_centre, double bw, const double* dms, int32_t ndm,
                     int32_t fft_len, int32_t n_int, const cdd_opts* opts,
                     BeamPlan* out) {
  BeamPlan p;
  if (dtype != CDD_CI8 && dtype != CDD_CF32)
    return fail(CDD_EINVAL, "dtype %d is not CDD_CI8 or CDD_CF32", dtype);
  if (nsamp < 1) return fail(CDD_EINVAL, "nsamp must be >= 1 (got %lld)", (long long)nsamp);
  if (nchan < 1) return fail(CDD_EINVAL, "nchan must be >= 1 (got %d)", nchan);
  if (n_int < 1) return fail(CDD_EINVAL, "n_int must be >= 1 (got %d)", n_int);
  if (n_int > nsamp)
    return fail(CDD_EINVAL, "n_int (%d) exceeds nsamp (%lld)", n_int, (long long)nsamp);
  if (!std::isfinite(f_centre) || !std::isfinite(bw))
    return fail(CDD_EINVAL, "frequencies must be finite");
  if (!(bw > 0)) return fail(CDD_EINVAL, "bw must be > 0 (got %g)", bw);
  if (!(f_centre - bw / 2.0 > 0))
    return fail(CDD_EINVAL, "band must lie above 0 MHz (f_centre - bw/2 = %g)",
                f_centre - bw / 2.0);
  if (ndm < 1 || dms == nullptr) return fail(CDD_EINVAL, "no DM given");
  for (int i = 0; i < ndm; ++i)
    if (!std::isfinite(dms[i])) return fail(CDD_EINVAL, "DM %d is not finite", i);
  p.dtype = dtype;
  p.nsamp = nsamp;
  p.nchan = nchan;
  p.f_centre = f_centre;
  p.bw = bw;
  p.df = bw / nchan;
  p.f_lo = f_centre - bw / 2.0;
  p.n_int = n_int;
  p.dms.assign(dms, dms + ndm);
  if (opts) {
    if (opts->dm_const != 0) {
      if (!std::isfinite(opts->dm_const) || opts->dm_const <= 0)
        return fail(CDD_EINVAL, "dm_const must be finite and > 0");
      p.dconst = opts->dm_const;
    }
    if (opts->phase_mode != CDD_PHASE_FP64_REDUCED && opts->phase_mode != CDD_PHASE_FP32)
      return fail(CDD_EINVAL, "unknown phase_mode %d", opts->phase_mode);
    p.phase_mode = opts->phase_mode;
    if (opts->taper < CDD_TAPER_NONE || opts->taper > CDD_TAPER_WELCH)
      return fail(CDD_EINVAL, "unknown taper %d", opts->taper);
    p.taper = opts->taper;
    p.variant = opts->kernel_variant;
  }

  // Reach of the impulse response and widest dispersion, over channels/DMs.
  double front = 0, back = 0, disp = 0;
  for (double dm : p.dms) {
    for (int c = 0; c < nchan; ++c) {
      double fc = channel_centre(p, c);
      double lo = group_delay_samples(p.dconst, dm, fc, -p.df / 2.0, p.df);
      double hi = group_delay_samples(p.dconst, dm, fc, +p.df / 2.0, p.df);
      front = std::fmax(front, std::fmax(lo, hi));
      back = std::fmax(back, -std::fmin(lo, hi));
      double flo = fc - p.df / 2.0, fhi = fc + p.df / 2.0;
      double ds = p.dconst * std::fabs(dm) * (1.0 / (flo * flo) - 1.0 / (fhi * fhi)) * p.df;
      disp = std::fmax(disp, ds);
    }
  }
  if (front > 1e9 || back > 1e9)
    return fail(CDD_EINVAL, "dispersion too large (impulse response %g samples)",
                front + back);
  p.front = (int32_t)std::ceil(front);
  p.back = (int32_t)std::ceil(back);

  bool expl = opts && opts->explicit_plan;
  int64_t want_n = expl ? opts->fft_len : fft_len;
  if (want_n != 0 && (!pow2(want_n) || want_n < kMinFFT || want_n > kMaxFFT))
    return fail(CDD_EINVAL, "fft_len %lld must be a power of two in [%d, %d]",
                (long long)want_n, kMinFFT, kMaxFFT);
  if (expl) {
    if (want_n == 0) return fail(CDD_EINVAL, "explicit_plan needs fft_len");
    p.N = (int32_t)want_n;
    p.L = opts->overlap;
    p.nfront = opts->nfront;
    if (p.L < 0 || p.L >= p.N)
      return fail(CDD_EINVAL, "overlap %d must lie in [0, fft_len)", p.L);
    if ((p.N - p.L) % n_int != 0)
      return fail(CDD_EINVAL, "fft_len - overlap (%d) must be a multiple of n_int (%d)",
                  p.N - p.L, n_int);
    if (p.L < p.front + p.back)
      return fail(CDD_EINVAL, "overlap %d shorter than the impulse response (%d); "
                  "DM too large for this overlap", p.L, p.front + p.back);
    if (p.nfront < p.front || p.nfront > p.L - p.back)
      return fail(CDD_EINVAL, "nfront %d outside [%d, %d]", p.nfront, p.front,
                  p.L - p.back);
  } else {
    int64_t L = 1;
    while (L < (int64_t)p.front + p.back) L *= 2;
    int64_t N = want_n;
    if (N == 0) {
      int64_t r = 1;
      while (!((double)r > 2.0 * disp)) r *= 2;
      N = std::max<int64_t>(std::max<int64_t>(r, 2 * L), kMinFFT);
      if (N > kMaxFFT)
        return fail(CDD_EINVAL, "DM too large: length rule asks for N = %lld > %d",
                    (long long)N, kMaxFFT);
    }
    while (L < N && (N - L) % n_int != 0) ++L;
    if (L >= N)
      return fail(CDD_EINVAL, "DM too large for fft_len %lld; need N > %lld",
                  (long long)N, (long long)L);
    p.N = (int32_t)N;
    p.L = (int32_t)L;
    // the spare margin centred, then the start moved down to a multiple of
    // 16 samples where the margin allows (the long transforms then write the
    // kept window in whole 128-byte runs)
    p.nfront = p.front + (p.L - p.front - p.back) / 2;
    if (p.nfront - p.nfront % 16 >= p.front) p.nfront -= p.nfront % 16;
  }
  if (p.variant < 0 || (block_supported(p.N) && p.variant >= block_variants(p.N)))
    return fail(CDD_EINVAL, "kernel_variant %d not available for fft_len %d", p.variant, p.N);
  p.M = p.N - p.L;
  p.nblocks = (nsamp + p.M - 1) / p.M;
  p.t_int = nsamp / n_int;
  int64_t dmax = 0;
  for (double dm : p.dms) {
    dmax = std::max<int64_t>(dmax, channel_delay(p, dm, 0));
    dmax = std::max<int64_t>(dmax, channel_delay(p, dm, nchan - 1));
  }
  p.d_max = dmax;
  *out = p;
  return CDD_OK;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t xt_stride(const BeamPlan& p) {
  return !large_supported(p.N) && p.nchan > 1 ? (p.nsamp + 63) / 64 * 64 : p.nsamp;
}

WsLayout ws_layout(const BeamPlan& p, int ndm_tile, bool need_p, bool chirp_table) {
  WsLayout w;
  size_t off = 0;
  size_t elem = p.dtype == CDD_CI8 ? 2 : 8;
  if (p.nchan > 1) {
    w.xt_off = off;
    w.xt_bytes = (size_t)p.nchan * xt_stride(p) * elem;
    off = align256(off + w.xt_bytes);
  }
  if (need_p) {
    w.p_off = off;
    w.p_bytes = (size_t)ndm_tile * p.nchan * p.t_int * sizeof(float);
    off = align256(off + w.p_bytes);
  }
  w.d_off = off;
  w.d_bytes = (size_t)ndm_tile * p.nchan * sizeof(int32_t);
  off = align256(off + w.d_bytes);
  if (!block_supported(p.N) && large_supported(p.N)) {
    // one chunk of spectra, then the call's chirp table (nchan x N)
    w.s_off = off;
    w.s_bytes = (size_t)(large_chunk_items(p) + p.nchan) * p.N * 8;
    off = align256(off + w.s_bytes);
    w.pb_off = off;
    w.pb_bytes = std::max((size_t)p.nchan * p.nsamp * sizeof(float),
                          large_partial_bytes(p.N, large_chunk_items(p)));
    off = align256(off + w.pb_bytes);
  }
  if (chirp_table && block_supported(p.N)) {
    w.h_off = off;
    w.h_bytes = (size_t)p.nchan * p.N * 8;
    off = align256(off + w.h_bytes);
  }
  w.total = off;
  return w;
}

}  // namespace cdd

extern "C" {

const char* cdd_last_error(void) { return cdd::g_err.c_str(); }

const char* cdd_status_str(cdd_status s) {
  switch (s) {
    case CDD_OK: return "CDD_OK";
    case CDD_EINVAL: return "CDD_EINVAL";
    case CDD_ENOMEM: return "CDD_ENOMEM";
    case CDD_EDEVICE: return "CDD_EDEVICE";
    case CDD_EBUSY: return "CDD_EBUSY";
    case CDD_EAGAIN: return "CDD_EAGAIN";
    case CDD_EINTERNAL: return "CDD_EINTERNAL";
    case CDD_ENOTSUP: return "CDD_ENOTSUP";
  }
  return "CDD_UNKNOWN";
}

int32_t cdd_abi_version(void) { return CDD_ABI_VERSION; }

int32_t cdd_kernel_variants(int32_t fft_len) { return cdd::block_variants(fft_len); }

cdd_status cdd_query(int32_t dtype, int64_t nsamp, int32_t nchan,
                     double f_centre_mhz, double bw_mhz, double dm,
                     int32_t fft_len, int32_t n_int, int32_t want_voltages,
                     const cdd_opts* opts, cdd_plan_info* info) {
  (void)want_voltages;
  if (!info) return cdd::fail(CDD_EINVAL, "info is NULL");
  cdd::BeamPlan p;
  cdd_status s = cdd::make_plan(dtype, nsamp, nchan, f_centre_mhz, bw_mhz, &dm, 1,
                                fft_len, n_int, opts, &p);
  if (s != CDD_OK) return s;
  std::memset(info, 0, sizeof *info);
  info->fft_len = p.N;
  info->overlap = p.L;
  info->nfront = p.nfront;
  info->step = p.M;
  info->nblocks = p.nblocks;
  info->t_int = p.t_int;
  info->front = p.front;
  info->back = p.back;
  info->d_max = p.d_max;
  info->ws_bytes = cdd::ws_layout(p, 1, true, true).total;
  cdd::clear_error();
  return CDD_OK;
}

}  // extern "C"
