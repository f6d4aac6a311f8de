// Layout change, channel delays and the delay-aligned channel sum.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cdd_fft.h"
#include "cdd_internal.h"

namespace cdd {

// Delay of channel c at one DM in integrated samples (the expression of
// delays_kernel below and of the host planner, in the same order, without
// fused multiply-adds, so all three round to the same integers).
__device__ __forceinline__ int32_t channel_delay(int c, double dm, int32_t nchan, double f_centre,
                                                 double bw, double df, double dconst,
                                                 int32_t n_int) {
#pragma clang fp contract(off)
  const double fc = (f_centre - bw / 2.0) + ((double)c + 0.5) * df;
  const int cref = dm >= 0 ? nchan - 1 : 0;
  const double fref = (f_centre - bw / 2.0) + ((double)cref + 0.5) * df;
  const double x = dconst * dm * (1.0 / (fc * fc) - 1.0 / (fref * fref)) * df / (double)n_int;
  return (int32_t)floor(x + 0.5);
}

// One DM's channel delays, computed by one workgroup of the layout change.
struct DelayArgs {
  int32_t* d;  // null: none
  double dm, f_centre, bw, df, dconst;
  int32_t nchan, n_int;
};

// ---------------------------------------------------------------------------
// Time-major [nsamp][nchan] -> channel-major [nchan][nsamp].
// int8 pairs (2 bytes per complex sample): 64 samples x 128 channels per
// workgroup through LDS; each lane moves 8 bytes (4 complex samples) on both
// the load (along channels) and the store (along time) side.
// Float pairs: a 64 x 64 tile, one element per lane access.
// ---------------------------------------------------------------------------
// With ct.H set, workgroup w < ct.nwg also writes table workgroup w's share
// of the one-DM chirp table once its tile stores are issued: the table's
// FP64 arithmetic runs while the memory-bound layout change's traffic is in
// flight, instead of in a kernel of its own beside it.  With dl.d set, the
// last workgroup also writes the channel delays.
__global__ __launch_bounds__(256) void transpose_i8_kernel(const unsigned short* __restrict__ in,
                                                           unsigned short* __restrict__ out,
                                                           int64_t nsamp, int32_t nchan,
                                                           int32_t tiles_c, int32_t in_aligned,
                                                           int64_t ostr, const ChirpTableArgs ct,
                                                           const DelayArgs dl) {
  __shared__ unsigned short tile[64][128 + 4];
  const int64_t bid = blockIdx.x;
  const int c0 = (int)(bid % tiles_c) * 128;
  const int64_t t0 = (bid / tiles_c) * 64;
  const int l = threadIdx.x;
  const bool full =
      in_aligned && (c0 + 128 <= nchan) && (t0 + 64 <= nsamp) && (nchan % 4 == 0);
  // load: 32 lanes per row, 4 channels each; 8 rows per pass of 256 lanes
  {
    const int cl = (l & 31) * 4, rl = l >> 5;
#pragma unroll
    for (int i = 0; i < 64; i += 8) {
      const int r = rl + i;
      const int64_t ts = t0 + r;
      if (full) {
        const uint2 w = *(const uint2*)(in + ts * nchan + c0 + cl);
        tile[r][cl + 0] = (unsigned short)(w.x & 0xffff);
        tile[r][cl + 1] = (unsigned short)(w.x >> 16);
        tile[r][cl + 2] = (unsigned short)(w.y & 0xffff);
        tile[r][cl + 3] = (unsigned short)(w.y >> 16);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int cs = c0 + cl + q;
          tile[r][cl + q] = (ts < nsamp && cs < nchan) ? in[ts * nchan + cs] : (unsigned short)0;
        }
      }
    }
  }
  __syncthreads();
  // store: 16 lanes per channel row, 4 samples each; 16 channels per pass
  {
    const int tl = (l & 15) * 4, cr = l >> 4;
#pragma unroll
    for (int i = 0; i < 128; i += 16) {
      const int c = cr + i;
      const int cs = c0 + c;
      if (cs >= nchan) continue;
      const int64_t ts = t0 + tl;
      if (full || ts + 4 <= nsamp) {
        if ((nsamp & 3) == 0 || full) {
          uint2 w;
          w.x = (unsigned)tile[tl + 0][c] | ((unsigned)tile[tl + 1][c] << 16);
          w.y = (unsigned)tile[tl + 2][c] | ((unsigned)tile[tl + 3][c] << 16);
          if (((int64_t)cs * ostr + ts) % 4 == 0) {
            *(uint2*)(out + (int64_t)cs * ostr + ts) = w;
            continue;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (ts + q < nsamp) out[(int64_t)cs * ostr + ts + q] = tile[tl + q][c];
    }
  }
  if (ct.H != nullptr && blockIdx.x < ct.nwg) chirp_table_part(ct, blockIdx.x, l);
  if (dl.d != nullptr && blockIdx.x == gridDim.x - 1)
    for (int c = l; c < dl.nchan; c += 256)
      dl.d[c] = channel_delay(c, dl.dm, dl.nchan, dl.f_centre, dl.bw, dl.df, dl.dconst, dl.n_int);
}

__global__ __launch_bounds__(256) void transpose_c8_kernel(const float2* __restrict__ in,
                                                           float2* __restrict__ out,
                                                           int64_t nsamp, int32_t nchan,
                                                           int32_t tiles_c, int64_t ostr) {
  __shared__ float2 tile[64][65];
  const int64_t bid = blockIdx.x;
  const int c0 = (int)(bid % tiles_c) * 64;
  const int64_t t0 = (bid / tiles_c) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 64; i += 4) {
    const int64_t ts = t0 + ty + i;
    const int cs = c0 + tx;
    if (ts < nsamp && cs < nchan) tile[ty + i][tx] = in[ts * nchan + cs];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 64; i += 4) {
    const int cs = c0 + ty + i;
    const int64_t ts = t0 + tx;
    if (cs < nchan && ts < nsamp) out[(int64_t)cs * ostr + ts] = tile[tx][ty + i];
  }
}

int launch_transpose(const void* in, void* out, int32_t dtype, int64_t nsamp, int32_t nchan,
                     int64_t out_stride, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dtype == CDD_CI8) {
    const int64_t tiles_c = (nchan + 127) / 128, tiles_t = (nsamp + 63) / 64;
    const int64_t n = tiles_c * tiles_t;
    if (n <= 0 || n > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose_i8_kernel, dim3((unsigned)n), dim3(256), 0, st,
                       (const unsigned short*)in, (unsigned short*)out, nsamp, nchan,
                       (int32_t)tiles_c, (int32_t)(((uintptr_t)in & 7u) == 0), out_stride,
                       ChirpTableArgs{}, DelayArgs{});
  } else {
    const int64_t tiles_c = (nchan + 63) / 64, tiles_t = (nsamp + 63) / 64;
    const int64_t n = tiles_c * tiles_t;
    if (n <= 0 || n > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose_c8_kernel, dim3((unsigned)n), dim3(256), 0, st,
                       (const float2*)in, (float2*)out, nsamp, nchan, (int32_t)tiles_c,
                       out_stride);
  }
  return (int)hipGetLastError();
}

bool transpose_chirp_fits(const BeamPlan& p) {
  if (p.dtype != CDD_CI8 || p.nchan < 2 || !block_supported(p.N)) return false;
  const int64_t n = (int64_t)((p.nchan + 127) / 128) * ((p.nsamp + 63) / 64);
  return (int64_t)p.nchan <= n;  // at least one channel's table per workgroup at kpt = N/256
}

int launch_transpose_chirp(const BeamPlan& p, const void* in, void* out, double dm, void* H,
                           void* stream, int32_t* delays) {
  if (!transpose_chirp_fits(p) || H == nullptr) return (int)hipErrorInvalidValue;
  const int64_t tiles_c = (p.nchan + 127) / 128, tiles_t = (p.nsamp + 63) / 64;
  const int64_t n = tiles_c * tiles_t;
  if (n > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  // the fewest table entries per thread that the layout change's workgroups cover
  int kpt = 1;
  while ((int64_t)p.nchan * (p.N / (256 * kpt)) > n && 256 * kpt * 2 <= p.N) kpt *= 2;
  const ChirpTableArgs ct = chirp_table_args(p, dm, H, kpt);
  DelayArgs dl{};
  if (delays) {
    dl.d = delays;
    dl.dm = dm;
    dl.f_centre = p.f_centre;
    dl.bw = p.bw;
    dl.df = p.df;
    dl.dconst = p.dconst;
    dl.nchan = p.nchan;
    dl.n_int = p.n_int;
  }
  hipLaunchKernelGGL(transpose_i8_kernel, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream,
                     (const unsigned short*)in, (unsigned short*)out, p.nsamp, p.nchan,
                     (int32_t)tiles_c, (int32_t)(((uintptr_t)in & 7u) == 0), xt_stride(p), ct,
                     dl);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Channel delays in FP64 (Sec. 1.2; the linear term of Eq. 2): the same
// operations, in the same order and without fused multiply-adds, as the
// host planner, so both round to the same integers.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void delays_kernel(int32_t* __restrict__ d, DmTile dms,
                                                     int32_t nchan, double f_centre, double bw,
                                                     double df, double dconst, int32_t n_int) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (c >= nchan || i >= dms.ndm) return;
  d[(int64_t)i * nchan + c] =
      channel_delay(c, dms.dm[i], nchan, f_centre, bw, df, dconst, n_int);
}
#pragma clang fp contract(on)

int launch_delays(const BeamPlan& p, const DmTile& dms, int32_t* d, void* stream) {
  dim3 grid((unsigned)((p.nchan + 255) / 256), (unsigned)dms.ndm);
  hipLaunchKernelGGL(delays_kernel, grid, dim3(256), 0, (hipStream_t)stream, d, dms, p.nchan,
                     p.f_centre, p.bw, p.df, p.dconst, p.n_int);
  return (int)hipGetLastError();
}

// v[i] = x for i < n (four per thread).
__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ v, int64_t n,
                                                       int32_t x) {
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (i + j < n) v[i + j] = x;
}

int launch_fill_i32(int32_t* v, int64_t n, int32_t x, void* stream) {
  if (n <= 0) return 0;
  const int64_t nb = (n + 1023) / 1024;
  if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, v,
                     n, x);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Detection and integration without the coherent step (incoherent
// dedispersion): P[c][u] = sum over r < n_int of |x_c[u n_int + r]|^2, in
// order; consecutive threads take consecutive u of one channel.
// ---------------------------------------------------------------------------
template <int DT>
__global__ __launch_bounds__(256) void detect_kernel(const void* __restrict__ xt,
                                                     float* __restrict__ P, int64_t xstride,
                                                     int64_t t_int, int32_t n_int) {
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (u >= t_int) return;
  float s = 0.f;
  const int64_t base = (int64_t)c * xstride + u * n_int;
  for (int r = 0; r < n_int; ++r) {
    float re, im;
    if constexpr (DT == CDD_CI8) {
      const unsigned short w = ((const unsigned short*)xt)[base + r];
      re = (float)(signed char)(w & 0xff);
      im = (float)(signed char)(w >> 8);
    } else {
      const float2 z = ((const float2*)xt)[base + r];
      re = z.x;
      im = z.y;
    }
    s += re * re + im * im;
  }
  P[(int64_t)c * t_int + u] = s;
}

int launch_detect(const BeamPlan& p, const void* xt, float* P, void* stream) {
  const int64_t nb = (p.t_int + 255) / 256;
  if (nb <= 0) return 0;
  if (nb > 0x7fffffffLL || p.nchan > 65535) return (int)hipErrorInvalidValue;
  dim3 grid((unsigned)nb, (unsigned)p.nchan);
  if (p.dtype == CDD_CI8)
    hipLaunchKernelGGL(detect_kernel<CDD_CI8>, grid, dim3(256), 0, (hipStream_t)stream, xt, P,
                       xt_stride(p), p.t_int, p.n_int);
  else
    hipLaunchKernelGGL(detect_kernel<CDD_CF32>, grid, dim3(256), 0, (hipStream_t)stream, xt, P,
                       xt_stride(p), p.t_int, p.n_int);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Folding at a known period: one thread per phase bin b.  Sample u belongs to
// bin floor(frac(u/period + phase0) * nbins) (FP64, contraction off, clamped
// to nbins - 1); the thread visits, for each period k, the samples around
// [(k + b/nbins - phase0) period, (k + (b+1)/nbins - phase0) period), keeps
// those whose bin is b, and adds them in ascending u (a fixed order) in FP64,
// rounding the sum to FP32 once (a bin may hold the whole series).
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
__device__ __forceinline__ int fold_bin(int64_t u, double period, double phase0, int nbins) {
  const double x = (double)u / period + phase0;
  const int b = (int)floor((x - floor(x)) * (double)nbins);
  return b < nbins ? b : nbins - 1;
}

__global__ __launch_bounds__(256) void fold_kernel(const float* __restrict__ I, int64_t t_int,
                                                   double period, double phase0, int32_t nbins,
                                                   float* __restrict__ prof,
                                                   int32_t* __restrict__ cnt) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nbins) return;
  const int64_t k0 = (int64_t)floor(phase0) - 1;
  const int64_t k1 = (int64_t)floor((double)(t_int - 1) / period + phase0) + 1;
  double s = 0.0;
  int32_t n = 0;
  int64_t next = 0;  // samples below have been visited
  for (int64_t k = k0; k <= k1; ++k) {
    const double lo = ((double)k + (double)b / nbins - phase0) * period;
    const double hi = ((double)k + (double)(b + 1) / nbins - phase0) * period;
    int64_t u0 = (int64_t)floor(lo) - 2, u1 = (int64_t)ceil(hi) + 2;
    if (u0 < next) u0 = next;
    if (u1 > t_int) u1 = t_int;
    for (int64_t u = u0; u < u1; ++u)
      if (fold_bin(u, period, phase0, nbins) == b) {
        s += (double)I[u];
        ++n;
      }
    if (u1 > next) next = u1;
  }
  prof[b] = (float)s;
  if (cnt) cnt[b] = n;
}
#pragma clang fp contract(on)

int launch_fold(const float* I, int64_t t_int, double period, double phase0, int32_t nbins,
                float* profile, int32_t* counts, void* stream) {
  const int64_t nb = ((int64_t)nbins + 255) / 256;
  if (nb <= 0 || nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(fold_kernel, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, I,
                     t_int, period, phase0, nbins, profile, counts);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// I[u] = sum over channels c with u + d_c < T_int of P_c[u + d_c], cov[u] =
// number of terms.  A workgroup covers 64 consecutive u; its G waves each sum
// a contiguous channel range in ascending order, and the G partial sums are
// added in ascending wave order -- a fixed order, no atomics, so results do
// not depend on scheduling.  grid.y = DM trial.
// Each channel row is read through a buffer resource whose range ends at
// src_lim: a term past the end is pointed at src_lim itself and reads as zero
// (adding +0 leaves the sum unchanged), so the loads carry no branch; eight
// channels' loads are issued before they are added.  Rows of 2^29 floats or
// more take the checked loop.
// ---------------------------------------------------------------------------
template <int G, bool BUF>
__global__ __launch_bounds__(64 * G) void dsum_kernel(const float* __restrict__ P,
                                                      const int32_t* __restrict__ d,
                                                      float* __restrict__ I,
                                                      int32_t* __restrict__ cov, int32_t nchan,
                                                      int64_t p_stride, int64_t p_dm_stride,
                                                      int64_t src_lim, int64_t u_begin,
                                                      int64_t u_count, int64_t out_stride) {
  __shared__ float ps[G][64];
  __shared__ int32_t pn[G][64];
  const int i = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index (uniform)
  const int64_t uo = (int64_t)blockIdx.x * 64 + lane;
  const int64_t u = u_begin + uo;
  const float* Pi = P + (int64_t)i * p_dm_stride;
  const int32_t* di = d + (int64_t)i * nchan;
  const int per = (nchan + G - 1) / G;
  const int c_lo = g * per, c_hi = min(nchan, c_lo + per);
  float acc = 0.f;
  int32_t n = 0;
  if constexpr (BUF) {
    // lanes past u_count read offset 0 (in range or zero) and are not stored
    const bool live = uo < u_count;
    const int ub = live ? (int)u : 0;
    const int lim = (int)src_lim;
    int c = c_lo;
    for (; c + 8 <= c_hi; c += 8) {
      float x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(Pi + (int64_t)(c + j) * p_stride), (short)0, lim * 4, 0x00020000);
        const int64_t src = (int64_t)ub + di[c + j];
        const bool in = src < lim;
        x[j] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rs, (in ? (int)src : lim) * 4, 0, 0));
        n += in;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += x[j];
    }
    for (; c < c_hi; ++c) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(Pi + (int64_t)c * p_stride), (short)0, lim * 4, 0x00020000);
      const int64_t src = (int64_t)ub + di[c];
      const bool in = src < lim;
      acc += __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(rs, (in ? (int)src : lim) * 4, 0, 0));
      n += in;
    }
  } else {
    if (uo < u_count) {
      for (int c = c_lo; c < c_hi; ++c) {
        const int64_t src = u + di[c];
        if (src < src_lim) {
          acc += Pi[(int64_t)c * p_stride + src];
          ++n;
        }
      }
    }
  }
  ps[g][lane] = acc;
  pn[g][lane] = n;
  __syncthreads();
  if (g == 0 && uo < u_count) {
    float s = ps[0][lane];
    int32_t m = pn[0][lane];
#pragma unroll
    for (int k = 1; k < G; ++k) {
      s += ps[k][lane];
      m += pn[k][lane];
    }
    I[(int64_t)i * out_stride + uo] = s;
    if (cov) cov[(int64_t)i * out_stride + uo] = m;
  }
}

template <int G>
static void dsum_launch(bool buf, dim3 grid, hipStream_t st, const float* P, const int32_t* d,
                        float* I, int32_t* cov, int nchan, int64_t p_stride, int64_t p_dm_stride,
                        int64_t src_lim, int64_t u_begin, int64_t u_count, int64_t out_stride) {
  if (buf)
    hipLaunchKernelGGL((dsum_kernel<G, true>), grid, dim3(64 * G), 0, st, P, d, I, cov, nchan,
                       p_stride, p_dm_stride, src_lim, u_begin, u_count, out_stride);
  else
    hipLaunchKernelGGL((dsum_kernel<G, false>), grid, dim3(64 * G), 0, st, P, d, I, cov, nchan,
                       p_stride, p_dm_stride, src_lim, u_begin, u_count, out_stride);
}

int launch_dsum_range(int nchan, int ndm, const float* P, int64_t p_stride, int64_t p_dm_stride,
                      int64_t src_lim, int64_t u_begin, int64_t u_count, const int32_t* d,
                      float* I, int32_t* cov, int64_t out_stride, void* stream) {
  if (u_count <= 0) return 0;
  const int64_t nb = (u_count + 63) / 64;
  if (nb > 0x7fffffffLL || ndm < 1 || ndm > 65535) return (int)hipErrorInvalidValue;
  dim3 grid((unsigned)nb, (unsigned)ndm);
  hipStream_t st = (hipStream_t)stream;
  // 32-bit byte offsets: row lengths and output positions below 2^29
  const bool buf = src_lim >= 0 && src_lim < (1LL << 29) && u_begin + u_count < (1LL << 29);
  if (nchan >= 256)
    dsum_launch<16>(buf, grid, st, P, d, I, cov, nchan, p_stride, p_dm_stride, src_lim, u_begin,
                    u_count, out_stride);
  else if (nchan >= 64)
    dsum_launch<8>(buf, grid, st, P, d, I, cov, nchan, p_stride, p_dm_stride, src_lim, u_begin,
                   u_count, out_stride);
  else
    dsum_launch<1>(buf, grid, st, P, d, I, cov, nchan, p_stride, p_dm_stride, src_lim, u_begin,
                   u_count, out_stride);
  return (int)hipGetLastError();
}

int launch_dsum(const BeamPlan& p, int ndm, const float* P, const int32_t* d, float* I,
                int32_t* cov, int64_t out_stride, void* stream) {
  return launch_dsum_range(p.nchan, ndm, P, p.t_int, (int64_t)p.nchan * p.t_int, p.t_int, 0,
                           p.t_int, d, I, cov, out_stride, stream);
}

}  // namespace cdd
