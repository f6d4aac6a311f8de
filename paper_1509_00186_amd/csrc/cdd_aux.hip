// Layout change, channel delays and the delay-aligned channel sum.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cdd_internal.h"

namespace cdd {

// ---------------------------------------------------------------------------
// Time-major [nsamp][nchan] -> channel-major [nchan][nsamp], one element per
// complex sample (2 bytes for int8 pairs, 8 bytes for float pairs), through
// a 64 x 64 LDS tile.  Grid: one workgroup per tile, flattened.
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(256) void transpose_kernel(const E* __restrict__ in,
                                                        E* __restrict__ out, int64_t nsamp,
                                                        int32_t nchan, int32_t tiles_c) {
  __shared__ E tile[64][65];
  const int64_t bid = blockIdx.x;
  const int tc = (int)(bid % tiles_c);
  const int64_t tt = bid / tiles_c;
  const int c0 = tc * 64;
  const int64_t t0 = tt * 64;
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
    if (cs < nchan && ts < nsamp) out[(int64_t)cs * nsamp + ts] = tile[tx][ty + i];
  }
}

int launch_transpose(const void* in, void* out, int32_t dtype, int64_t nsamp, int32_t nchan,
                     void* stream) {
  const int64_t tiles_c = (nchan + 63) / 64, tiles_t = (nsamp + 63) / 64;
  const int64_t n = tiles_c * tiles_t;
  if (n <= 0 || n > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == CDD_CI8)
    hipLaunchKernelGGL(transpose_kernel<unsigned short>, dim3((unsigned)n), dim3(256), 0, st,
                       (const unsigned short*)in, (unsigned short*)out, nsamp, nchan,
                       (int32_t)tiles_c);
  else
    hipLaunchKernelGGL(transpose_kernel<float2>, dim3((unsigned)n), dim3(256), 0, st,
                       (const float2*)in, (float2*)out, nsamp, nchan, (int32_t)tiles_c);
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
  const double dm = dms.dm[i];
  const double fc = (f_centre - bw / 2.0) + ((double)c + 0.5) * df;
  const int cref = dm >= 0 ? nchan - 1 : 0;
  const double fref = (f_centre - bw / 2.0) + ((double)cref + 0.5) * df;
  const double x = dconst * dm * (1.0 / (fc * fc) - 1.0 / (fref * fref)) * df / (double)n_int;
  d[(int64_t)i * nchan + c] = (int32_t)floor(x + 0.5);
}
#pragma clang fp contract(on)

int launch_delays(const BeamPlan& p, const DmTile& dms, int32_t* d, void* stream) {
  dim3 grid((unsigned)((p.nchan + 255) / 256), (unsigned)dms.ndm);
  hipLaunchKernelGGL(delays_kernel, grid, dim3(256), 0, (hipStream_t)stream, d, dms, p.nchan,
                     p.f_centre, p.bw, p.df, p.dconst, p.n_int);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// I[u] = sum over channels c = 0, 1, ... with u + d_c < T_int of P_c[u + d_c]
// (fixed order, no atomics), cov[u] = number of terms.  grid.y = DM trial.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void dsum_kernel(const float* __restrict__ P,
                                                   const int32_t* __restrict__ d,
                                                   float* __restrict__ I, int32_t* __restrict__ cov,
                                                   int32_t nchan, int64_t t_int,
                                                   int64_t out_stride) {
  const int i = blockIdx.y;
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= t_int) return;
  const float* Pi = P + (int64_t)i * nchan * t_int;
  const int32_t* di = d + (int64_t)i * nchan;
  float acc = 0.f;
  int32_t n = 0;
  for (int c = 0; c < nchan; ++c) {
    const int64_t src = u + di[c];
    if (src < t_int) {
      acc += Pi[(int64_t)c * t_int + src];
      ++n;
    }
  }
  I[(int64_t)i * out_stride + u] = acc;
  if (cov) cov[(int64_t)i * out_stride + u] = n;
}

int launch_dsum(const BeamPlan& p, int ndm, const float* P, const int32_t* d, float* I,
                int32_t* cov, int64_t out_stride, void* stream) {
  const int64_t nb = (p.t_int + 255) / 256;
  if (nb <= 0 || nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(dsum_kernel, dim3((unsigned)nb, (unsigned)ndm), dim3(256), 0,
                     (hipStream_t)stream, P, d, I, cov, p.nchan, p.t_int, out_stride);
  return (int)hipGetLastError();
}

}  // namespace cdd
