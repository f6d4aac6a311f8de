// Long overlap-save transforms (N = 2^15 .. 2^22) as a four-step FFT.
//
// The paper dedisperses the full band with transforms of millions of points
// (Sec. 1.3, 2.3, 4.5); here N = N1 * N2 with n = n1 + N1 n2 and
// k = k2 + N2 k1:
//   cols_fwd : for each column n1, DFT over n2 of x[n1 + N1 n2] (length N2),
//              times W_N^(n1 k2), stored row-major as S[k2][n1]
//   rows     : for each row k2, DFT over n1 (length N1) gives X[k2 + N2 k1];
//              multiply by the chirp of Eq. 3 (and 1/N); inverse DFT over k1;
//              times W_N^(-n1 k2); stored back in place as S[k2][n1]
//   cols_inv : for each column n1, inverse DFT over k2 gives z[n1 + N1 n2];
//              samples [nfront, nfront + M) of block k become y[k M + m]:
//              |y|^2 to a per-sample buffer and, if asked, y itself
//   integrate: P[u] = sum of n_int consecutive |y|^2
// Every sub-transform reuses the register/LDS Stockham passes of the block
// kernel; a workgroup runs G sub-transforms side by side, lanes ordered so
// that global accesses along n1 are contiguous.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "cdd_fft.h"
#include "cdd_internal.h"

namespace cdd {

// Sub-transform schedules (length L, Tsub threads, 16 points per thread).
template <int L>
struct SubSched;
template <> struct SubSched<128> { using type = Sched<128, 8, 8, 16, 1, 1>; };
template <> struct SubSched<256> { using type = Sched<256, 16, 16, 16, 1, 1>; };
template <> struct SubSched<512> { using type = Sched<512, 32, 8, 8, 8, 1>; };
template <> struct SubSched<1024> { using type = Sched<1024, 64, 16, 16, 4, 1>; };
template <> struct SubSched<2048> { using type = Sched<2048, 128, 16, 16, 8, 1>; };

struct LargeArgs {
  const void* x;        // channel-major input [nchan][nsamp]
  float2* S;            // [items][N] intermediate spectra (items of this chunk)
  float* p;             // [nchan][nsamp] |y|^2
  float2* vout;         // [nchan][nsamp] or null
  const float2* twc;    // column sub-transform twiddles
  const float2* twr;    // row sub-transform twiddles
  const float2* tw4;    // four-step twiddles: W_N^m = lo[m & (2^sl-1)] * hi[m >> sl]
  int64_t nsamp, nblocks, item0;
  int32_t nchan, N1, N2, M, nfront, sl, phase_mode, exact_div, taper;
  double f_lo, df, dconst, dm;
};

__device__ __forceinline__ float2 tw4_fwd(const LargeArgs& a, int64_t m) {
  const float2 lo = a.tw4[m & ((1 << a.sl) - 1)];
  const float2 hi = a.tw4[(1 << a.sl) + (m >> a.sl)];
  return cmul(lo, hi);
}

// ---------------------------------------------------------------------------
// cols_fwd
// ---------------------------------------------------------------------------
template <class SC, int G, int DT>
__global__ __launch_bounds__(SC::T * G) void cols_fwd_kernel(const LargeArgs a) {
  __shared__ float lds[G * (SC::lds_floats() + 1)];
  constexpr int L = SC::N, R0 = SC::rad_f(0), B0 = L / (R0 * SC::T);
  constexpr int RL = SC::rad_f(SC::NP - 1), BL = L / (RL * SC::T);
  const int t = threadIdx.x, g = t % G, tl = t / G;
  const int ngrp = a.N1 / G;
  const int64_t item = a.item0 + blockIdx.x / ngrp;
  const int n1 = (blockIdx.x % ngrp) * G + g;
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  const int64_t base = k * a.M - a.nfront + n1;
  float2 v[SC::E];
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n2 = tl + SC::T * b + r * (L / R0);
      const int64_t ts = base + (int64_t)a.N1 * n2;
      float2 z = make_float2(0.f, 0.f);
      if (ts >= 0 && ts < a.nsamp) {
        if constexpr (DT == CDD_CI8) {
          const short w = ((const short*)a.x)[(int64_t)c * a.nsamp + ts];
          z = make_float2((float)(signed char)(w & 0xff), (float)(signed char)(w >> 8));
        } else {
          z = ((const float2*)a.x)[(int64_t)c * a.nsamp + ts];
        }
      }
      v[b * R0 + r] = z;
    }
  fft_forward<SC>(v, lds + g * (SC::lds_floats() + 1), a.twc, tl);
  float2* S = a.S + (item - a.item0) * ((int64_t)a.N1 * a.N2);
#pragma unroll
  for (int b = 0; b < BL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int k2 = tl + SC::T * b + r * (L / RL);
      S[(int64_t)k2 * a.N1 + n1] = cmul(v[b * RL + r], tw4_fwd(a, (int64_t)n1 * k2));
    }
}

// ---------------------------------------------------------------------------
// rows: forward row DFT, chirp, inverse row DFT, conjugate four-step twiddle
// ---------------------------------------------------------------------------
template <class SR, int G>
__global__ __launch_bounds__(SR::T * G) void rows_kernel(const LargeArgs a) {
  __shared__ float lds[G * (SR::lds_floats() + 1)];
  constexpr int L = SR::N, R0 = SR::rad_f(0), B0 = L / (R0 * SR::T);
  constexpr int RL = SR::rad_f(SR::NP - 1), BL = L / (RL * SR::T);
  const int t = threadIdx.x, g = t / SR::T, tl = t % SR::T;
  const int ngrp = a.N2 / G;
  const int64_t item = a.item0 + blockIdx.x / ngrp;
  const int k2 = (blockIdx.x % ngrp) * G + g;
  const int c = (int)(item / a.nblocks);
  const int64_t N = (int64_t)a.N1 * a.N2;
  float2* row = a.S + (item - a.item0) * N + (int64_t)k2 * a.N1;
  float2 v[SR::E];
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) v[b * R0 + r] = row[tl + SR::T * b + r * (L / R0)];
  float* my = lds + g * (SR::lds_floats() + 1);
  fft_forward<SR>(v, my, a.twr, tl);
  // chirp on bins i = k2 + N2 k1
  const double fc = a.f_lo + ((double)c + 0.5) * a.df;
  const float inv_n = 1.0f / (float)N;
  if (a.phase_mode == CDD_PHASE_FP64_REDUCED) {
    const double dfn = a.df / (double)N;
    const double B = a.dconst * a.dm * dfn * dfn / (fc * fc * fc);
    const double beta = dfn / fc;
#pragma unroll
    for (int b = 0; b < BL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int64_t k1 = tl + SR::T * b + r * (L / RL);
        const int64_t i = k2 + (int64_t)a.N2 * k1;
        const double sd = (double)(i < N / 2 ? i : i - N);
        const double x = beta * sd;
        const double q = a.exact_div ? (B * (sd * sd)) / fma(beta, sd, 1.0)
                                     : (B * (sd * sd)) * fma(x, x, 1.0 - x);
        const float2 h = expi_neg_turns(q - rint(q));
        const float g = inv_n * taper_gain<false>(a.taper, (float)sd * inv_n);
        v[b * RL + r] = cmul(v[b * RL + r], make_float2(h.x * g, h.y * g));
      }
  } else {
    const float fcf = (float)fc;
    const float Af = (float)(a.dconst * a.dm) / (fcf * fcf);
    const float dfn = (float)a.df / (float)N;
#pragma unroll
    for (int b = 0; b < BL; ++b)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int64_t k1 = tl + SR::T * b + r * (L / RL);
        const int64_t i = k2 + (int64_t)a.N2 * k1;
        const float sf = (float)(i < N / 2 ? i : i - N);
        const float f = sf * dfn;
        const float q = Af * (f * f) / (fcf + f);
        float sn, cs;
        sincospif(2.0f * q, &sn, &cs);
        const float g = inv_n * taper_gain<false>(a.taper, sf * inv_n);
        v[b * RL + r] = cmul(v[b * RL + r], make_float2(cs * g, -sn * g));
      }
  }
  fft_inverse<SR>(v, my, a.twr, tl);
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n1 = tl + SR::T * b + r * (L / R0);
      const float2 w = tw4_fwd(a, (int64_t)n1 * k2);
      row[n1] = cmul(v[b * R0 + r], make_float2(w.x, -w.y));
    }
}

// ---------------------------------------------------------------------------
// cols_inv: inverse column DFT, overlap-save window, detection, voltages
// ---------------------------------------------------------------------------
template <class SC, int G>
__global__ __launch_bounds__(SC::T * G) void cols_inv_kernel(const LargeArgs a) {
  __shared__ float lds[G * (SC::lds_floats() + 1)];
  constexpr int L = SC::N, RI = SC::rad_i(0), BI = L / (RI * SC::T);
  constexpr int R0 = SC::rad_f(0), B0 = L / (R0 * SC::T);
  const int t = threadIdx.x, g = t % G, tl = t / G;
  const int ngrp = a.N1 / G;
  const int64_t item = a.item0 + blockIdx.x / ngrp;
  const int n1 = (blockIdx.x % ngrp) * G + g;
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  const float2* S = a.S + (item - a.item0) * ((int64_t)a.N1 * a.N2);
  float2 v[SC::E];
#pragma unroll
  for (int b = 0; b < BI; ++b)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int k2 = tl + SC::T * b + r * (L / RI);
      v[b * RI + r] = S[(int64_t)k2 * a.N1 + n1];
    }
  fft_inverse<SC>(v, lds + g * (SC::lds_floats() + 1), a.twc, tl);
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n2 = tl + SC::T * b + r * (L / R0);
      const int64_t n = n1 + (int64_t)a.N1 * n2;
      const int64_t m = n - a.nfront;
      const int64_t o = k * a.M + m;
      if (m >= 0 && m < a.M && o < a.nsamp) {
        const float2 z = v[b * R0 + r];
        a.p[(int64_t)c * a.nsamp + o] = z.x * z.x + z.y * z.y;
        if (a.vout) a.vout[(int64_t)c * a.nsamp + o] = z;
      }
    }
}

// P[c][u] = sum_{r < n_int} p[c][u n_int + r], grid (u blocks, channels)
__global__ __launch_bounds__(256) void integrate_kernel(const float* __restrict__ p,
                                                        float* __restrict__ P, int64_t nsamp,
                                                        int64_t t_int, int32_t n_int) {
  const int c = blockIdx.y;
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= t_int) return;
  const float* pc = p + (int64_t)c * nsamp + u * n_int;
  float s = 0.f;
  for (int r = 0; r < n_int; ++r) s += pc[r];
  P[(int64_t)c * t_int + u] = s;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <int LGN>
static std::vector<float2> make_fourstep() {
  const int sl = (LGN + 1) / 2;
  const int64_t N = (int64_t)1 << LGN;
  const int64_t nlo = (int64_t)1 << sl, nhi = N >> sl;
  std::vector<float2> t(nlo + nhi);
  for (int64_t m = 0; m < nlo; ++m) {
    const double ang = -2.0 * M_PI * (double)m / (double)N;
    t[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  for (int64_t h = 0; h < nhi; ++h) {
    const double ang = -2.0 * M_PI * (double)(h << sl) / (double)N;
    t[nlo + h] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  return t;
}

constexpr int64_t kChunkBytes = (int64_t)512 << 20;  // intermediate spectra per chunk

bool large_supported(int N) { return N >= (1 << 15) && N <= (1 << 22) && (N & (N - 1)) == 0; }

int64_t large_chunk_items(const BeamPlan& p) {
  const int64_t items = (int64_t)p.nchan * p.nblocks;
  const int64_t per = std::max<int64_t>(1, kChunkBytes / ((int64_t)p.N * 8));
  return std::min(items, per);
}

template <int LGN>
static int launch_large_t(const BeamPlan& p, const void* xt, double dm, float2* S, float* pbuf,
                          float* P, void* vout, int exact_div, void* stream) {
  constexpr int N2 = 1 << (LGN / 2), N1 = 1 << (LGN - LGN / 2);
  using SC = typename SubSched<N2>::type;
  using SR = typename SubSched<N1>::type;
  constexpr int GC = SC::T * 16 <= 1024 ? 16 : 8;
  constexpr int GR = SR::T * 8 <= 1024 ? 8 : 4;
  static_assert(N1 % GC == 0 && N2 % GR == 0, "group sizes must tile the transform");
  LargeArgs a{};
  int e = twiddles_of<SC>(&a.twc);
  if (!e) e = twiddles_of<SR>(&a.twr);
  if (!e) e = cached_table((std::string("fourstep") + std::to_string(LGN)).c_str(),
                           &make_fourstep<LGN>, &a.tw4);
  if (e) return e;
  a.x = xt;
  a.S = S;
  a.p = pbuf;
  a.vout = (float2*)vout;
  a.nsamp = p.nsamp;
  a.nblocks = p.nblocks;
  a.nchan = p.nchan;
  a.N1 = N1;
  a.N2 = N2;
  a.M = p.M;
  a.nfront = p.nfront;
  a.sl = (LGN + 1) / 2;
  a.phase_mode = p.phase_mode;
  a.taper = p.taper;
  a.exact_div = exact_div;
  a.f_lo = p.f_lo;
  a.df = p.df;
  a.dconst = p.dconst;
  a.dm = dm;
  hipStream_t st = (hipStream_t)stream;
  const int64_t items = (int64_t)p.nchan * p.nblocks;
  const int64_t chunk = large_chunk_items(p);
  for (int64_t i0 = 0; i0 < items; i0 += chunk) {
    const int64_t q = std::min(chunk, items - i0);
    a.item0 = i0;
    const int64_t gc = q * (N1 / GC), gr = q * (N2 / GR);
    if (gc > 0x7fffffffLL || gr > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    if (p.dtype == CDD_CI8)
      hipLaunchKernelGGL((cols_fwd_kernel<SC, GC, CDD_CI8>), dim3((unsigned)gc), dim3(SC::T * GC),
                         0, st, a);
    else
      hipLaunchKernelGGL((cols_fwd_kernel<SC, GC, CDD_CF32>), dim3((unsigned)gc),
                         dim3(SC::T * GC), 0, st, a);
    hipLaunchKernelGGL((rows_kernel<SR, GR>), dim3((unsigned)gr), dim3(SR::T * GR), 0, st, a);
    hipLaunchKernelGGL((cols_inv_kernel<SC, GC>), dim3((unsigned)gc), dim3(SC::T * GC), 0, st,
                       a);
    e = (int)hipGetLastError();
    if (e) return e;
  }
  const int64_t nb = (p.t_int + 255) / 256;
  if (nb > 0x7fffffffLL || p.nchan > 65535) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(integrate_kernel, dim3((unsigned)nb, (unsigned)p.nchan), dim3(256), 0, st,
                     pbuf, P, p.nsamp, p.t_int, p.n_int);
  return (int)hipGetLastError();
}

int exact_division_needed(const BeamPlan& p, double dm_abs_max);

int launch_large(const BeamPlan& p, const void* xt, double dm, void* Sv, float* pbuf, float* P,
                 void* vout, void* stream) {
  float2* S = (float2*)Sv;
  const int ex = exact_division_needed(p, std::fabs(dm));
  switch (p.N) {
    case 1 << 15: return launch_large_t<15>(p, xt, dm, S, pbuf, P, vout, ex, stream);
    case 1 << 16: return launch_large_t<16>(p, xt, dm, S, pbuf, P, vout, ex, stream);
    case 1 << 17: return launch_large_t<17>(p, xt, dm, S, pbuf, P, vout, ex, stream);
    case 1 << 18: return launch_large_t<18>(p, xt, dm, S, pbuf, P, vout, ex, stream);
    case 1 << 19: return launch_large_t<19>(p, xt, dm, S, pbuf, P, vout, ex, stream);
    case 1 << 20: return launch_large_t<20>(p, xt, dm, S, pbuf, P, vout, ex, stream);
    case 1 << 21: return launch_large_t<21>(p, xt, dm, S, pbuf, P, vout, ex, stream);
    case 1 << 22: return launch_large_t<22>(p, xt, dm, S, pbuf, P, vout, ex, stream);
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace cdd
