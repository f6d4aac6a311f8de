// Fused per-(channel, block) coherent dedispersion kernel for gfx950.
//
// One workgroup owns one overlap-save block of one channel (N <= 16384):
//   load N samples (int8 or float complex) -> FP32 registers
//   forward FFT: Stockham autosort radix passes, butterflies in registers,
//                exchanges through LDS (real and imaginary halves in turn)
//   chirp:       exp(-2 pi i q_j)/N per bin, q_j from Eq. 3 evaluated in FP64
//                and reduced to [-1/2, 1/2] turns; with one DM it is read
//                from a per-channel table built once per call,
//                with several it is formed in the kernel (FP32 sin/cos)
//   inverse FFT: the same passes in reverse radix order, conjugate twiddles;
//                its first pass consumes the forward result in registers
//   epilogue:    keep samples [nfront, nfront + M), |y|^2, sum n_int samples
//                (optionally also write the dedispersed voltages)
// With several DM trials the forward spectrum stays in registers and the
// chirp, inverse transform and epilogue repeat per trial.
//
// Transform conventions follow the paper's use of FFTW/cuFFT (Sec. 3, 4.1):
// forward exp(-2 pi i j n/N), inverse exp(+2 pi i j n/N) with 1/N.  The
// butterflies are radix-2/4 compositions with constants folded at compile
// time; inter-pass twiddles come from tables computed on the host in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <utility>
#include <vector>

#include "cdd_fft.h"
#include "cdd_internal.h"

namespace cdd {

// Schedules per length; variant 0 is the default, others are autotuner
// candidates.
template <int N, int V>
struct SchedFor;
template <> struct SchedFor<256, 0> { using type = Sched<256, 64, 4, 4, 4, 4>; };
template <> struct SchedFor<512, 0> { using type = Sched<512, 64, 8, 8, 8, 1>; };
template <> struct SchedFor<1024, 0> { using type = Sched<1024, 64, 16, 16, 4, 1>; };
template <> struct SchedFor<2048, 0> { using type = Sched<2048, 128, 16, 16, 8, 1>; };
template <> struct SchedFor<4096, 0> { using type = Sched<4096, 128, 16, 16, 16, 1, true, true, 3>; };
template <> struct SchedFor<4096, 1> { using type = Sched<4096, 256, 16, 16, 16, 1, false, false, 2>; };
template <> struct SchedFor<4096, 2> { using type = Sched<4096, 256, 16, 16, 16, 1, true, true, 3>; };
template <> struct SchedFor<4096, 3> { using type = Sched<4096, 256, 16, 16, 16, 1, true, false, 3>; };
template <> struct SchedFor<8192, 0> { using type = Sched<8192, 256, 16, 16, 32, 1, true, false, 3>; };
template <> struct SchedFor<8192, 1> { using type = Sched<8192, 512, 16, 16, 16, 2, true, true, 4>; };
template <> struct SchedFor<8192, 2> { using type = Sched<8192, 512, 16, 16, 16, 2, true, false, 6>; };
template <> struct SchedFor<8192, 3> { using type = Sched<8192, 512, 16, 16, 16, 2, false, true, 4>; };
template <> struct SchedFor<8192, 4> { using type = Sched<8192, 256, 32, 16, 16, 1, true, true, 3>; };
template <> struct SchedFor<8192, 5> { using type = Sched<8192, 256, 16, 32, 16, 1, true, true, 3>; };
template <> struct SchedFor<8192, 6> { using type = Sched<8192, 256, 16, 16, 32, 1, true, true, 3>; };
template <> struct SchedFor<8192, 7> { using type = Sched<8192, 256, 16, 16, 32, 1, true, true, 2>; };
template <> struct SchedFor<8192, 8> { using type = Sched<8192, 256, 16, 16, 32, 1, true, false, 4>; };
template <> struct SchedFor<8192, 9> { using type = Sched<8192, 128, 16, 16, 32, 1, true, false, 2>; };
template <> struct SchedFor<16384, 0> { using type = Sched<16384, 512, 16, 32, 32, 1, true, true, 2>; };
template <> struct SchedFor<16384, 1> { using type = Sched<16384, 512, 16, 32, 32, 1, false, false, 2>; };
template <> struct SchedFor<16384, 2> { using type = Sched<16384, 1024, 16, 16, 16, 4, true, false, 4>; };
template <> struct SchedFor<16384, 3> { using type = Sched<16384, 512, 32, 32, 16, 1, true, true, 2>; };
constexpr int kVariants[] = {1, 1, 1, 1, 4, 10, 4};  // per log2(N) - 8

// ---------------------------------------------------------------------------
// Kernel
// ---------------------------------------------------------------------------
// One beam's launch description.  Coordinates are relative to this launch:
// block k reads input samples k*M - load_off + n (valid in [0, x_len)) and
// yields output samples o = k*M + m, m < M, and integrated samples
// u = k*M/n_int + ul.
struct BlockArgs {
  const void* x;        // channel-major input, channel stride x_stride (int8x2 or float2)
  float* P;             // P[dmi*p_dm_stride + c*p_stride + u]
  float2* vout;         // vout[c*v_stride + o] or null (single DM only)
  const float2* tw;     // twiddle tables
  const float2* H;      // single DM: chirp table H[c*N + i] (see chirp_table_kernel)
  int64_t x_stride, x_len, load_off;
  int64_t p_stride, p_dm_stride, u_lim;
  int64_t v_stride, o_lim;
  int64_t nblocks, item0;   // blocks per channel; first work item of this beam
  int32_t nchan, M, nfront, n_int, dtype, phase_mode, exact_div, taper;
  int32_t accum;        // add to P instead of storing (second polarisation)
  int32_t lgn;          // log2 N (mixed launches switch on it)
  double f_lo, df, dconst;
  double dm_step;       // DM tiles: dms.dm[i] = dms.dm[0] + i dm_step, or 0 if not so spaced
  DmTile dms;
};

// Bin i of the forward transform holds the spectrum at offset f = s*df/N from
// the channel centre fc, s = i (i < N/2) or i - N.  Multiply it by
// exp(-2 pi i q)/N with q = D*DM*f^2/(fc^2 (fc + f)) turns (Eq. 3), evaluated
// in FP64 as q = B s^2 / (1 + x), B = D*DM*(df/N)^2/fc^3, x = s*(df/N)/fc.
// When the channel is narrow enough that q*x^3 stays below 1e-9 turns, 1/(1+x)
// is replaced by 1 - x + x^2 (no division); otherwise the division is exact.
// The phase is reduced to r = q - rint(q) in [-1/2, 1/2] turns in FP64; the
// rotation takes the hardware sine and cosine, whose argument is in turns
// (absolute error about 1.2e-7 on [-1/2, 1/2]).
template <class S>
__device__ __forceinline__ void apply_chirp(float2* v, double dm, double fc, const BlockArgs& a,
                                            int t) {
  constexpr int N = S::N, R = S::rad_f(S::NP - 1), BPT = N / (R * S::T);
  // This thread holds bins i = (t + T b) + r N/R with t + T b < N/R, so
  // i >= N/2 exactly when r >= R/2: the signed bin is a per-b base plus a
  // compile-time constant per r.  The spectrum arrives already scaled by
  // 1/N (once per item, not once per trial).
  if (a.phase_mode == CDD_PHASE_FP64_REDUCED) {
    const double dfn = a.df / (double)N;
    const double B = a.dconst * dm * dfn * dfn / (fc * fc * fc);  // turns
    const double beta = dfn / fc;
    const double Bb = B * beta, Bbb = Bb * beta;
    auto rot = [&](float2 z, double q) {
      const float r = (float)(q - rint(q));
      const float c = __builtin_amdgcn_cosf(r), s = __builtin_amdgcn_sinf(r);
      return make_float2(z.x * c + z.y * s, z.y * c - z.x * s);  // z (c - i s)
    };
    if (a.exact_div == 0) {
      // B s^2 (1 - x + x^2), x = beta s, as s^2 (B + s (-B beta + s B beta^2))
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const double s0 = (double)(t + S::T * b);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double sd = s0 + (double)(r * (N / R) - (2 * r >= R ? N : 0));
          v[b * R + r] = rot(v[b * R + r], (sd * sd) * fma(sd, fma(sd, Bbb, -Bb), B));
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const double s0 = (double)(t + S::T * b);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double sd = s0 + (double)(r * (N / R) - (2 * r >= R ? N : 0));
          v[b * R + r] = rot(v[b * R + r], (B * (sd * sd)) / fma(beta, sd, 1.0));
        }
      }
    }
  } else {
    // all-FP32 phase (precision study): q straight from Eq. 3 in FP32
    const float fcf = (float)fc;
    const float Af = (float)(a.dconst * dm) / (fcf * fcf);
    const float dfn = (float)a.df / (float)N;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = t + S::T * b + r * (N / R);
        const int s = i < N / 2 ? i : i - N;
        const float f = (float)s * dfn;
        const float q = Af * (f * f) / (fcf + f);
        float sn, cs;
        sincospif(2.0f * q, &sn, &cs);
        v[b * R + r] = cmul(v[b * R + r], make_float2(cs, -sn));
      }
    }
  }
}

// The chirp phase is linear in DM (Eq. 3: q = DM x a function of the bin),
// so a tile of DM trials forms the per-unit-DM phase of every bin of its
// channel once per work item, in FP64 with the same expression as
// apply_chirp at DM = 1, and each trial then costs one FP64 multiply per bin
// before the same reduction and rotation.  Entry (b R + r) T + t belongs to
// thread t alone (written and read by it, no barrier needed).
template <class S>
__device__ __forceinline__ void chirp_phase_per_dm(double* qd, double fc, const BlockArgs& a,
                                                   int t) {
  constexpr int N = S::N, R = S::rad_f(S::NP - 1), BPT = N / (R * S::T);
  const double dfn = a.df / (double)N;
  const double B = a.dconst * dfn * dfn / (fc * fc * fc);  // turns per unit DM
  const double beta = dfn / fc;
  const double Bb = B * beta, Bbb = Bb * beta;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const double s0 = (double)(t + S::T * b);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double sd = s0 + (double)(r * (N / R) - (2 * r >= R ? N : 0));
      qd[(b * R + r) * S::T + t] = a.exact_div ? (B * (sd * sd)) / fma(beta, sd, 1.0)
                                               : (sd * sd) * fma(sd, fma(sd, Bbb, -Bb), B);
    }
  }
}

template <class S>
__device__ __forceinline__ void apply_chirp_dm(float2* v, double dm, const double* qd, int t) {
  constexpr int N = S::N, R = S::rad_f(S::NP - 1), BPT = N / (R * S::T);
#pragma unroll
  for (int b = 0; b < BPT; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double q = dm * qd[(b * R + r) * S::T + t];
      const float x = (float)(q - rint(q));
      const float c = __builtin_amdgcn_cosf(x), sn = __builtin_amdgcn_sinf(x);
      const float2 z = v[b * R + r];
      v[b * R + r] = make_float2(z.x * c + z.y * sn, z.y * c - z.x * sn);  // z (c - i s)
    }
  (void)N;
}

// exp(-2 pi i x) for |x| <= 1/2 turn, rounded to FP32: the quadrant
// n = rint(4x) is taken out exactly, and the sine and cosine of the remaining
// angle (at most pi/4) come from their Taylor series in FP64 through the
// 11th and 12th powers (truncation below 1e-11, far under FP32 rounding).
__device__ __forceinline__ float2 expi_neg_turns_fp64(double x) {
  const double n = rint(4.0 * x);
  const double th = 6.283185307179586 * fma(n, -0.25, x);
  const double t2 = th * th;
  double sp = fma(t2, -2.505210838544172e-08, 2.755731922398589e-06);  // 1/11!, 1/9!
  sp = fma(t2, sp, -1.984126984126984e-04);                            // 1/7!
  sp = fma(t2, sp, 8.333333333333333e-03);                             // 1/5!
  sp = fma(t2, sp, -1.666666666666667e-01);                            // 1/3!
  const double sv = fma(th * t2, sp, th);
  double cp = fma(t2, 2.087675698786810e-09, -2.755731922398589e-07);  // 1/12!, 1/10!
  cp = fma(t2, cp, 2.480158730158730e-05);                             // 1/8!
  cp = fma(t2, cp, -1.388888888888889e-03);                            // 1/6!
  cp = fma(t2, cp, 4.166666666666667e-02);                             // 1/4!
  cp = fma(t2, cp, -0.5);
  const double cv = fma(t2, cp, 1.0);
  // rotate by the quadrant: exp(2 pi i x) = i^n exp(i th)
  const int q = ((int)n) & 3;
  const double c = q == 0 ? cv : q == 1 ? -sv : q == 2 ? -cv : sv;
  const double sn = q == 0 ? sv : q == 1 ? cv : q == 2 ? -sv : -cv;
  return make_float2((float)c, (float)-sn);
}

// Evenly spaced DM trials, DM_i = DM_0 + i step: the chirp of trial i + 1 is
// that of trial i times exp(-2 pi i step Q) with Q the per-unit-DM phase of
// the bin (Eq. 3 is linear in DM), so a tile keeps the chirped spectrum of
// the current trial and advances it by one complex multiply per bin and
// trial instead of forming the FP64 phase and its sine and cosine again.
// The first trial's chirp and then the step rotation of every bin are formed
// once per work item in FP64 (phase reduced to [-1/2, 1/2] turns, then an
// FP64 sine and cosine) and rounded to FP32 once, so each step carries the
// same relative error of at most 2^-24 sqrt 2 (8.4e-8) in the rotation, plus
// the rounding of the product: after k steps the chirp is off by at most
// about k 1e-7 (6e-6 relative at the 64th trial of a tile; measured on the
// 512-channel beam, the intensities of 64 trials differ from 64 one-DM calls
// by 1.1e-7 relative L2).  Entry (b R + r) T + t belongs to thread t alone,
// as in chirp_phase_per_dm (whose LDS the table takes).
// rs[] receives exp(-2 pi i DM Q) of this thread's bins for the given DM.
template <class S>
__device__ __forceinline__ void rotation_table(float2* rs, double dm, double fc,
                                               const BlockArgs& a, int t) {
  constexpr int N = S::N, R = S::rad_f(S::NP - 1), BPT = N / (R * S::T);
  const double dfn = a.df / (double)N;
  const double B = a.dconst * dm * dfn * dfn / (fc * fc * fc);  // turns
  const double beta = dfn / fc;
  const double Bb = B * beta, Bbb = Bb * beta;
#pragma unroll 1
  for (int b = 0; b < BPT; ++b) {
    const double s0 = (double)(t + S::T * b);
#pragma unroll 1
    for (int r = 0; r < R; ++r) {
      const double sd = s0 + (double)(r * (N / R) - (2 * r >= R ? N : 0));
      const double q = a.exact_div ? (B * (sd * sd)) / fma(beta, sd, 1.0)
                                   : (sd * sd) * fma(sd, fma(sd, Bbb, -Bb), B);
      rs[(b * R + r) * S::T + t] = expi_neg_turns_fp64(q - rint(q));
    }
  }
}

template <class S>
__device__ __forceinline__ void step_chirp(float2* y, const float2* rs, int t) {
#pragma unroll
  for (int e = 0; e < S::E; ++e) y[e] = cmul(y[e], rs[e * S::T + t]);
}

// Taper (Sec. 2.2) on the bins this thread holds after the forward transform
// (same bin layout as apply_chirp).
template <class S>
__device__ __forceinline__ void apply_taper(float2* v, int kind, int t) {
  constexpr int N = S::N, R = S::rad_f(S::NP - 1), BPT = N / (R * S::T);
  constexpr float inv_n = 1.0f / (float)N;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = t + S::T * b + r * (N / R) - (2 * r >= R ? N : 0);
      const float w = taper_gain<false>(kind, (float)s * inv_n);
      v[b * R + r] = make_float2(v[b * R + r].x * w, v[b * R + r].y * w);
    }
  }
}

// Single DM: multiply by the channel's chirp row h[i] (bins in natural order).
// The row is read through a buffer resource so that the per-bin offsets are
// compile-time constants in scalar registers; consecutive lanes read
// consecutive bins.
template <class S>
__device__ __forceinline__ void chirp_from_table(float2* v, const float2* h, int t) {
  constexpr int N = S::N, R = S::rad_f(S::NP - 1), BPT = N / (R * S::T);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)h, (short)0, N * 8, 0x00020000);
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int soff = (S::T * b + r * (N / R)) * 8;
      const float2 w =
          __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, t * 8, soff, 0));
      v[b * R + r] = cmul(v[b * R + r], w);
    }
  }
}

// Load block k of channel c: sample n of the block is input sample
// k*M - load_off + n, zero outside [0, x_len).  Blocks that start inside the
// data read through a buffer resource whose range ends at the data's end, so
// the hardware returns zeros past it and no per-sample test is needed.
template <class S, int DT>
__device__ __forceinline__ void load_block(float2* v, const BlockArgs& a, int c, int64_t k, int t) {
  constexpr int N = S::N, R = S::rad_f(0), BPT = N / (R * S::T);
  constexpr int ES = DT == CDD_CI8 ? 2 : 8;
  const int64_t t0 = k * a.M - a.load_off;
  if (t0 >= 0) {
    const int64_t avail = a.x_len - t0;
    const int nrec = (int)(avail < N ? avail * ES : (int64_t)N * ES);
    const char* base = (const char*)a.x + ((int64_t)c * a.x_stride + t0) * ES;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, nrec, 0x00020000);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int soff = (S::T * b + r * (N / R)) * ES;
        if constexpr (DT == CDD_CI8) {
          const unsigned short w = __builtin_amdgcn_raw_buffer_load_b16(rs, t * ES, soff, 0);
          v[b * R + r] = make_float2((float)(signed char)(w & 0xff), (float)(signed char)(w >> 8));
        } else {
          // the whole 64-bit result reinterpreted at once: indexing its two
          // halves separately compiles to a single 32-bit load here
          v[b * R + r] =
              __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, t * ES, soff, 0));
        }
      }
    }
    return;
  }
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = t + S::T * b + r * (N / R);
      const int64_t tt = t0 + n;
      float2 z = make_float2(0.f, 0.f);
      if (tt >= 0 && tt < a.x_len) {
        if constexpr (DT == CDD_CI8) {
          const short w = gptr((const short*)a.x)[(int64_t)c * a.x_stride + tt];
          z = make_float2((float)(signed char)(w & 0xff), (float)(signed char)(w >> 8));
        } else {
          z = gload2((const float2*)a.x, (int64_t)c * a.x_stride + tt);
        }
      }
      v[b * R + r] = z;
    }
  }
}

template <class S, bool VOUT>
__device__ __forceinline__ void epilogue(const float2* v, float* lds, const BlockArgs& a, int c,
                                         int64_t k, int dmi, int t, bool live = true) {
  constexpr int N = S::N, R = S::rad_i(S::NP - 1), BPT = N / (R * S::T);
  if constexpr (VOUT) {
    if (a.vout && live) {
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int n = t + S::T * b + r * (N / R);
          const int m = n - a.nfront;
          const int64_t o = k * a.M + m;
          if (m >= 0 && m < a.M && o < a.o_lim) gstore2(a.vout, (int64_t)c * a.v_stride + o, v[b * R + r]);
        }
      }
    }
  }
  // |z|^2 to LDS in natural order (unpadded: consecutive lanes write
  // consecutive words), then each output sums n_int consecutive words.
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = t + S::T * b + r * (N / R);
      const float2 z = v[b * R + r];
      lds[n] = z.x * z.x + z.y * z.y;
    }
  }
  __syncthreads();
  if (!live) return;  // a workgroup's spare transform: its barriers only
  const int nu = a.M / a.n_int;
  const int64_t u0 = k * (a.M / a.n_int);
  const auto P = gptr(a.P) + (int64_t)dmi * a.p_dm_stride + (int64_t)c * a.p_stride;
  if (a.n_int == 4 && (a.nfront & 3) == 0) {
    for (int ul = t; ul < nu; ul += S::T) {
      const int64_t u = u0 + ul;
      if (u >= a.u_lim) break;
      const float4 q = *(const float4*)&lds[a.nfront + 4 * ul];
      const float s = ((q.x + q.y) + q.z) + q.w;
      P[u] = a.accum ? P[u] + s : s;
    }
  } else {
    for (int ul = t; ul < nu; ul += S::T) {
      const int64_t u = u0 + ul;
      if (u >= a.u_lim) break;
      const int base = a.nfront + ul * a.n_int;
      float s = 0.f;
      for (int r = 0; r < a.n_int; ++r) s += lds[base + r];
      P[u] = a.accum ? P[u] + s : s;
    }
  }
}

// qd: N doubles of LDS for the per-unit-DM chirp phase (DM tiles with the
// FP64 phase), or null to form the phase per trial.
template <class S, int DT, bool MULTI>
__device__ __forceinline__ void process_item(const BlockArgs& a, int c, int64_t k, float* lds,
                                             int t, bool live = true, double* qd = nullptr) {
  const double fc = a.f_lo + ((double)c + 0.5) * a.df;
  // evenly spaced DM trials: the step rotations, formed before anything else
  // holds registers (the entries are this thread's own)
  const bool stepped = MULTI && qd != nullptr && a.phase_mode == CDD_PHASE_FP64_REDUCED &&
                       a.dm_step != 0.0;
  if (stepped) rotation_table<S>(reinterpret_cast<float2*>(qd), a.dms.dm[0], fc, a, t);
  float2 v[S::E];
  load_block<S, DT>(v, a, c, k, t);
  fft_forward<S>(v, lds, a.tw, t);
  if constexpr (!MULTI) {
    (void)fc;
    int tt = t;  // opaque copy: keeps per-bin index math next to its use
    asm volatile("" : "+v"(tt));
    chirp_from_table<S>(v, a.H + (int64_t)c * S::N, tt);
    fft_inverse<S>(v, lds, a.tw, tt);
    epilogue<S, true>(v, lds, a, c, k, 0, tt, live);
  } else {
    // The taper depends on the bin only: it scales the shared spectrum once,
    // and the per-trial chirp is a pure rotation.
    if (a.taper) apply_taper<S>(v, a.taper, t);
    // the inverse transform's 1/N (a power of two, so exact) once per item
    constexpr float inv_n = 1.0f / (float)S::N;
    float2 X[S::E];
#pragma unroll
    for (int e = 0; e < S::E; ++e) X[e] = make_float2(v[e].x * inv_n, v[e].y * inv_n);
    const bool per_dm = qd != nullptr && a.phase_mode == CDD_PHASE_FP64_REDUCED;
    if (stepped) {
      // X becomes the chirped spectrum of the current trial; the table then
      // takes the step rotation
      float2* rs = reinterpret_cast<float2*>(qd);
      step_chirp<S>(X, rs, t);
      rotation_table<S>(rs, a.dm_step, fc, a, t);
      for (int i = 0; i < a.dms.ndm; ++i) {
        int tt = t;
        asm volatile("" : "+v"(tt));
#pragma unroll
        for (int e = 0; e < S::E; ++e) v[e] = X[e];
        fft_inverse<S>(v, lds, a.tw, tt);
        epilogue<S, false>(v, lds, a, c, k, i, tt, live);
        if (i + 1 < a.dms.ndm) step_chirp<S>(X, rs, tt);
      }
      return;
    }
    if (per_dm) chirp_phase_per_dm<S>(qd, fc, a, t);
    for (int i = 0; i < a.dms.ndm; ++i) {
      // Per-bin indices do not depend on the DM; an opaque copy of the
      // thread index keeps the compiler from hoisting them (and holding them
      // in registers) across the whole loop.
      int tt = t;
      asm volatile("" : "+v"(tt));
#pragma unroll
      for (int e = 0; e < S::E; ++e) v[e] = X[e];
      if (per_dm)
        apply_chirp_dm<S>(v, a.dms.dm[i], qd, tt);
      else
        apply_chirp<S>(v, a.dms.dm[i], fc, a, tt);
      fft_inverse<S>(v, lds, a.tw, tt);
      epilogue<S, false>(v, lds, a, c, k, i, tt, live);
    }
  }
}

// DM tiles keep the per-unit-DM chirp phase in LDS up to 4096 points (8 N
// bytes beside the exchange buffer, within what the register budget's
// occupancy leaves); longer transforms form the phase per trial.
template <class S>
constexpr bool qd_in_lds() {
  return S::N <= 4096;
}

// Workgroups are dispatched round-robin over the XCDs (8 on this chip, each
// with its own L2).  Workgroup w runs on XCD w % 8; giving XCD x the
// contiguous item range [x q + min(x, r), ...) of its own (total = 8 q + r)
// keeps the blocks of one channel, and so its chirp row and the overlap
// between neighbouring blocks, in one L2.  A bijection for any total.
__device__ __forceinline__ int64_t xcd_item(int64_t w, int64_t total) {
  constexpr int X = 8;
  const int64_t q = total / X, r = total - q * X;
  const int64_t x = w % X, slot = w / X;
  return x * q + (x < r ? x : r) + slot;
}

// One workgroup per (channel, block) of one beam.
template <class S, int DT, bool MULTI>
__global__ __launch_bounds__(S::T, MULTI ? (S::MINB + 1) / 2 : S::MINB) void block_kernel(
    const BlockArgs a) {
  __shared__ __align__(16) float lds[S::lds_floats()];
  constexpr bool QD = MULTI && qd_in_lds<S>();
  __shared__ double qd[QD ? S::N : 1];
  const int64_t item = xcd_item(blockIdx.x, (int64_t)gridDim.x);
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  process_item<S, DT, MULTI>(a, c, k, lds, threadIdx.x, true, QD ? qd : nullptr);
}

// Persistent form for several beams sharing one transform length and sample
// type (one instantiation per type: a run-time switch between the two load
// paths makes the register allocator spill): a grid sized to the machine
// pulls work items (beam, channel, block) from a counter until all are
// taken; beams are listed longest work first.  Every wave leaves the loop
// once the counter passes the item count.
template <class S, int DT>
__global__ __launch_bounds__(S::T, (S::MINB + 1) / 2) void batch_kernel(
    const BlockArgs* __restrict__ beams, int32_t nbeams, int64_t total,
    unsigned int* __restrict__ counter) {
  __shared__ __align__(16) float lds[S::lds_floats()];
  constexpr bool QD = qd_in_lds<S>();
  __shared__ double qd[QD ? S::N : 1];
  __shared__ unsigned int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    // uniform across the workgroup: kept in a scalar register, so the beam's
    // arguments below are scalar loads and stay out of the vector registers
    const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= total) break;
    int b = 0;
    while (b + 1 < nbeams && item >= beams[b + 1].item0) ++b;
    const BlockArgs& a = beams[b];
    const int64_t local = item - a.item0;
    const int c = (int)(local / a.nblocks);
    const int64_t k = local - (int64_t)c * a.nblocks;
    // an opaque copy of the thread index per item keeps the compiler from
    // hoisting per-thread index math out of this loop (and holding it in
    // registers across it)
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    process_item<S, DT, true>(a, c, k, lds, t, true, QD ? qd : nullptr);
  }
}

// Several one-DM beams of one transform length in one launch: one workgroup
// per (beam, channel, block) over the concatenated items (beams listed with
// their first item), XCD-aware as block_kernel; each beam's chirp comes from
// its own table.
template <class S, int DT>
__global__ __launch_bounds__(S::T, S::MINB) void multi_single_kernel(
    const BlockArgs* __restrict__ beams, int32_t nbeams, int64_t total) {
  __shared__ __align__(16) float lds[S::lds_floats()];
  const int64_t item = xcd_item(blockIdx.x, total);
  int b = 0;
  while (b + 1 < nbeams && item >= beams[b + 1].item0) ++b;
  const BlockArgs& a = beams[b];
  const int64_t local = item - a.item0;
  const int c = (int)(local / a.nblocks);
  const int64_t k = local - (int64_t)c * a.nblocks;
  process_item<S, DT, false>(a, c, k, lds, threadIdx.x);
}

// ---------------------------------------------------------------------------
// One persistent launch for beams of different transform lengths
// ---------------------------------------------------------------------------
// Workgroups of kMixT threads; a length whose schedule has T < kMixT threads
// runs G = kMixT / T transforms side by side, each on its own slice of the
// LDS.  A unit of work is G consecutive (channel, block) items of one beam;
// the last unit of a beam may hold fewer items, and its spare transforms run
// on a valid block without storing anything (they keep the workgroup's
// barriers in step).  Beams are listed longest work per unit first; the
// workgroups pull units from a counter until none are left, and every wave
// leaves the loop once the counter passes the unit count.
constexpr int kMixT = 256;
template <int N>
struct MixSchedOf {
  using type = typename SchedFor<N, 0>::type;
};
// 4096 with 256 threads (its default 128-thread schedule prefetches twiddles
// and needs more registers than the one-DM budget holds)
template <>
struct MixSchedOf<4096> {
  using type = typename SchedFor<4096, 3>::type;
};
template <int N>
using MixSched = typename MixSchedOf<N>::type;
template <class S>
constexpr int mix_lds_floats() {
  return (kMixT / S::T) * S::lds_floats();
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kMixLds =
    cmax(cmax(cmax(mix_lds_floats<MixSched<256>>(), mix_lds_floats<MixSched<512>>()),
              cmax(mix_lds_floats<MixSched<1024>>(), mix_lds_floats<MixSched<2048>>())),
         cmax(mix_lds_floats<MixSched<4096>>(), mix_lds_floats<MixSched<8192>>()));
constexpr bool mix_len_ok(int lg) { return lg >= 8 && lg <= 13; }
static_assert(MixSched<8192>::T == kMixT && MixSched<256>::T <= kMixT, "mixed schedules");

template <class S, int DT, bool MULTI>
__device__ __forceinline__ void mix_unit(const BlockArgs& a, int64_t unit, float* lds) {
  constexpr int G = kMixT / S::T;
  static_assert(G * S::T == kMixT, "schedule threads must divide the workgroup");
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));  // per-unit opaque copy (see batch_kernel)
  const int g = tid / S::T, t = tid - g * S::T;
  const int64_t items = (int64_t)a.nchan * a.nblocks;
  int64_t item = unit * G + g;
  const bool live = item < items;
  if (!live) item = 0;  // a valid block, nothing stored
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  float* my = lds + g * S::lds_floats();
  if (MULTI && a.H == nullptr)
    process_item<S, DT, true>(a, c, k, my, t, live);
  else
    process_item<S, DT, false>(a, c, k, my, t, live);
}

// MULTI: some beam carries DM trials or generates its one-DM chirp in the
// kernel (register budget of the batched path); otherwise every beam reads
// its chirp table (register budget of the one-DM path).  DT: the sample type
// of every beam in the launch.
template <bool MULTI, int DT>
__global__ __launch_bounds__(kMixT, MULTI ? 2 : 3) void mixed_kernel(
    const BlockArgs* __restrict__ beams, int32_t nbeams, int64_t total,
    unsigned int* __restrict__ counter) {
  __shared__ __align__(16) float lds[kMixLds];
  __shared__ unsigned int s_unit;
  for (;;) {
    if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t unit = (int64_t)__builtin_amdgcn_readfirstlane(s_unit);  // scalar (see above)
    __syncthreads();
    if (unit >= total) break;
    int b = 0;
    while (b + 1 < nbeams && unit >= beams[b + 1].item0) ++b;
    const BlockArgs& a = beams[b];
    const int64_t u = unit - a.item0;
    switch (a.lgn) {
      case 8: mix_unit<MixSched<256>, DT, MULTI>(a, u, lds); break;
      case 9: mix_unit<MixSched<512>, DT, MULTI>(a, u, lds); break;
      case 10: mix_unit<MixSched<1024>, DT, MULTI>(a, u, lds); break;
      case 11: mix_unit<MixSched<2048>, DT, MULTI>(a, u, lds); break;
      case 12: mix_unit<MixSched<4096>, DT, MULTI>(a, u, lds); break;
      default: mix_unit<MixSched<8192>, DT, MULTI>(a, u, lds); break;
    }
  }
}

__global__ void zero_counter_kernel(unsigned int* c) { *c = 0u; }

// The one-DM chirp table as a kernel of its own (see chirp_table_part).
__global__ __launch_bounds__(256) void chirp_table_kernel(const ChirpTableArgs a) {
  chirp_table_part(a, blockIdx.x, threadIdx.x);
}

// ---------------------------------------------------------------------------
// Host side: FP64 twiddle tables (cached per device, length and schedule)
// and launch
// ---------------------------------------------------------------------------
// The tables of every schedule live in one static device pool, filled on
// first use per device and kept until the process ends, so that building a
// table never allocates device memory.  Entries are placed at 256-byte
// boundaries.
constexpr size_t kTablePoolEntries = (size_t)1 << 20;  // float2 entries, 8 MiB
static __device__ __align__(256) float2 g_table_pool[kTablePoolEntries];

static std::mutex g_tab_mu;
static std::map<std::pair<int, std::string>, float2*> g_tab;  // (device, key)
struct TablePool {
  float2* base = nullptr;  // this device's copy of g_table_pool
  size_t used = 0;         // entries handed out
};
static std::map<int, TablePool> g_pool;

int cached_table(const char* key, std::vector<float2> (*make)(), const float2** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto k = std::make_pair(dev, std::string(key));
  auto it = g_tab.find(k);
  if (it != g_tab.end()) {
    *out = it->second;
    return 0;
  }
  TablePool& pool = g_pool[dev];
  if (pool.base == nullptr) {
    void* addr = nullptr;
    e = hipGetSymbolAddress(&addr, HIP_SYMBOL(g_table_pool));
    if (e != hipSuccess) return (int)e;
    pool.base = (float2*)addr;
  }
  std::vector<float2> h = make();
  const size_t n = (h.size() + 31) & ~(size_t)31;
  if (pool.used + n > kTablePoolEntries) return (int)hipErrorOutOfMemory;
  float2* d = pool.base + pool.used;
  e = hipMemcpy(d, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return (int)e;
  pool.used += n;
  g_tab[k] = d;
  *out = d;
  return 0;
}

// Whether 1/(1+x) needs the exact division: the series 1 - x + x^2 is used
// when its truncation, q*x^3/(1-x), stays below 1e-9 turns over the beam's
// channels for DMs up to dm_abs_max (x = f/fc, |f| <= df/2).
int exact_division_needed(const BeamPlan& p, double dm_abs_max) {
  const double fmin = p.f_lo + 0.5 * p.df;
  const double xm = 0.5 * p.df / fmin;
  const double qmax =
      p.dconst * dm_abs_max * 0.25 * p.df * p.df / (fmin * fmin * (fmin - 0.5 * p.df));
  return qmax * xm * xm * xm / (1.0 - xm) > 1e-9 ? 1 : 0;
}

static int needs_exact_division(const BeamPlan& p, const DmTile& dms) {
  double dmax = 0;
  for (int i = 0; i < dms.ndm; ++i) dmax = std::fmax(dmax, std::fabs(dms.dm[i]));
  return exact_division_needed(p, dmax);
}

Coords offline_coords(const BeamPlan& p) {
  Coords co;
  co.x_stride = xt_stride(p);
  co.x_len = p.nsamp;
  co.load_off = p.nfront;
  co.p_stride = p.t_int;
  co.p_dm_stride = (int64_t)p.nchan * p.t_int;
  co.u_lim = p.t_int;
  co.v_stride = p.nsamp;
  co.o_lim = p.nsamp;
  co.nblocks = p.nblocks;
  return co;
}

// The step of a tile of three or more DM trials spaced evenly to within
// 1e-13 of the largest |DM| (so the phase of every trial differs from that of
// DM_0 + i step by at most 1e-13 of the largest phase), else 0.
static double even_dm_step(const DmTile& t) {
  if (t.ndm < 3) return 0.0;
  const double step = (t.dm[t.ndm - 1] - t.dm[0]) / (double)(t.ndm - 1);
  double mx = 0.0;
  for (int i = 0; i < t.ndm; ++i) mx = std::max(mx, std::fabs(t.dm[i]));
  if (!(std::fabs(step) > 1e-12 * mx)) return 0.0;
  for (int i = 0; i < t.ndm; ++i)
    if (std::fabs(t.dm[0] + (double)i * step - t.dm[i]) > 1e-13 * mx) return 0.0;
  return step;
}

static BlockArgs make_args(const BeamPlan& p, const Coords& co, const void* xt, const DmTile& dms,
                           float* P, void* vout, const float2* H) {
  BlockArgs a{};
  a.x = xt;
  a.H = H;
  a.P = P;
  a.vout = (float2*)vout;
  a.x_stride = co.x_stride;
  a.x_len = co.x_len;
  a.load_off = co.load_off;
  a.p_stride = co.p_stride;
  a.p_dm_stride = co.p_dm_stride;
  a.u_lim = co.u_lim;
  a.v_stride = co.v_stride;
  a.o_lim = co.o_lim;
  a.nblocks = co.nblocks;
  a.accum = co.accum;
  a.item0 = 0;
  a.lgn = 0;
  while ((1 << a.lgn) < p.N) ++a.lgn;
  a.nchan = p.nchan;
  a.M = p.M;
  a.nfront = p.nfront;
  a.n_int = p.n_int;
  a.dtype = p.dtype;
  a.phase_mode = p.phase_mode;
  a.exact_div = needs_exact_division(p, dms);
  a.taper = p.taper;
  a.f_lo = p.f_lo;
  a.df = p.df;
  a.dconst = p.dconst;
  a.dms = dms;
  a.dm_step = even_dm_step(dms);
  return a;
}

// Workgroups of a persistent kernel that fit on the device at once, per
// (device, kernel), computed once under a lock (callers on several threads
// may launch at the same time).
static std::mutex g_occ_mu;
static std::map<std::pair<int, const void*>, int64_t> g_occ;

static int resident_workgroups(const void* fn, int threads, int64_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  auto key = std::make_pair(dev, fn);
  auto it = g_occ.find(key);
  if (it != g_occ.end()) {
    *out = it->second;
    return 0;
  }
  int ncu = 0, per_cu = 0;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return (int)e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0)) != hipSuccess)
    return (int)e;
  const int64_t n = (int64_t)std::max(ncu, 1) * std::max(per_cu, 1);
  g_occ[key] = n;
  *out = n;
  return 0;
}

template <int N, int V>
static int launch_block_t(const BlockArgs& a0, void* stream) {
  using S = typename SchedFor<N, V>::type;
  BlockArgs a = a0;
  int err = twiddles_of<S>(&a.tw);
  if (err) return err;
  const int64_t items = (int64_t)a.nchan * a.nblocks;
  if (items <= 0 || items > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  dim3 grid((unsigned)items), block(S::T);
  hipStream_t st = (hipStream_t)stream;
  const bool multi = a.dms.ndm > 1;
  if (a.dtype == CDD_CI8) {
    if (multi) hipLaunchKernelGGL((block_kernel<S, CDD_CI8, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((block_kernel<S, CDD_CI8, false>), grid, block, 0, st, a);
  } else {
    if (multi) hipLaunchKernelGGL((block_kernel<S, CDD_CF32, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((block_kernel<S, CDD_CF32, false>), grid, block, 0, st, a);
  }
  return (int)hipGetLastError();
}

// Persistent batched launch; host_tab must stay unchanged until the copy has
// run (the plan and the server keep it for that long), dev_tab and counter
// are device memory.
static int log2i(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

bool block_supported(int N) {
  return N >= 256 && N <= 16384 && (N & (N - 1)) == 0;
}

int block_variants(int N) { return block_supported(N) ? kVariants[log2i(N) - 8] : 0; }

int launch_block(const BeamPlan& p, const void* xt, const DmTile& dms, float* P, void* vout,
                 const void* H, void* stream) {
  return launch_block_co(p, offline_coords(p), xt, dms, P, vout, H, stream);
}

int launch_block_co(const BeamPlan& p, const Coords& co, const void* xt, const DmTile& dms,
                    float* P, void* vout, const void* H, void* stream) {
  if (dms.ndm < 1 || dms.ndm > kMaxDmTile) return (int)hipErrorInvalidValue;
  if (dms.ndm == 1 && H == nullptr) return (int)hipErrorInvalidValue;  // one DM needs its table
  const BlockArgs a = make_args(p, co, xt, dms, P, vout, (const float2*)H);
  const int v = p.variant;
  switch (p.N) {
    case 256: return launch_block_t<256, 0>(a, stream);
    case 512: return launch_block_t<512, 0>(a, stream);
    case 1024: return launch_block_t<1024, 0>(a, stream);
    case 2048: return launch_block_t<2048, 0>(a, stream);
    case 4096:
      switch (v) {
        case 1: return launch_block_t<4096, 1>(a, stream);
        case 2: return launch_block_t<4096, 2>(a, stream);
        case 3: return launch_block_t<4096, 3>(a, stream);
        default: return launch_block_t<4096, 0>(a, stream);
      }
    case 8192:
      switch (v) {
        case 1: return launch_block_t<8192, 1>(a, stream);
        case 2: return launch_block_t<8192, 2>(a, stream);
        case 3: return launch_block_t<8192, 3>(a, stream);
        case 4: return launch_block_t<8192, 4>(a, stream);
        case 5: return launch_block_t<8192, 5>(a, stream);
        case 6: return launch_block_t<8192, 6>(a, stream);
        case 7: return launch_block_t<8192, 7>(a, stream);
        case 8: return launch_block_t<8192, 8>(a, stream);
        case 9: return launch_block_t<8192, 9>(a, stream);
        default: return launch_block_t<8192, 0>(a, stream);
      }
    case 16384:
      switch (v) {
        case 1: return launch_block_t<16384, 1>(a, stream);
        case 2: return launch_block_t<16384, 2>(a, stream);
        case 3: return launch_block_t<16384, 3>(a, stream);
        default: return launch_block_t<16384, 0>(a, stream);
      }
  }
  return (int)hipErrorInvalidValue;
}

size_t batch_table_bytes(int nbeams) { return sizeof(BlockArgs) * (size_t)nbeams; }

size_t chirp_table_bytes(const BeamPlan& p) {
  return block_supported(p.N) ? (size_t)p.nchan * p.N * sizeof(float2) : 0;
}

ChirpTableArgs chirp_table_args(const BeamPlan& p, double dm, void* H, int kpt) {
  ChirpTableArgs a{};
  a.H = (float2*)H;
  a.f_lo = p.f_lo;
  a.df = p.df;
  a.dconst = p.dconst;
  a.dm = dm;
  a.lgN = log2i(p.N);
  a.kpt = kpt;
  a.phase_mode = p.phase_mode;
  a.taper = p.taper;
  a.exact_div = exact_division_needed(p, std::fabs(dm));
  a.nwg = (uint32_t)((int64_t)p.nchan * (p.N / (256 * kpt)));
  return a;
}

int launch_chirp_table(const BeamPlan& p, double dm, void* H, void* stream) {
  if (!block_supported(p.N) || H == nullptr) return (int)hipErrorInvalidValue;
  const int kpt = std::max(1, std::min(8, p.N / 256));
  const int64_t grid = (int64_t)p.nchan * (p.N / (256 * kpt));
  if (grid > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(chirp_table_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                     chirp_table_args(p, dm, H, kpt));
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched launches in two steps: prepare_launch forms the table of per-beam
// arguments in host memory, enqueue_launch copies it to the device and
// launches.  The host table must stay unchanged until the stream has run the
// copy (the plan keeps it in pinned memory and rewrites it only after the
// previous copy; the server keeps one per batch in flight).
// ---------------------------------------------------------------------------
bool batch_variant_ok(int N, int V) {
  if (V == 0) return block_supported(N);
  if (N == 4096) return V == 3;
  if (N == 8192) return V == 1 || V == 2;
  if (N == 16384) return V == 2;
  return false;
}

bool mixed_supported(int N) { return N >= 256 && N <= 8192 && (N & (N - 1)) == 0; }

static int mix_group(int N) {
  switch (N) {
    case 256: return kMixT / MixSched<256>::T;
    case 512: return kMixT / MixSched<512>::T;
    case 1024: return kMixT / MixSched<1024>::T;
    case 2048: return kMixT / MixSched<2048>::T;
    case 4096: return kMixT / MixSched<4096>::T;
    case 8192: return kMixT / MixSched<8192>::T;
  }
  return 0;
}

// Twiddle table of the schedule a launch kind runs for (N, V).
static int launch_twiddles(int kind, int N, int V, const float2** tw) {
  if (kind == kLaunchMixed) {
    switch (N) {
      case 256: return twiddles_of<MixSched<256>>(tw);
      case 512: return twiddles_of<MixSched<512>>(tw);
      case 1024: return twiddles_of<MixSched<1024>>(tw);
      case 2048: return twiddles_of<MixSched<2048>>(tw);
      case 4096: return twiddles_of<MixSched<4096>>(tw);
      case 8192: return twiddles_of<MixSched<8192>>(tw);
    }
    return (int)hipErrorInvalidValue;
  }
  if (kind == kLaunchBatch && V != 0) {
    if (N == 4096 && V == 3) return twiddles_of<SchedFor<4096, 3>::type>(tw);
    if (N == 8192 && V == 1) return twiddles_of<SchedFor<8192, 1>::type>(tw);
    if (N == 8192 && V == 2) return twiddles_of<SchedFor<8192, 2>::type>(tw);
    if (N == 16384 && V == 2) return twiddles_of<SchedFor<16384, 2>::type>(tw);
    return (int)hipErrorInvalidValue;
  }
  switch (N) {
    case 256: return twiddles_of<SchedFor<256, 0>::type>(tw);
    case 512: return twiddles_of<SchedFor<512, 0>::type>(tw);
    case 1024: return twiddles_of<SchedFor<1024, 0>::type>(tw);
    case 2048: return twiddles_of<SchedFor<2048, 0>::type>(tw);
    case 4096: return twiddles_of<SchedFor<4096, 0>::type>(tw);
    case 8192: return twiddles_of<SchedFor<8192, 0>::type>(tw);
    case 16384: return twiddles_of<SchedFor<16384, 0>::type>(tw);
  }
  return (int)hipErrorInvalidValue;
}

int prepare_launch(int kind, const BatchBeam* beams, const void* const* H, int nbeams,
                   void* host_tab, LaunchDesc* d) {
  if (nbeams < 1 || !d) return (int)hipErrorInvalidValue;
  BlockArgs* ht = (BlockArgs*)host_tab;
  LaunchDesc out;
  out.kind = kind;
  out.nbeams = nbeams;
  out.N = beams[0].p->N;
  out.dtype = beams[0].p->dtype;
  out.variant = kind == kLaunchBatch ? beams[0].p->variant : 0;
  if (!batch_variant_ok(out.N, out.variant)) out.variant = 0;
  // order: longest work per unit first (a unit = the transforms one
  // workgroup runs at once, each N log N per DM trial)
  std::vector<int> order(nbeams);
  std::vector<double> work(nbeams);
  for (int b = 0; b < nbeams; ++b) {
    const BeamPlan& p = *beams[b].p;
    const int ndm = beams[b].dms.ndm;
    const void* h = H ? H[b] : nullptr;
    if (ndm < 1 || ndm > kMaxDmTile || p.dtype != out.dtype) return (int)hipErrorInvalidValue;
    if (kind == kLaunchMixed) {
      if (!mixed_supported(p.N) || (ndm > 1 && h)) return (int)hipErrorInvalidValue;
    } else {
      if (p.N != out.N || !block_supported(p.N)) return (int)hipErrorInvalidValue;
      if (kind == kLaunchTables && (ndm != 1 || !h)) return (int)hipErrorInvalidValue;
      if (kind == kLaunchBatch && h) return (int)hipErrorInvalidValue;
    }
    if (!h) out.multi = 1;
    order[b] = b;
    const int G = kind == kLaunchMixed ? mix_group(p.N) : 1;
    work[b] = (double)G * p.N * std::log2((double)p.N) * (1 + ndm);
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  int64_t total = 0;
  for (int i = 0; i < nbeams; ++i) {
    const int b = order[i];
    const BeamPlan& p = *beams[b].p;
    ht[i] = make_args(p, beams[b].co, beams[b].xt, beams[b].dms, beams[b].P, nullptr,
                      (const float2*)(H ? H[b] : nullptr));
    int err = launch_twiddles(kind, p.N, out.variant, &ht[i].tw);
    if (err) return err;
    ht[i].item0 = total;
    const int64_t items = (int64_t)p.nchan * beams[b].co.nblocks;
    const int G = kind == kLaunchMixed ? mix_group(p.N) : 1;
    total += (items + G - 1) / G;
  }
  if (total > (kind == kLaunchTables ? 0x7fffffffLL : 0xffffffffLL))
    return (int)hipErrorInvalidValue;
  out.total = total;
  *d = out;
  return 0;
}

template <int N, int V, int DT>
static int enqueue_batch_t(const LaunchDesc& d, const void* dev_tab, unsigned int* counter,
                           hipStream_t st) {
  using S = typename SchedFor<N, V>::type;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, st, counter);
  int64_t resident = 0;
  int err = resident_workgroups(reinterpret_cast<const void*>(&batch_kernel<S, DT>), S::T,
                                &resident);
  if (err) return err;
  const int64_t grid = std::min<int64_t>(d.total, resident);
  hipLaunchKernelGGL((batch_kernel<S, DT>), dim3((unsigned)grid), dim3(S::T), 0, st,
                     (const BlockArgs*)dev_tab, d.nbeams, d.total, counter);
  return (int)hipGetLastError();
}

template <int N, int V>
static int enqueue_batch_dt(const LaunchDesc& d, const void* dev_tab, unsigned int* counter,
                            hipStream_t st) {
  return d.dtype == CDD_CI8 ? enqueue_batch_t<N, V, CDD_CI8>(d, dev_tab, counter, st)
                            : enqueue_batch_t<N, V, CDD_CF32>(d, dev_tab, counter, st);
}

template <int N>
static int enqueue_tables_t(const LaunchDesc& d, const void* dev_tab, hipStream_t st) {
  using S = typename SchedFor<N, 0>::type;
  if (d.dtype == CDD_CI8)
    hipLaunchKernelGGL((multi_single_kernel<S, CDD_CI8>), dim3((unsigned)d.total), dim3(S::T), 0,
                       st, (const BlockArgs*)dev_tab, d.nbeams, d.total);
  else
    hipLaunchKernelGGL((multi_single_kernel<S, CDD_CF32>), dim3((unsigned)d.total), dim3(S::T),
                       0, st, (const BlockArgs*)dev_tab, d.nbeams, d.total);
  return (int)hipGetLastError();
}

template <bool MULTI, int DT>
static int enqueue_mixed_t(const LaunchDesc& d, const void* dev_tab, unsigned int* counter,
                           hipStream_t st) {
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, st, counter);
  int64_t resident = 0;
  int err = resident_workgroups(reinterpret_cast<const void*>(&mixed_kernel<MULTI, DT>), kMixT,
                                &resident);
  if (err) return err;
  const int64_t grid = std::min<int64_t>(d.total, resident);
  hipLaunchKernelGGL((mixed_kernel<MULTI, DT>), dim3((unsigned)grid), dim3(kMixT), 0, st,
                     (const BlockArgs*)dev_tab, d.nbeams, d.total, counter);
  return (int)hipGetLastError();
}

static int enqueue_mixed(const LaunchDesc& d, const void* dev_tab, unsigned int* counter,
                         hipStream_t st) {
  if (d.dtype == CDD_CI8)
    return d.multi ? enqueue_mixed_t<true, CDD_CI8>(d, dev_tab, counter, st)
                   : enqueue_mixed_t<false, CDD_CI8>(d, dev_tab, counter, st);
  return d.multi ? enqueue_mixed_t<true, CDD_CF32>(d, dev_tab, counter, st)
                 : enqueue_mixed_t<false, CDD_CF32>(d, dev_tab, counter, st);
}

int enqueue_launch(const LaunchDesc& d, const void* host_tab, void* dev_tab,
                   unsigned int* counter, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(dev_tab, host_tab, batch_table_bytes(d.nbeams),
                                hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return (int)e;
  if (d.total <= 0) return 0;
  if (d.kind == kLaunchMixed) return enqueue_mixed(d, dev_tab, counter, st);
  if (d.kind == kLaunchTables) {
    switch (d.N) {
      case 256: return enqueue_tables_t<256>(d, dev_tab, st);
      case 512: return enqueue_tables_t<512>(d, dev_tab, st);
      case 1024: return enqueue_tables_t<1024>(d, dev_tab, st);
      case 2048: return enqueue_tables_t<2048>(d, dev_tab, st);
      case 4096: return enqueue_tables_t<4096>(d, dev_tab, st);
      case 8192: return enqueue_tables_t<8192>(d, dev_tab, st);
      case 16384: return enqueue_tables_t<16384>(d, dev_tab, st);
    }
    return (int)hipErrorInvalidValue;
  }
  switch (d.N) {
    case 256: return enqueue_batch_dt<256, 0>(d, dev_tab, counter, st);
    case 512: return enqueue_batch_dt<512, 0>(d, dev_tab, counter, st);
    case 1024: return enqueue_batch_dt<1024, 0>(d, dev_tab, counter, st);
    case 2048: return enqueue_batch_dt<2048, 0>(d, dev_tab, counter, st);
    case 4096:
      return d.variant == 3 ? enqueue_batch_dt<4096, 3>(d, dev_tab, counter, st)
                            : enqueue_batch_dt<4096, 0>(d, dev_tab, counter, st);
    case 8192:
      switch (d.variant) {
        case 1: return enqueue_batch_dt<8192, 1>(d, dev_tab, counter, st);
        case 2: return enqueue_batch_dt<8192, 2>(d, dev_tab, counter, st);
        default: return enqueue_batch_dt<8192, 0>(d, dev_tab, counter, st);
      }
    case 16384:
      return d.variant == 2 ? enqueue_batch_dt<16384, 2>(d, dev_tab, counter, st)
                            : enqueue_batch_dt<16384, 0>(d, dev_tab, counter, st);
  }
  return (int)hipErrorInvalidValue;
}

int launch_batch(const BatchBeam* beams, int nbeams, void* host_tab, void* dev_tab,
                 unsigned int* counter, void* stream) {
  if (nbeams < 1) return 0;
  LaunchDesc d;
  int err = prepare_launch(kLaunchBatch, beams, nullptr, nbeams, host_tab, &d);
  return err ? err : enqueue_launch(d, host_tab, dev_tab, counter, stream);
}

const char* hip_error_string(int err) { return hipGetErrorString((hipError_t)err); }

}  // namespace cdd
