// Fused per-(channel, block) coherent dedispersion kernel for gfx950.
//
// One workgroup owns one overlap-save block of one channel (N <= 16384):
//   load N samples (int8 or float complex) -> FP32 registers
//   forward FFT: Stockham autosort radix passes, butterflies in registers,
//                exchanges through LDS (real and imaginary halves in turn)
//   chirp:       exp(-2 pi i q_j)/N per bin, q_j from Eq. 3 evaluated in FP64
//                and reduced to [-1/2, 1/2] turns before an FP32 sin/cos
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

#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <utility>
#include <vector>

#include "cdd_internal.h"

namespace cdd {

// ---------------------------------------------------------------------------
// Compile-time helpers
// ---------------------------------------------------------------------------
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double ct_sin(double x) {  // Taylor series, |x| <= pi
  double term = x, sum = x;
  for (int n = 1; n < 32; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 32; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
constexpr int ct_wrap(int m, int R) {  // m mod R mapped to (-R/2, R/2]
  int mm = ((m % R) + R) % R;
  return 2 * mm > R ? mm - R : mm;
}
constexpr double ct_cos2pi(int m, int R) { return ct_cos(2.0 * kPi * ct_wrap(m, R) / R); }
constexpr double ct_sin2pi(int m, int R) { return ct_sin(2.0 * kPi * ct_wrap(m, R) / R); }

// ---------------------------------------------------------------------------
// Complex arithmetic on float2
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by s*i, s = +1 or -1
template <int S>
__device__ __forceinline__ float2 mul_i(float2 a) {
  if constexpr (S > 0) return make_float2(-a.y, a.x);
  else return make_float2(a.y, -a.x);
}
// multiply by W_R^m = exp(DIR * 2 pi i m / R), constants folded
template <int R, int M, int DIR>
__device__ __forceinline__ float2 twc(float2 a) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (4 * m == R) {
    return mul_i<DIR>(a);
  } else if constexpr (2 * m == R) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * m == 3 * R) {
    return mul_i<-DIR>(a);
  } else {
    constexpr float c = (float)ct_cos2pi(m, R);
    constexpr float s = (float)(DIR * ct_sin2pi(m, R));
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// In-register DFT of R points, natural order in and out.
template <int R, int DIR>
struct Dft;
template <int DIR>
struct Dft<1, DIR> {
  static __device__ __forceinline__ void run(float2*) {}
};
template <int DIR>
struct Dft<2, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <int DIR>
struct Dft<4, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = mul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};
// R = 4 Q: x[Q n1 + n2] -> DFT_4 over n1, twiddle W_R^(n2 k1), DFT_Q over n2,
// output X[k1 + 4 k2].
template <int R, int DIR>
struct Dft {
  static __device__ __forceinline__ void run(float2* v) {
    constexpr int Q = R / 4;
    float2 y[R];
    sfor<0, Q>([&](auto N2) {
      constexpr int n2 = decltype(N2)::value;
      float2 t[4] = {v[n2], v[Q + n2], v[2 * Q + n2], v[3 * Q + n2]};
      Dft<4, DIR>::run(t);
      y[n2 * 4 + 0] = t[0];
      y[n2 * 4 + 1] = twc<R, n2 * 1, DIR>(t[1]);
      y[n2 * 4 + 2] = twc<R, n2 * 2, DIR>(t[2]);
      y[n2 * 4 + 3] = twc<R, n2 * 3, DIR>(t[3]);
    });
    sfor<0, 4>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      float2 s[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) s[n2] = y[n2 * 4 + k1];
      Dft<Q, DIR>::run(s);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) v[k1 + 4 * k2] = s[k2];
    });
  }
};

// ---------------------------------------------------------------------------
// Schedules: threads per workgroup and forward radix order per length
// ---------------------------------------------------------------------------
template <int N_, int T_, int A, int B, int C, int D, bool SPLIT_ = true, bool PF_ = false,
          int MINB_ = 1>
struct Sched {
  static constexpr int N = N_, T = T_, E = N_ / T_;
  static constexpr bool SPLIT = SPLIT_;  // exchange real and imaginary halves in turn
  static constexpr bool PF = PF_;        // load a pass's twiddles before its exchange
  static constexpr int MINB = MINB_;     // waves per SIMD the register budget targets
  static constexpr int NP = (A > 1) + (B > 1) + (C > 1) + (D > 1);
  static constexpr int rad_f(int p) { return p == 0 ? A : p == 1 ? B : p == 2 ? C : D; }
  static constexpr int rad_i(int q) { return rad_f(NP - 1 - q); }
  static constexpr int ns_f(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= rad_f(i);
    return s;
  }
  static constexpr int ns_i(int q) {
    int s = 1;
    for (int i = 0; i < q; ++i) s *= rad_i(i);
    return s;
  }
  // twiddle rows of R entries for every pass after the first
  static constexpr int tw_f(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += ns_f(i) * rad_f(i);
    return o;
  }
  static constexpr int tw_i(int q) {
    int o = tw_f(NP);
    for (int i = 1; i < q; ++i) o += ns_i(i) * rad_i(i);
    return o;
  }
  static constexpr int tw_total() { return tw_i(NP); }
  static constexpr int lds_floats() { return (SPLIT ? 1 : 2) * (N + N / 16); }
};

// Schedules per length; variant 0 is the default, others are autotuner
// candidates.
template <int N, int V>
struct SchedFor;
template <> struct SchedFor<256, 0> { using type = Sched<256, 64, 4, 4, 4, 4>; };
template <> struct SchedFor<512, 0> { using type = Sched<512, 64, 8, 8, 8, 1>; };
template <> struct SchedFor<1024, 0> { using type = Sched<1024, 64, 16, 16, 4, 1>; };
template <> struct SchedFor<2048, 0> { using type = Sched<2048, 128, 16, 16, 8, 1>; };
template <> struct SchedFor<4096, 0> { using type = Sched<4096, 256, 16, 16, 16, 1, true, false, 3>; };
template <> struct SchedFor<4096, 1> { using type = Sched<4096, 256, 16, 16, 16, 1, false, false, 2>; };
template <> struct SchedFor<8192, 0> { using type = Sched<8192, 512, 16, 16, 16, 2, true, false, 4>; };
template <> struct SchedFor<8192, 1> { using type = Sched<8192, 512, 16, 16, 16, 2, false, false, 4>; };
template <> struct SchedFor<8192, 2> { using type = Sched<8192, 512, 16, 16, 16, 2, false, false, 3>; };
template <> struct SchedFor<8192, 3> { using type = Sched<8192, 512, 16, 16, 16, 2, true, true, 4>; };
template <> struct SchedFor<8192, 4> { using type = Sched<8192, 256, 16, 16, 32, 1, false, false, 2>; };
template <> struct SchedFor<16384, 0> { using type = Sched<16384, 1024, 16, 16, 16, 4, true, false, 4>; };
template <> struct SchedFor<16384, 1> { using type = Sched<16384, 512, 16, 32, 32, 1, false, false, 2>; };
constexpr int kVariants[] = {1, 1, 1, 1, 2, 5, 2};  // per log2(N) - 8

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// ---------------------------------------------------------------------------
// Stockham pass pieces
// ---------------------------------------------------------------------------
// Twiddles of one pass (radix R, span NS) for this thread's butterflies,
// loaded ahead of the exchange that precedes the pass.
template <class S, int R, int NS, int TWOFF>
struct PassTw {
  static constexpr int BPT = S::N / (R * S::T);
  static constexpr int CNT = NS > 1 ? BPT * (R - 1) : 1;
  float2 w[CNT];
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int t) {
    if constexpr (NS > 1) {
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const int k = (t + S::T * b) & (NS - 1);
        const float2* row = tw + TWOFF + k * R;
#pragma unroll
        for (int r = 1; r < R; ++r) w[b * (R - 1) + r - 1] = row[r];
      }
    }
  }
};

// Butterflies of one pass: twiddle then DFT_R in place.
template <class S, int R, int NS, int DIR, int TWOFF>
__device__ __forceinline__ void butterflies(float2* v, const PassTw<S, R, NS, TWOFF>& pt) {
  constexpr int BPT = S::N / (R * S::T);
  static_assert(BPT * R * S::T == S::N, "schedule does not tile N");
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    float2* w = v + b * R;
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) w[r] = cmul(w[r], pt.w[b * (R - 1) + r - 1]);
    }
    Dft<R, DIR>::run(w);
  }
}

// Move the outputs of a pass (radix RP, span NSP) to the input layout of the
// next pass (radix RN) through LDS: whole complex values, or real parts then
// imaginary parts (half the LDS, twice the barriers).
template <class S, int RP, int NSP, int RN>
__device__ __forceinline__ void exchange(float2* v, float* lds, int t) {
  constexpr int N = S::N, T = S::T;
  constexpr int BP = N / (RP * T), BN = N / (RN * T);
  if constexpr (!S::SPLIT) {
    float2* l2 = (float2*)lds;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BP; ++b) {
      const int j = t + T * b;
      const int base = (j / NSP) * NSP * RP + (j % NSP);
#pragma unroll
      for (int r = 0; r < RP; ++r) l2[lpad(base + r * NSP)] = v[b * RP + r];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      const int j = t + T * b;
#pragma unroll
      for (int r = 0; r < RN; ++r) v[b * RN + r] = l2[lpad(j + r * (N / RN))];
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BP; ++b) {
      const int j = t + T * b;
      const int base = (j / NSP) * NSP * RP + (j % NSP);
#pragma unroll
      for (int r = 0; r < RP; ++r) lds[lpad(base + r * NSP)] = v[b * RP + r].x;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      const int j = t + T * b;
#pragma unroll
      for (int r = 0; r < RN; ++r) v[b * RN + r].x = lds[lpad(j + r * (N / RN))];
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BP; ++b) {
      const int j = t + T * b;
      const int base = (j / NSP) * NSP * RP + (j % NSP);
#pragma unroll
      for (int r = 0; r < RP; ++r) lds[lpad(base + r * NSP)] = v[b * RP + r].y;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      const int j = t + T * b;
#pragma unroll
      for (int r = 0; r < RN; ++r) v[b * RN + r].y = lds[lpad(j + r * (N / RN))];
    }
  }
}

template <class S>
__device__ __forceinline__ void fft_forward(float2* v, float* lds, const float2* __restrict__ tw,
                                            int t) {
  sfor<0, S::NP>([&](auto P) {
    constexpr int p = decltype(P)::value;
    PassTw<S, S::rad_f(p), S::ns_f(p), S::tw_f(p)> pt;
    if constexpr (S::PF) pt.load(tw, t);
    if constexpr (p > 0) exchange<S, S::rad_f(p - 1), S::ns_f(p - 1), S::rad_f(p)>(v, lds, t);
    if constexpr (!S::PF) pt.load(tw, t);
    butterflies<S, S::rad_f(p), S::ns_f(p), -1, S::tw_f(p)>(v, pt);
  });
}

template <class S>
__device__ __forceinline__ void fft_inverse(float2* v, float* lds, const float2* __restrict__ tw,
                                            int t) {
  sfor<0, S::NP>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    PassTw<S, S::rad_i(q), S::ns_i(q), S::tw_i(q)> pt;
    if constexpr (S::PF) pt.load(tw, t);
    if constexpr (q > 0) exchange<S, S::rad_i(q - 1), S::ns_i(q - 1), S::rad_i(q)>(v, lds, t);
    if constexpr (!S::PF) pt.load(tw, t);
    butterflies<S, S::rad_i(q), S::ns_i(q), +1, S::tw_i(q)>(v, pt);
  });
}

// ---------------------------------------------------------------------------
// Kernel
// ---------------------------------------------------------------------------
struct BlockArgs {
  const void* x;        // channel-major input [nchan][nsamp] (int8x2 or float2)
  float* P;             // [ndm][nchan][t_int]
  float2* vout;         // [nchan][nsamp] or null (single DM only)
  const float2* tw;     // twiddle tables
  int64_t nsamp, t_int, nblocks;
  int32_t nchan, M, nfront, n_int, phase_mode, exact_div;
  double f_lo, df, dconst;
  DmTile dms;
};

// cos and sin of 2 pi k / 64 for the 64 octant-of-an-octant rotations.
struct RotTable {
  float c[64], s[64];
};
constexpr RotTable make_rot() {
  RotTable t{};
  for (int i = 0; i < 64; ++i) {
    t.c[i] = (float)ct_cos2pi(i, 64);
    t.s[i] = (float)ct_sin2pi(i, 64);
  }
  return t;
}
__constant__ RotTable kRot = make_rot();

// exp(-2 pi i r) for r in [-1/2, 1/2] turns given in FP64: r = (k + d)/64
// with k integer and |d| <= 1/2; exp(-2 pi i k/64) from the table, the rest
// from short Taylor series of cos and sin of x = 2 pi d / 64 (|x| <= pi/64,
// truncation below 2e-11).
__device__ __forceinline__ float2 expi_neg_turns(double r) {
  const double r64 = r * 64.0;
  const double k = rint(r64);
  const float x = (float)(r64 - k) * (float)(2.0 * kPi / 64.0);
  const int ki = (int)k & 63;
  const float x2 = x * x;
  const float cs = 1.0f + x2 * (-0.5f + x2 * (1.0f / 24.0f));
  const float sn = x * (1.0f + x2 * (-1.0f / 6.0f + x2 * (1.0f / 120.0f)));
  const float C = kRot.c[ki], Sn = kRot.s[ki];
  // cos(a+b) - i sin(a+b)
  return make_float2(C * cs - Sn * sn, -(Sn * cs + C * sn));
}

// Bin i of the forward transform holds the spectrum at offset f = s*df/N from
// the channel centre fc, s = i (i < N/2) or i - N.  Multiply it by
// exp(-2 pi i q)/N with q = D*DM*f^2/(fc^2 (fc + f)) turns (Eq. 3), evaluated
// in FP64 as q = B s^2 / (1 + x), B = D*DM*(df/N)^2/fc^3, x = s*(df/N)/fc.
// When the channel is narrow enough that q*x^3 stays below 1e-9 turns, 1/(1+x)
// is replaced by 1 - x + x^2 (no division); otherwise the division is exact.
// The phase is reduced to [-1/2, 1/2] turns before the FP32 rotation.
template <class S>
__device__ __forceinline__ void apply_chirp(float2* v, double dm, double fc, const BlockArgs& a,
                                            int t) {
  constexpr int N = S::N, R = S::rad_f(S::NP - 1), BPT = N / (R * S::T);
  const float inv_n = 1.0f / (float)N;
  if (a.phase_mode == CDD_PHASE_FP64_REDUCED) {
    const double dfn = a.df / (double)N;
    const double B = a.dconst * dm * dfn * dfn / (fc * fc * fc);
    const double beta = dfn / fc;
    if (a.exact_div == 0) {
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = t + S::T * b + r * (N / R);
          const double sd = (double)(i < N / 2 ? i : i - N);
          const double x = beta * sd;
          const double q = (B * (sd * sd)) * fma(x, x, 1.0 - x);
          const float2 h = expi_neg_turns(q - rint(q));
          v[b * R + r] = cmul(v[b * R + r], make_float2(h.x * inv_n, h.y * inv_n));
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = t + S::T * b + r * (N / R);
          const double sd = (double)(i < N / 2 ? i : i - N);
          const double q = (B * (sd * sd)) / fma(beta, sd, 1.0);
          const float2 h = expi_neg_turns(q - rint(q));
          v[b * R + r] = cmul(v[b * R + r], make_float2(h.x * inv_n, h.y * inv_n));
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
        v[b * R + r] = cmul(v[b * R + r], make_float2(cs * inv_n, -sn * inv_n));
      }
    }
  }
}

template <class S, int DT>
__device__ __forceinline__ void load_block(float2* v, const BlockArgs& a, int c, int64_t k, int t) {
  constexpr int N = S::N, R = S::rad_f(0), BPT = N / (R * S::T);
  const int64_t t0 = k * a.M - a.nfront;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = t + S::T * b + r * (N / R);
      const int64_t tt = t0 + n;
      float2 z = make_float2(0.f, 0.f);
      if (tt >= 0 && tt < a.nsamp) {
        if constexpr (DT == CDD_CI8) {
          const short w = ((const short*)a.x)[(int64_t)c * a.nsamp + tt];
          z = make_float2((float)(signed char)(w & 0xff), (float)(signed char)(w >> 8));
        } else {
          z = ((const float2*)a.x)[(int64_t)c * a.nsamp + tt];
        }
      }
      v[b * R + r] = z;
    }
  }
}

template <class S, bool VOUT>
__device__ __forceinline__ void epilogue(const float2* v, float* lds, const BlockArgs& a, int c,
                                         int64_t k, int dmi, int t) {
  constexpr int N = S::N, R = S::rad_i(S::NP - 1), BPT = N / (R * S::T);
  if constexpr (VOUT) {
    if (a.vout) {
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int n = t + S::T * b + r * (N / R);
          const int m = n - a.nfront;
          const int64_t o = k * a.M + m;
          if (m >= 0 && m < a.M && o < a.nsamp) a.vout[(int64_t)c * a.nsamp + o] = v[b * R + r];
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = t + S::T * b + r * (N / R);
      const float2 z = v[b * R + r];
      lds[lpad(n)] = z.x * z.x + z.y * z.y;
    }
  }
  __syncthreads();
  const int nu = a.M / a.n_int;
  const int64_t u0 = k * (a.M / a.n_int);
  float* P = a.P + ((int64_t)dmi * a.nchan + c) * a.t_int;
  for (int ul = t; ul < nu; ul += S::T) {
    const int64_t u = u0 + ul;
    if (u >= a.t_int) break;
    const int base = a.nfront + ul * a.n_int;
    float s = 0.f;
    for (int r = 0; r < a.n_int; ++r) s += lds[lpad(base + r)];
    P[u] = s;
  }
}

template <class S, int DT, bool MULTI>
__global__ __launch_bounds__(S::T, MULTI ? (S::MINB + 1) / 2 : S::MINB) void block_kernel(const BlockArgs a) {
  __shared__ float lds[S::lds_floats()];
  const int t = threadIdx.x;
  const int64_t item = blockIdx.x;
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  const double fc = a.f_lo + ((double)c + 0.5) * a.df;
  float2 v[S::E];
  load_block<S, DT>(v, a, c, k, t);
  fft_forward<S>(v, lds, a.tw, t);
  if constexpr (!MULTI) {
    apply_chirp<S>(v, a.dms.dm[0], fc, a, t);
    fft_inverse<S>(v, lds, a.tw, t);
    epilogue<S, true>(v, lds, a, c, k, 0, t);
  } else {
    float2 X[S::E];
#pragma unroll
    for (int e = 0; e < S::E; ++e) X[e] = v[e];
    for (int i = 0; i < a.dms.ndm; ++i) {
#pragma unroll
      for (int e = 0; e < S::E; ++e) v[e] = X[e];
      apply_chirp<S>(v, a.dms.dm[i], fc, a, t);
      fft_inverse<S>(v, lds, a.tw, t);
      epilogue<S, false>(v, lds, a, c, k, i, t);
    }
  }
}

// ---------------------------------------------------------------------------
// Host side: FP64 twiddle tables (cached per device, length and schedule)
// and launch
// ---------------------------------------------------------------------------
template <class S>
static std::vector<float2> make_twiddles() {
  std::vector<float2> tw(S::tw_total() > 0 ? S::tw_total() : 1);
  for (int p = 1; p < S::NP; ++p) {
    const int R = S::rad_f(p), ns = S::ns_f(p), off = S::tw_f(p);
    for (int k = 0; k < ns; ++k)
      for (int r = 0; r < R; ++r) {
        const double ang = -2.0 * M_PI * (double)(r * k) / (double)(ns * R);
        tw[off + k * R + r] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
  }
  for (int q = 1; q < S::NP; ++q) {
    const int R = S::rad_i(q), ns = S::ns_i(q), off = S::tw_i(q);
    for (int k = 0; k < ns; ++k)
      for (int r = 0; r < R; ++r) {
        const double ang = 2.0 * M_PI * (double)(r * k) / (double)(ns * R);
        tw[off + k * R + r] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
  }
  return tw;
}

static std::mutex g_tw_mu;
static std::map<std::tuple<int, int, int>, float2*> g_tw;  // (device, N, variant)

template <class S, int V>
static int twiddles_for(const float2** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  auto key = std::make_tuple(dev, S::N, V);
  auto it = g_tw.find(key);
  if (it != g_tw.end()) {
    *out = it->second;
    return 0;
  }
  std::vector<float2> h = make_twiddles<S>();
  float2* d = nullptr;
  e = hipMalloc(&d, h.size() * sizeof(float2));
  if (e != hipSuccess) return (int)e;
  e = hipMemcpy(d, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return (int)e;
  }
  g_tw[key] = d;
  *out = d;
  return 0;
}

// Whether 1/(1+x) needs the exact division: the series 1 - x + x^2 is used
// when its truncation, q*x^3/(1-x), stays below 1e-9 turns over the beam's
// channels and DMs (x = f/fc, |f| <= df/2).
static int needs_exact_division(const BeamPlan& p, const DmTile& dms) {
  const double fmin = p.f_lo + 0.5 * p.df;
  const double xm = 0.5 * p.df / fmin;
  double dmax = 0;
  for (int i = 0; i < dms.ndm; ++i) dmax = std::fmax(dmax, std::fabs(dms.dm[i]));
  const double qmax = p.dconst * dmax * 0.25 * p.df * p.df / (fmin * fmin * (fmin - 0.5 * p.df));
  return qmax * xm * xm * xm / (1.0 - xm) > 1e-9 ? 1 : 0;
}

template <int N, int V>
static int launch_block_t(const BeamPlan& p, const void* xt, const DmTile& dms, float* P,
                          void* vout, void* stream) {
  using S = typename SchedFor<N, V>::type;
  BlockArgs a{};
  int err = twiddles_for<S, V>(&a.tw);
  if (err) return err;
  a.x = xt;
  a.P = P;
  a.vout = (float2*)vout;
  a.nsamp = p.nsamp;
  a.t_int = p.t_int;
  a.nblocks = p.nblocks;
  a.nchan = p.nchan;
  a.M = p.M;
  a.nfront = p.nfront;
  a.n_int = p.n_int;
  a.phase_mode = p.phase_mode;
  a.exact_div = needs_exact_division(p, dms);
  a.f_lo = p.f_lo;
  a.df = p.df;
  a.dconst = p.dconst;
  a.dms = dms;
  const int64_t items = (int64_t)p.nchan * p.nblocks;
  if (items <= 0 || items > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  dim3 grid((unsigned)items), block(S::T);
  hipStream_t st = (hipStream_t)stream;
  const bool multi = dms.ndm > 1;
  if (p.dtype == CDD_CI8) {
    if (multi) hipLaunchKernelGGL((block_kernel<S, CDD_CI8, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((block_kernel<S, CDD_CI8, false>), grid, block, 0, st, a);
  } else {
    if (multi) hipLaunchKernelGGL((block_kernel<S, CDD_CF32, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((block_kernel<S, CDD_CF32, false>), grid, block, 0, st, a);
  }
  return (int)hipGetLastError();
}

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
                 void* stream) {
  if (dms.ndm < 1 || dms.ndm > kMaxDmTile) return (int)hipErrorInvalidValue;
  const int v = p.variant;
  switch (p.N) {
    case 256: return launch_block_t<256, 0>(p, xt, dms, P, vout, stream);
    case 512: return launch_block_t<512, 0>(p, xt, dms, P, vout, stream);
    case 1024: return launch_block_t<1024, 0>(p, xt, dms, P, vout, stream);
    case 2048: return launch_block_t<2048, 0>(p, xt, dms, P, vout, stream);
    case 4096:
      return v == 1 ? launch_block_t<4096, 1>(p, xt, dms, P, vout, stream)
                    : launch_block_t<4096, 0>(p, xt, dms, P, vout, stream);
    case 8192:
      switch (v) {
        case 1: return launch_block_t<8192, 1>(p, xt, dms, P, vout, stream);
        case 2: return launch_block_t<8192, 2>(p, xt, dms, P, vout, stream);
        case 3: return launch_block_t<8192, 3>(p, xt, dms, P, vout, stream);
        case 4: return launch_block_t<8192, 4>(p, xt, dms, P, vout, stream);
        default: return launch_block_t<8192, 0>(p, xt, dms, P, vout, stream);
      }
    case 16384:
      return v == 1 ? launch_block_t<16384, 1>(p, xt, dms, P, vout, stream)
                    : launch_block_t<16384, 0>(p, xt, dms, P, vout, stream);
  }
  return (int)hipErrorInvalidValue;
}

const char* hip_error_string(int err) { return hipGetErrorString((hipError_t)err); }

}  // namespace cdd
