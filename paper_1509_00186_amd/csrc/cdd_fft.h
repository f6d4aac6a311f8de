// Device-side FFT building blocks shared by the block and large-transform
// kernels: compile-time constants, in-register radix-2/4 DFTs, Stockham
// passes with LDS exchanges, and the reduced-phase rotation.
#pragma once

#include <hip/hip_runtime.h>

#include <typeinfo>

#include "cdd.h"

#include <cmath>
#include <type_traits>
#include <utility>
#include <vector>

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
// Global-memory pointers
// ---------------------------------------------------------------------------
// A pointer that a kernel reads out of a table in device memory (rather than
// receiving as a kernel argument) is generic to the compiler, which then
// emits flat loads and stores; those also count against the LDS wait
// counter, so every LDS wait of the transform waits for them too.  gptr
// states that the pointer is into global memory.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
// float2 element i through a global-memory pointer (the vector type's own
// assignment cannot take an operand in another address space)
__device__ __forceinline__ float2 gload2(const float2* p, int64_t i) {
  return __builtin_bit_cast(float2, gptr((const unsigned long long*)p)[i]);
}
__device__ __forceinline__ void gstore2(float2* p, int64_t i, float2 v) {
  gptr((unsigned long long*)p)[i] = __builtin_bit_cast(unsigned long long, v);
}

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

// DFT of R points whose inputs first take the twiddles w[r - 1] (r >= 1):
// the products are folded into the first radix-4 stage.  For a pair
// (a, c) with C = c w, a + C is formed with four fused multiply-adds and
// a - C as 2a - (a + C) with two more, instead of a complex product and two
// complex additions (20 instead of 24 operations per radix-4 group).
__device__ __forceinline__ float2 cfma(float2 c, float2 w, float2 a) {  // a + c w
  return make_float2(fmaf(-c.y, w.y, fmaf(c.x, w.x, a.x)), fmaf(c.y, w.x, fmaf(c.x, w.y, a.y)));
}
__device__ __forceinline__ float2 ctwice_minus(float2 a, float2 s) {  // 2a - s
  return make_float2(fmaf(2.0f, a.x, -s.x), fmaf(2.0f, a.y, -s.y));
}
template <int R, int DIR>
struct DftTw {
  // w[r - 1] multiplies input r, r = 1 .. R-1
  static __device__ __forceinline__ void run(float2* v, const float2* w) {
    if constexpr (R == 2) {
      const float2 s = cfma(v[1], w[0], v[0]);
      v[1] = ctwice_minus(v[0], s);
      v[0] = s;
    } else {
      constexpr int Q = R / 4;
      float2 y[R];
      sfor<0, Q>([&](auto N2) {
        constexpr int n2 = decltype(N2)::value;
        float2 a = v[n2];
        if constexpr (n2 > 0) a = cmul(a, w[n2 - 1]);
        const float2 b = cmul(v[Q + n2], w[Q + n2 - 1]);
        const float2 t0 = cfma(v[2 * Q + n2], w[2 * Q + n2 - 1], a);
        const float2 t1 = ctwice_minus(a, t0);
        const float2 t2 = cfma(v[3 * Q + n2], w[3 * Q + n2 - 1], b);
        const float2 t3 = mul_i<DIR>(ctwice_minus(b, t2));
        y[n2 * 4 + 0] = cadd(t0, t2);
        y[n2 * 4 + 1] = twc<R, n2 * 1, DIR>(cadd(t1, t3));
        y[n2 * 4 + 2] = twc<R, n2 * 2, DIR>(csub(t0, t2));
        y[n2 * 4 + 3] = twc<R, n2 * 3, DIR>(csub(t1, t3));
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
  }
};

// ---------------------------------------------------------------------------
// Schedules: threads per workgroup and forward radix order per length
// ---------------------------------------------------------------------------
// LDS layout of a split exchange (one 4-byte word per element): word i of a
// pass's output goes to xpad(i) = i + ((i >> 5) << TS).  The reads of the
// next pass take 32 consecutive elements per half-wave from a 32-aligned run,
// which stays contiguous (every bank once).  The writes of a pass of radix R
// and span Ns put Ns consecutive lanes on consecutive words and 32/Ns such
// groups R*Ns words apart; TS = log2(32/R) spaces the groups exactly Ns banks
// apart when 1 < Ns < 32 and R < 32, and 0 does in the other cases.  (With
// the LDS's 32 banks served per 32 lanes, both sides are then conflict-free
// for the radix-16 and radix-32 passes.)
constexpr int xpad_shift(int R, int Ns) {
  if (Ns == 1 || Ns >= 32 || R >= 32) return 0;
  int t = 0;
  while ((R << t) < 32) ++t;
  return t;
}
template <int TS>
__device__ __forceinline__ constexpr int xpad(int i) { return i + ((i >> 5) << TS); }

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
  // twiddle tables (R x NS entries) for every pass after the first
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
  // Split exchanges pad every 32 words by 2^xpad_shift words (see xpad); the
  // largest pad over the schedule's exchanges sizes the LDS.
  static constexpr int xpad_max() {
    int m = 0;
    for (int p = 0; p + 1 < NP; ++p) {
      const int a = xpad_shift(rad_f(p), ns_f(p)), b = xpad_shift(rad_i(p), ns_i(p));
      m = a > m ? a : m;
      m = b > m ? b : m;
    }
    return m;
  }
  static constexpr int lds_floats() {
    return SPLIT ? N + ((N >> 5) << xpad_max()) : 2 * (N + N / 16);
  }
};

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// ---------------------------------------------------------------------------
// Stockham pass pieces
// ---------------------------------------------------------------------------
// Twiddles of one pass (radix R, span NS) for this thread's butterflies,
// loaded ahead of the exchange that precedes the pass.  The table holds
// W^(r k) at r * NS + k, so the lanes of a wave, whose k are consecutive,
// read consecutive entries.  The loads go through a buffer resource on the
// pass's table (scalar base, constant offset r NS per load), so each needs
// only the thread's offset k, formed once per butterfly group, and no
// 64-bit address arithmetic.
template <class S, int R, int NS, int TWOFF>
struct PassTw {
  static constexpr int BPT = S::N / (R * S::T);
  static constexpr int CNT = NS > 1 ? BPT * (R - 1) : 1;
  float2 w[CNT];
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int t) {
    if constexpr (NS > 1) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(tw + TWOFF), (short)0, R * NS * 8, 0x00020000);
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const int k = (t + S::T * b) & (NS - 1);
#pragma unroll
        for (int r = 1; r < R; ++r)
          w[b * (R - 1) + r - 1] = __builtin_bit_cast(
              float2, __builtin_amdgcn_raw_buffer_load_b64(rs, k * 8, r * NS * 8, 0));
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
    if constexpr (NS > 1)
      DftTw<R, DIR>::run(w, pt.w + b * (R - 1));
    else
      Dft<R, DIR>::run(w);
  }
}

// Padded LDS index of element i: one spare word after every 16.  For the
// strided patterns of the passes, lpad(base + x) = lpad(base) + loff(x) with
// loff a compile-time constant (the low 4 bits of base plus those of x never
// carry), so each access is one LDS instruction with an immediate offset.
__device__ __forceinline__ constexpr int loff(int x) { return 17 * (x >> 4) + (x & 15); }

// Move the outputs of a pass (radix RP, span NSP) to the input layout of the
// next pass (radix RN) through LDS: whole complex values, or real parts then
// imaginary parts (half the LDS, twice the barriers).
template <class S, int RP, int NSP, int RN>
__device__ __forceinline__ void exchange(float2* v, float* lds, int t) {
  constexpr int N = S::N, T = S::T;
  constexpr int BP = N / (RP * T), BN = N / (RN * T);
  if constexpr (!S::SPLIT) {
    int wb[BP], rb[BN];
#pragma unroll
    for (int b = 0; b < BP; ++b) {
      const int j = t + T * b;
      wb[b] = lpad((j / NSP) * NSP * RP + (j % NSP));
    }
#pragma unroll
    for (int b = 0; b < BN; ++b) rb[b] = lpad(t + T * b);
    float2* l2 = (float2*)lds;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BP; ++b)
#pragma unroll
      for (int r = 0; r < RP; ++r) l2[wb[b] + loff(r * NSP)] = v[b * RP + r];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int r = 0; r < RN; ++r) v[b * RN + r] = l2[rb[b] + loff(r * (N / RN))];
  } else {
    // The per-thread base and the compile-time offset occupy disjoint bits,
    // so xpad(base + off) = xpad(base) + xpad(off).
    constexpr int TS = xpad_shift(RP, NSP);
    int xw[BP], xr[BN];
#pragma unroll
    for (int b = 0; b < BP; ++b) {
      const int j = t + T * b;
      xw[b] = xpad<TS>((j / NSP) * NSP * RP + (j % NSP));
    }
#pragma unroll
    for (int b = 0; b < BN; ++b) xr[b] = xpad<TS>(t + T * b);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BP; ++b)
#pragma unroll
      for (int r = 0; r < RP; ++r) lds[xw[b] + xpad<TS>(r * NSP)] = v[b * RP + r].x;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int r = 0; r < RN; ++r) v[b * RN + r].x = lds[xr[b] + xpad<TS>(r * (N / RN))];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BP; ++b)
#pragma unroll
      for (int r = 0; r < RP; ++r) lds[xw[b] + xpad<TS>(r * NSP)] = v[b * RP + r].y;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int r = 0; r < RN; ++r) v[b * RN + r].y = lds[xr[b] + xpad<TS>(r * (N / RN))];
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

// Taper of the chirp function over the channel (Sec. 2.2) at x = the bin's
// offset over the channel width, x in [-1/2, 1/2): Hanning (1 + cos 2 pi x)/2,
// Welch 1 - (2x)^2, else 1.  FAST takes the hardware cosine (argument in
// turns, absolute error about 1.2e-7) instead of cospif.
template <bool FAST>
__device__ __forceinline__ float taper_gain(int kind, float x) {
  if (kind == CDD_TAPER_HANN) {
    const float c = FAST ? __builtin_amdgcn_cosf(x) : cospif(2.0f * x);
    return 0.5f + 0.5f * c;
  }
  if (kind == CDD_TAPER_WELCH) return fmaf(-4.0f * x, x, 1.0f);
  return 1.0f;
}

// Chirp table of one DM: H[c*N + i] = exp(-2 pi i q)/N for bin i of channel c
// (signed bin s = i or i - N, offset f = s*df/N from the channel centre fc),
// q = D*DM*f^2/(fc^2 (fc + f)) turns (Eq. 3), evaluated in FP64 exactly as
// apply_chirp does -- q = B s^2 / (1 + beta s) with B = D*DM*(df/N)^2/fc^3 and
// beta = (df/N)/fc, the division replaced by the series s^2 (B - B beta s +
// B beta^2 s^2) where its truncation is negligible (exact_div = 0) -- so the
// table and the in-kernel chirp give the same numbers.  The channel
// constants are formed once per thread for kpt entries of one channel.  The
// reduction r = q - rint(q) to [-1/2, 1/2] turns is FP64; sin/cos of 2 pi r
// are FP32.  The FP32 phase mode forms q itself in FP32 (precision study).
// The taper (Sec. 2.2) scales the entry with the 1/N of the inverse transform.
struct ChirpTableArgs {
  float2* H;
  double f_lo, df, dconst, dm;
  int32_t lgN, kpt, phase_mode, taper, exact_div;
  uint32_t nwg;  // workgroups of 256 threads covering the table (nchan N / (256 kpt))
};

// Entries of table workgroup wg (< a.nwg), thread tid: kpt entries of one
// channel, 256 apart.
__device__ __forceinline__ void chirp_table_part(const ChirpTableArgs& a, unsigned wg, int tid) {
  const int lgN = a.lgN, kpt = a.kpt, phase_mode = a.phase_mode, taper = a.taper;
  const double f_lo = a.f_lo, df = a.df, dconst = a.dconst, dm = a.dm;
  float2* H = a.H;
  const int N = 1 << lgN;
  const int per_wg = 256 * kpt;
  const int bpc = N / per_wg;                       // workgroups per channel
  const int c = (int)(wg / bpc);
  const int i0 = (int)(wg - (unsigned)c * bpc) * per_wg + tid;
  const double fc = f_lo + ((double)c + 0.5) * df;
  const float inv_n = ldexpf(1.0f, -lgN);
  float2* row = H + ((int64_t)c << lgN);
  if (phase_mode == CDD_PHASE_FP64_REDUCED) {
    const double dfn = df / (double)N;
    const double B = dconst * dm * dfn * dfn / (fc * fc * fc);  // turns
    const double beta = dfn / fc;
    const double Bb = B * beta, Bbb = Bb * beta;
    for (int k = 0; k < kpt; ++k) {
      const int i = i0 + 256 * k;
      const int s = i < N / 2 ? i : i - N;
      const double sd = (double)s;
      const double q = a.exact_div ? (B * (sd * sd)) / fma(beta, sd, 1.0)
                                 : (sd * sd) * fma(sd, fma(sd, Bbb, -Bb), B);
      // r in [-1/2, 1/2] turns: the hardware sine and cosine take turns
      // (absolute error about 1.2e-7)
      const float r = (float)(q - rint(q));
      const float gn = taper_gain<false>(taper, (float)s * inv_n) * inv_n;
      row[i] = make_float2(__builtin_amdgcn_cosf(r) * gn, -__builtin_amdgcn_sinf(r) * gn);
    }
  } else {
    const float fcf = (float)fc;
    const float Af = (float)(dconst * dm) / (fcf * fcf);
    const float dff = (float)df * inv_n;
    for (int k = 0; k < kpt; ++k) {
      const int i = i0 + 256 * k;
      const int s = i < N / 2 ? i : i - N;
      const float f = (float)s * dff;
      const float q = Af * (f * f) / (fcf + f);
      float sn, cs;
      sincospif(2.0f * q, &sn, &cs);
      const float gn = taper_gain<false>(taper, (float)s * inv_n) * inv_n;
      row[i] = make_float2(cs * gn, -sn * gn);
    }
  }
}

// Host: the table arguments of beam p at one DM (cdd_block.hip).
struct BeamPlan;
ChirpTableArgs chirp_table_args(const BeamPlan& p, double dm, void* H, int kpt);

// cos and sin of 2 pi k / 64 for the 64 octant-of-an-octant rotations.
struct RotTable {
  float cs[64][2];  // cos, sin of 2 pi k / 64
};
constexpr RotTable make_rot() {
  RotTable t{};
  for (int i = 0; i < 64; ++i) {
    t.cs[i][0] = (float)ct_cos2pi(i, 64);
    t.cs[i][1] = (float)ct_sin2pi(i, 64);
  }
  return t;
}
static __constant__ RotTable kRot = make_rot();

// exp(-2 pi i r) for r given as r64 = 64 r turns in FP64 (any magnitude
// below 2^31): r64 = k + d with k integer and |d| <= 1/2; exp(-2 pi i k/64)
// from the table, the rest from short Taylor series of cos and sin of
// x = 2 pi d / 64 (|x| <= pi/64, truncation below 2e-11).
__device__ __forceinline__ float2 expi_neg_turns64(double r64) {
  const double k = rint(r64);
  const float x = (float)(r64 - k) * (float)(2.0 * kPi / 64.0);
  const int ki = (int)k & 63;
  const float x2 = x * x;
  const float cs = 1.0f + x2 * (-0.5f + x2 * (1.0f / 24.0f));
  const float sn = x * (1.0f + x2 * (-1.0f / 6.0f + x2 * (1.0f / 120.0f)));
  const float2 CS = *(const float2*)kRot.cs[ki];
  // cos(a+b) - i sin(a+b)
  return make_float2(CS.x * cs - CS.y * sn, -(CS.y * cs + CS.x * sn));
}

// The same for r in turns (reduced internally).
__device__ __forceinline__ float2 expi_neg_turns(double r) {
  const double q = r - rint(r);
  return expi_neg_turns64(q * 64.0);
}

// Host: FP64 twiddle tables of a schedule, R x NS entries per pass after the
// first (entry r * NS + k = W^(r k)); forward tables then inverse
// (conjugate) tables.
template <class S>
std::vector<float2> make_twiddles() {
  std::vector<float2> tw(S::tw_total() > 0 ? S::tw_total() : 1);
  for (int p = 1; p < S::NP; ++p) {
    const int R = S::rad_f(p), ns = S::ns_f(p), off = S::tw_f(p);
    for (int k = 0; k < ns; ++k)
      for (int r = 0; r < R; ++r) {
        const double ang = -2.0 * M_PI * (double)(r * k) / (double)(ns * R);
        tw[off + r * ns + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
  }
  for (int q = 1; q < S::NP; ++q) {
    const int R = S::rad_i(q), ns = S::ns_i(q), off = S::tw_i(q);
    for (int k = 0; k < ns; ++k)
      for (int r = 0; r < R; ++r) {
        const double ang = 2.0 * M_PI * (double)(r * k) / (double)(ns * R);
        tw[off + r * ns + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      }
  }
  return tw;
}

// Device copy of a host-built table, created once per (device, key) and kept
// for the life of the process (cdd_block.hip).
int cached_table(const char* key, std::vector<float2> (*make)(), const float2** out);

template <class S>
int twiddles_of(const float2** out) {
  return cached_table(typeid(S).name(), &make_twiddles<S>, out);
}

}  // namespace cdd
