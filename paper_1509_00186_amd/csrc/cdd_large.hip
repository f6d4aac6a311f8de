// Long overlap-save transforms (N = 2^15 .. 2^26 complex points) as a four-step FFT.
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
// Above 2^22 points (N2 > 2048) each column transform is itself split in
// two, N2 = A B with n2 = a + A b and k2 = kb + B ka, so the column passes
// become two passes each (see "Three-level transforms" below); the spectrum
// bin k2 of a block is then stored in row ka + A kb.
// Every sub-transform reuses the register/LDS Stockham passes of the block
// kernel; a workgroup runs G sub-transforms side by side, lanes ordered so
// that global accesses along n1 are contiguous.  The twiddles W_N^(n1 k2)
// are computed (exact phase in turns, hardware sine and cosine), not read
// from a table.  The same passes carry the full-band mode (further below):
// a real series packed two samples per complex value, the row pass holding
// the mirror rows of each bin pair.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

#include "cdd_fft.h"
#include "cdd_fullband.h"
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
  int64_t nsamp, nblocks, item0;
  int32_t nchan, N1, N2, M, nfront, phase_mode, exact_div, taper;
  double f_lo, df, dconst, dm;
  // full-band mode: band width, chirp function per real-spectrum bin (N + 1 entries)
  double bw;
  const float2* hb;
  int32_t lgn;  // log2(N1 N2)
  // fused detection + integration in cols_inv (n_int divides the G columns
  // of a workgroup): P and the t_int outputs per channel, and the partial
  // sums of the groups that straddle two column runs (in p: per item, two
  // per run of G samples)
  float* P;
  int64_t t_int;
  int32_t n_int;
  int32_t fuse;
  // three-level transforms: N2 = A B (A = 1 for the two-level form), the
  // twiddles of the length-A sub-transform, and log2 of N2 and B
  int32_t A, lg2, lgB;
  const float2* twm;
  // one-channel calls: coverage set to 1 by the chirp-table kernel (or null)
  int32_t* cov_fill;
  int64_t cov_n;
};

// Row of the intermediate array that holds spectrum bin k2 (< N2): k2 itself
// in the two-level form; ka + A kb for k2 = kb + B ka in the three-level one.
__device__ __forceinline__ int64_t spec_row(const LargeArgs& a, int k2) {
  if (a.A == 1) return k2;
  return (int64_t)(k2 >> a.lgB) + (int64_t)a.A * (k2 & ((1 << a.lgB) - 1));
}

// exp(-2 pi i m / M) for M = 2^lg: v = ((m + M/2) mod M) - M/2 is m reduced
// to [-M/2, M/2), and t = v / M the phase in turns in [-1/2, 1/2).  The
// conversion of v to FP32 is the only rounding (none up to M = 2^25; beyond,
// t is the correctly rounded FP32 value, within 2^-26 turns), and the
// hardware sine and cosine take turns (absolute error about 1.2e-7).
// Computing the four-step twiddles this way keeps the passes free of table
// gathers, whose scattered indices (n1 k2) touch a cache line per lane.
__device__ __forceinline__ float2 expi_pow2(int64_t m, int lg) {
  const int64_t M = (int64_t)1 << lg;
  const int v = (int)(((m + (M >> 1)) & (M - 1)) - (M >> 1));  // |v| <= 2^26 for lg <= 27
  const float t = ldexpf((float)v, -lg);
  return make_float2(__builtin_amdgcn_cosf(t), -__builtin_amdgcn_sinf(t));
}

__device__ __forceinline__ float2 tw4_fwd(const LargeArgs& a, int64_t m) {
  return expi_pow2(m, a.lgn);
}

// ---------------------------------------------------------------------------
// cols_fwd
// ---------------------------------------------------------------------------
// Two-level form (THREE = false): the length-N2 column transforms.  Three-
// level form: the length-B transforms over b of x[n1 + N1 (a + A b)] for
// each a, times W_N2^(a kb), stored in row a + A kb (the first half of the
// column transform; cols_mid_kernel does the second).
template <class SC, int G, int DT, bool THREE>
__global__ __launch_bounds__(SC::T * G) void cols_fwd_kernel(const LargeArgs a) {
  __shared__ float lds[G * (SC::lds_floats() + 1)];
  constexpr int L = SC::N, R0 = SC::rad_f(0), B0 = L / (R0 * SC::T);
  constexpr int RL = SC::rad_f(SC::NP - 1), BL = L / (RL * SC::T);
  const int t = threadIdx.x, g = t % G, tl = t / G;
  const int ngrp = a.N1 / G;
  const int nsub = THREE ? a.A : 1;
  const int64_t item = a.item0 + blockIdx.x / ((unsigned)ngrp * nsub);
  const int rem = (int)(blockIdx.x % ((unsigned)ngrp * nsub));
  const int sa = THREE ? rem / ngrp : 0;  // a of this column run
  const int n1 = (rem % ngrp) * G + g;
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  const int64_t base = k * a.M - a.nfront + n1;
  float2 v[SC::E];
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int l = tl + SC::T * b + r * (L / R0);
      const int64_t n2 = THREE ? sa + (int64_t)a.A * l : l;
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
      const int kk = tl + SC::T * b + r * (L / RL);
      if (THREE)
        S[(sa + (int64_t)a.A * kk) * a.N1 + n1] =
            cmul(v[b * RL + r], expi_pow2((int64_t)sa * kk, a.lg2));
      else
        S[(int64_t)kk * a.N1 + n1] = cmul(v[b * RL + r], tw4_fwd(a, (int64_t)n1 * kk));
    }
}

// ---------------------------------------------------------------------------
// Three-level transforms: the second half of each column transform.  With
// n2 = a + A b and k2 = kb + B ka, the length-N2 column DFT is
//   C[kb + B ka] = sum_a W_A^(a ka) W_N2^(a kb) sum_b x[a + A b] W_B^(b kb);
// cols_fwd_kernel forms the inner sums (times W_N2^(a kb)) in rows a + A kb,
// and this kernel, for each kb, the outer sums over a, times the four-step
// twiddle W_N^(n1 k2), back into the same rows (bin k2 in row ka + A kb).
// The inverse (INV) takes the same steps backwards: the inverse DFT over ka
// of rows ka + A kb, times W_N2^(-a kb), into rows a + A kb, before
// cols_inv_kernel's inverse DFTs over kb.
// ---------------------------------------------------------------------------
template <class SC, int G, bool INV>
__global__ __launch_bounds__(SC::T * G) void cols_mid_kernel(const LargeArgs a) {
  __shared__ float lds[G * (SC::lds_floats() + 1)];
  constexpr int L = SC::N;  // A
  constexpr int RIN = INV ? SC::rad_i(0) : SC::rad_f(0), BIN = L / (RIN * SC::T);
  constexpr int ROUT = INV ? SC::rad_f(0) : SC::rad_f(SC::NP - 1), BOUT = L / (ROUT * SC::T);
  const int t = threadIdx.x, g = t % G, tl = t / G;
  const int ngrp = a.N1 / G;
  const int nsub = 1 << a.lgB;  // B
  const int64_t item = a.item0 + blockIdx.x / ((unsigned)ngrp * nsub);
  const int rem = (int)(blockIdx.x % ((unsigned)ngrp * nsub));
  const int kb = rem / ngrp;
  const int n1 = (rem % ngrp) * G + g;
  // rows l + A kb (l < A) of this item, column n1
  float2* S = a.S + (item - a.item0) * ((int64_t)a.N1 * a.N2) +
              (int64_t)L * kb * a.N1 + n1;
  float2 v[SC::E];
#pragma unroll
  for (int b = 0; b < BIN; ++b)
#pragma unroll
    for (int r = 0; r < RIN; ++r)
      v[b * RIN + r] = S[(int64_t)(tl + SC::T * b + r * (L / RIN)) * a.N1];
  float* my = lds + g * (SC::lds_floats() + 1);
  if (INV)
    fft_inverse<SC>(v, my, a.twm, tl);
  else
    fft_forward<SC>(v, my, a.twm, tl);
#pragma unroll
  for (int b = 0; b < BOUT; ++b)
#pragma unroll
    for (int r = 0; r < ROUT; ++r) {
      const int kk = tl + SC::T * b + r * (L / ROUT);
      float2 w;
      if (INV) {
        w = expi_pow2((int64_t)kk * kb, a.lg2);
        w.y = -w.y;
      } else {
        w = tw4_fwd(a, (int64_t)n1 * (kb + ((int64_t)kk << a.lgB)));
      }
      S[(int64_t)kk * a.N1] = cmul(v[b * ROUT + r], w);
    }
}

// ---------------------------------------------------------------------------
// Chirp function of channel c at bin i of the N-point transform (bin i < N/2
// lies +i df/N from the channel centre, else (i - N) df/N): exp(-2 pi i q) of
// Eq. 3 about the centre, times the taper and 1/N.  FP64 phase reduced before
// the FP32 rotation, or all FP32 (precision study).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 chan_chirp(const LargeArgs& a, double fc, int64_t i,
                                             int64_t N) {
  const float inv_n = 1.0f / (float)N;
  const int64_t si = i < N / 2 ? i : i - N;
  const float g = inv_n * taper_gain<false>(a.taper, (float)si * inv_n);
  if (a.phase_mode == CDD_PHASE_FP64_REDUCED) {
    const double dfn = a.df / (double)N;
    const double B = a.dconst * a.dm * dfn * dfn / (fc * fc * fc);
    const double beta = dfn / fc;
    const double sd = (double)si;
    const double x = beta * sd;
    const double q = a.exact_div ? (B * (sd * sd)) / fma(beta, sd, 1.0)
                                 : (B * (sd * sd)) * fma(x, x, 1.0 - x);
    const float2 h = expi_neg_turns(q - rint(q));
    return make_float2(h.x * g, h.y * g);
  }
  const float fcf = (float)fc;
  const float Af = (float)(a.dconst * a.dm) / (fcf * fcf);
  const float f = (float)si * ((float)a.df / (float)N);
  const float q = Af * (f * f) / (fcf + f);
  float sn, cs;
  sincospif(2.0f * q, &sn, &cs);
  return make_float2(cs * g, -sn * g);
}

// The chirp functions of one call, per channel in the order the row pass
// reads them: entry c N + k2 N1 + k1 holds bin i = k2 + N2 k1 of channel c.
// With a.cov_fill the same launch also sets a.cov_n coverage entries to 1.
__global__ __launch_bounds__(256) void chan_chirp_table_kernel(LargeArgs a, int64_t N,
                                                               float2* __restrict__ hb) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx < a.cov_n) a.cov_fill[idx] = 1;
  if (idx >= N * a.nchan) return;
  const int c = (int)(idx / N);
  const int64_t e = idx - (int64_t)c * N;
  const int64_t i = e / a.N1 + (int64_t)a.N2 * (e % a.N1);
  const double fc = a.f_lo + ((double)c + 0.5) * a.df;
  hb[idx] = chan_chirp(a, fc, i, N);
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
  float2* row = a.S + (item - a.item0) * N + spec_row(a, k2) * a.N1;
  float2 v[SR::E];
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) v[b * R0 + r] = row[tl + SR::T * b + r * (L / R0)];
  float* my = lds + g * (SR::lds_floats() + 1);
  fft_forward<SR>(v, my, a.twr, tl);
  // chirp on bins i = k2 + N2 k1, from the call's table
  const float2* h = a.hb + (int64_t)c * N + (int64_t)k2 * a.N1;
#pragma unroll
  for (int b = 0; b < BL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r)
      v[b * RL + r] = cmul(v[b * RL + r], h[tl + SR::T * b + r * (L / RL)]);
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
// Three-level form (THREE): for each a, the inverse DFTs over kb of rows
// a + A kb give the samples n2 = a + A b.
template <class SC, int G, bool THREE>
__global__ __launch_bounds__(SC::T * G) void cols_inv_kernel(const LargeArgs a) {
  __shared__ float lds[G * (SC::lds_floats() + 1)];
  constexpr int L = SC::N, RI = SC::rad_i(0), BI = L / (RI * SC::T);
  constexpr int R0 = SC::rad_f(0), B0 = L / (R0 * SC::T);
  const int t = threadIdx.x, g = t % G, tl = t / G;
  const int ngrp = a.N1 / G;
  const int nsub = THREE ? a.A : 1;
  const int64_t item = a.item0 + blockIdx.x / ((unsigned)ngrp * nsub);
  const int rem = (int)(blockIdx.x % ((unsigned)ngrp * nsub));
  const int sa = THREE ? rem / ngrp : 0;  // a of this column run
  const int sA = THREE ? a.A : 1;         // n2 = sa + sA * (local index)
  const int n1 = (rem % ngrp) * G + g;
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  const float2* S = a.S + (item - a.item0) * ((int64_t)a.N1 * a.N2);
  float2 v[SC::E];
#pragma unroll
  for (int b = 0; b < BI; ++b)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int kk = tl + SC::T * b + r * (L / RI);
      v[b * RI + r] = S[(sa + (int64_t)sA * kk) * a.N1 + n1];
    }
  fft_inverse<SC>(v, lds + g * (SC::lds_floats() + 1), a.twc, tl);
  if (!a.fuse) {
#pragma unroll
    for (int b = 0; b < B0; ++b)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int64_t n2 = sa + (int64_t)sA * (tl + SC::T * b + r * (L / R0));
        const int64_t n = n1 + (int64_t)a.N1 * n2;
        const int64_t m = n - a.nfront;
        const int64_t o = k * a.M + m;
        if (m >= 0 && m < a.M && o < a.nsamp) {
          const float2 z = v[b * R0 + r];
          a.p[(int64_t)c * a.nsamp + o] = z.x * z.x + z.y * z.y;
          if (a.vout) a.vout[(int64_t)c * a.nsamp + o] = z;
        }
      }
    return;
  }
  // Fused detection and integration.  The workgroup holds, for each of its
  // n2, the run of G consecutive samples n = n1b + N1 n2 + g (g < G).  |z|^2
  // of the kept samples goes to LDS as [local n2][g]; groups of n_int start where
  // n = nfront (mod n_int).  Groups inside a run are summed here and stored;
  // a group split across the end of one run and the start of the next is
  // left as two partial sums for integrate_fixup_kernel.
  __syncthreads();  // the transform's last LDS reads are done
  float* q = lds;
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int nl = tl + SC::T * b + r * (L / R0);
      const int64_t n = n1 + (int64_t)a.N1 * (sa + (int64_t)sA * nl);
      const int64_t m = n - a.nfront;
      const int64_t o = k * a.M + m;
      const float2 z = v[b * R0 + r];
      const bool kept = m >= 0 && m < a.M && o < a.nsamp;
      if (kept && a.vout) a.vout[(int64_t)c * a.nsamp + o] = z;
      q[nl * G + g] = kept ? z.x * z.x + z.y * z.y : 0.f;
    }
  __syncthreads();
  const int ni = a.n_int;
  const int phi = (int)(a.nfront % ni);
  const int per_run = G / ni;  // group starts per run
  const int n1b = n1 - g;
  const int64_t item_local = item - a.item0;
  float* part = a.p + item_local * ((int64_t)a.N1 * a.N2 / G) * 2;
  float* Pc = a.P + (int64_t)c * a.t_int;
  for (int j = threadIdx.x; j < L * (per_run + 1); j += SC::T * G) {
    const int nl = j / (per_run + 1), slot = j - nl * (per_run + 1);
    const float* run = q + nl * G;
    const int64_t n0 = n1b + (int64_t)a.N1 * (sa + (int64_t)sA * nl);  // run's first sample
    const int64_t ridx = n0 / G;                   // run index in the block
    if (slot == per_run) {
      // partial sums: the head [0, phi) and the tail [G - ni + phi, G)
      if (phi == 0) continue;
      float h = 0.f, t = 0.f;
      for (int i = 0; i < phi; ++i) h += run[i];
      for (int i = G - ni + phi; i < G; ++i) t += run[i];
      part[2 * ridx] = h;
      part[2 * ridx + 1] = t;
      continue;
    }
    const int s0 = phi + slot * ni;  // group start within the run
    if (s0 + ni > G) continue;       // the split group (partials above)
    const int64_t m = n0 + s0 - a.nfront;
    if (m < 0 || m >= a.M) continue;
    const int64_t u = (k * a.M + m) / ni;
    if (u >= a.t_int) continue;
    float acc = 0.f;
    for (int i = 0; i < ni; ++i) acc += run[s0 + i];
    Pc[u] = acc;
  }
}

// The integration groups split across two runs of G samples: the tail of
// run j plus the head of run j + 1 (partial sums from cols_inv_kernel).
__global__ __launch_bounds__(256) void integrate_fixup_kernel(const LargeArgs a, int32_t G,
                                                              int64_t items) {
  const int64_t runs = (int64_t)a.N1 * a.N2 / G;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= items * (runs - 1)) return;
  const int64_t item_local = idx / (runs - 1);
  const int64_t j = idx - item_local * (runs - 1);
  const int64_t item = a.item0 + item_local;
  const int c = (int)(item / a.nblocks);
  const int64_t k = item - (int64_t)c * a.nblocks;
  const int ni = a.n_int;
  const int phi = (int)(a.nfront % ni);
  const int64_t start = j * G + G - ni + phi;  // first sample of the split group
  const int64_t m = start - a.nfront;
  if (m < 0 || m >= a.M) return;
  const int64_t u = (k * a.M + m) / ni;
  if (u >= a.t_int) return;
  const float* part = a.p + item_local * runs * 2;
  a.P[(int64_t)c * a.t_int + u] = part[2 * j + 1] + part[2 * (j + 1)];
}

// P[c][u] = sum_{r < n_int} p[c][u n_int + r] in ascending r, grid (u
// blocks, channels).  V consecutive samples per load (V divides n_int and
// the channel stride, so every vector load is aligned).
template <int V>
__global__ __launch_bounds__(256) void integrate_kernel(const float* __restrict__ p,
                                                        float* __restrict__ P, int64_t nsamp,
                                                        int64_t t_int, int32_t n_int) {
  using VT = typename std::conditional<V == 4, float4, typename std::conditional<
                                                         V == 2, float2, float>::type>::type;
  const int c = blockIdx.y;
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= t_int) return;
  const VT* pc = (const VT*)(p + (int64_t)c * nsamp + u * n_int);
  float s = 0.f;
  for (int r = 0; r < n_int / V; ++r) {
    const VT x = pc[r];
    if constexpr (V == 4) {
      s += x.x;
      s += x.y;
      s += x.z;
      s += x.w;
    } else if constexpr (V == 2) {
      s += x.x;
      s += x.y;
    } else {
      s += x;
    }
  }
  P[(int64_t)c * t_int + u] = s;
}

static int launch_integrate(const float* p, float* P, int64_t nsamp, int64_t t_int,
                            int32_t n_int, int32_t nchan, hipStream_t st) {
  const int64_t nb = (t_int + 255) / 256;
  if (nb > 0x7fffffffLL || nchan > 65535) return (int)hipErrorInvalidValue;
  if (nb == 0) return 0;
  const dim3 grid((unsigned)nb, (unsigned)nchan);
  if (n_int % 4 == 0 && (nchan == 1 || nsamp % 4 == 0))
    hipLaunchKernelGGL(integrate_kernel<4>, grid, dim3(256), 0, st, p, P, nsamp, t_int, n_int);
  else if (n_int % 2 == 0 && (nchan == 1 || nsamp % 2 == 0))
    hipLaunchKernelGGL(integrate_kernel<2>, grid, dim3(256), 0, st, p, P, nsamp, t_int, n_int);
  else
    hipLaunchKernelGGL(integrate_kernel<1>, grid, dim3(256), 0, st, p, P, nsamp, t_int, n_int);
  return (int)hipGetLastError();
}

// The split integration groups of one chunk of items (fused path); none when
// the groups start on run boundaries.
static int launch_fixup(const LargeArgs& a, int G, int64_t items, hipStream_t st) {
  if (a.nfront % a.n_int == 0) return 0;
  const int64_t runs = (int64_t)a.N1 * a.N2 / G;
  const int64_t n = items * (runs - 1);
  const int64_t nb = (n + 255) / 256;
  if (nb > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  if (nb == 0) return 0;
  hipLaunchKernelGGL(integrate_fixup_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, G, items);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Full-band mode: one real series over the whole band (Sec. 2.1, 2.3, 3.1)
// ---------------------------------------------------------------------------
// A real block of 2N samples is transformed as N complex points z[n] =
// x[2n] + i x[2n+1].  With Z = DFT_N(z), the spectra of the even and odd
// samples are E_i = (Z_i + conj Z_(N-i)) / 2 and O_i = (Z_i - conj Z_(N-i)) /
// (2i), and the real spectrum is X_i = E_i + w^i O_i, X_(N-i) = conj(E_i -
// w^i O_i), w = exp(-i pi / N).  After the filter, Y = H X, the same relations
// taken backwards give Z', whose inverse DFT holds the filtered samples in
// pairs.  In the four-step layout bin i = k2 + N2 k1 sits in row k2 and its
// mirror N - i in row N2 - k2 at k1' = N1 - 1 - k1 (row 0: k1' = -k1 mod N1),
// so one workgroup transforms rows k2 and N2 - k2 together and hands each
// row to the other through LDS.
__device__ __forceinline__ float2 tw2_fwd(const LargeArgs& a, int64_t m) {
  return expi_pow2(m, a.lgn + 1);
}

// Chirp of Eq. 3 about the lower band edge at real-spectrum bin j (0 .. N):
// f = j bw / N above f_lo, q = D DM f^2 / (f_lo^2 (f_lo + f)) = B j^2 /
// (1 + beta j) turns in FP64, reduced before the FP32 rotation; times the
// band taper at x = j/N - 1/2 and the 1/N of the inverse transform.
__device__ __forceinline__ float2 band_chirp(const LargeArgs& a, double B, double beta,
                                             int64_t j, float inv_n) {
  const double s = (double)j;
  const double q = (B * (s * s)) / fma(beta, s, 1.0);
  const float2 h = expi_neg_turns(q);
  const float g = inv_n * taper_gain<false>(a.taper, (float)j * inv_n - 0.5f);
  return make_float2(h.x * g, h.y * g);
}

// The chirp function of one call for every real-spectrum bin, shared by all
// blocks of the record, in the order the row pass reads it: entry
// k2 N1 + k1 holds bin j = k2 + N2 k1 (j < N), entry N the Nyquist bin.
__global__ __launch_bounds__(256) void band_chirp_table_kernel(LargeArgs a, int64_t N,
                                                               float2* __restrict__ hb) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx > N) return;
  const int64_t j = idx == N ? N : idx / a.N1 + (int64_t)a.N2 * (idx % a.N1);
  const double dfn = a.bw / (double)N;
  const double B = a.dconst * a.dm * dfn * dfn / (a.f_lo * a.f_lo * a.f_lo);
  const double beta = dfn / a.f_lo;
  hb[idx] = band_chirp(a, B, beta, j, 1.0f / (float)N);
}

template <int L, int LDSF>
constexpr int pair_stride() {
  return 2 * L > LDSF + 1 ? 2 * L : ((LDSF + 1 + 3) & ~3);
}

// One mirror pair of the packed spectrum: from Z_i and Z_(N-i) (z, zm) to
// the filtered Z'_i and Z'_(N-i).  With E' = (Y_i + conj Y_(N-i)) / 2 and
// O' = (Y_i - conj Y_(N-i)) conj(w^i) / 2, Z'_i = E' + i O' and
// Z'_(N-i) = conj(E') + i conj(O').
__device__ __forceinline__ void real_pair(const LargeArgs& a, int64_t i, float2 hp, float2 hm,
                                          float2 z, float2 zm, float2* zi, float2* zmi) {
  const float2 e = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
  const float2 o = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
  const float2 w = tw2_fwd(a, i);
  const float2 wo = cmul(w, o);
  float2 yp = cmul(cadd(e, wo), hp);
  float2 ym = cmul(make_float2(e.x - wo.x, wo.y - e.y), hm);
  if (i == 0) {  // DC and Nyquist of a real series are real
    yp.y = 0.f;
    ym.y = 0.f;
  }
  const float2 e2 = make_float2(0.5f * (yp.x + ym.x), 0.5f * (yp.y - ym.y));
  const float2 o2 = cmul(make_float2(0.5f * (yp.x - ym.x), 0.5f * (yp.y + ym.y)),
                         make_float2(w.x, -w.y));
  *zi = make_float2(e2.x - o2.y, e2.y + o2.x);
  *zmi = make_float2(e2.x + o2.y, o2.x - e2.y);
}

template <class SR, int G>
__global__ __launch_bounds__(SR::T * G) void rows_real_kernel(const LargeArgs a) {
  constexpr int L = SR::N, STRIDE = pair_stride<SR::N, SR::lds_floats()>();
  __shared__ __align__(16) float lds[G * STRIDE];
  constexpr int R0 = SR::rad_f(0), B0 = L / (R0 * SR::T);
  constexpr int RL = SR::rad_f(SR::NP - 1), BL = L / (RL * SR::T);
  const int t = threadIdx.x, g = t / SR::T, tl = t % SR::T;
  // N2/2 row pairs per item, G/2 per workgroup: (0, N2/2), then (k, N2 - k)
  const int ngrp = a.N2 / G;
  const int64_t item = a.item0 + blockIdx.x / ngrp;
  const int pair = (blockIdx.x % ngrp) * (G / 2) + (g >> 1);
  const int side = g & 1;
  const int k2 = pair == 0 ? side * (a.N2 / 2) : (side ? a.N2 - pair : pair);
  const int64_t N = (int64_t)a.N1 * a.N2;
  float2* row = a.S + (item - a.item0) * N + spec_row(a, k2) * a.N1;
  float2 v[SR::E];
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) v[b * R0 + r] = row[tl + SR::T * b + r * (L / R0)];
  float* my = lds + g * STRIDE;
  fft_forward<SR>(v, my, a.twr, tl);
  __syncthreads();  // every read of the last exchange is done
  float2* mine = (float2*)my;
#pragma unroll
  for (int b = 0; b < BL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) mine[tl + SR::T * b + r * (L / RL)] = v[b * RL + r];
  __syncthreads();
  // Each mirror pair is filtered once, in place.  A row pair (k, N2 - k):
  // bin k1 of row k pairs with N1 - 1 - k1 of row N2 - k; side s takes
  // k1 in [s N1/2, (s+1) N1/2).  Row 0 pairs k1 with -k1 mod N1 (k1 = 0 and
  // N1/2 with themselves); row N2/2 pairs k1 with N1 - 1 - k1.
  float2* rowA = (float2*)(lds + (pair == 0 ? g : (g & ~1)) * STRIDE);
  float2* rowB = (float2*)(lds + (pair == 0 ? g : (g | 1)) * STRIDE);
  const int kA = pair == 0 ? k2 : pair;
  const int kB = pair == 0 ? k2 : a.N2 - pair;
  const float2* hA = a.hb + (int64_t)kA * L;  // chirp of row kA's bins, then row kB's
  const float2* hB = a.hb + (int64_t)kB * L;
  const float2 hnyq = a.hb[N];
  constexpr int half = L / 2;
#pragma unroll 2
  for (int p = tl; p < half; p += SR::T) {
    int k1, k1m;
    if (pair != 0) {
      k1 = p + side * half;
      k1m = L - 1 - k1;
    } else if (side == 0) {
      k1 = p;
      k1m = (L - p) & (L - 1);
    } else {
      k1 = p;
      k1m = L - 1 - p;
    }
    float2 zi, zmi;
    const int64_t i = kA + (int64_t)a.N2 * k1;
    real_pair(a, i, hA[k1], i == 0 ? hnyq : hB[k1m], rowA[k1], rowB[k1m], &zi, &zmi);
    rowA[k1] = zi;
    rowB[k1m] = zmi;
    if (pair == 0 && side == 0 && p == 0) {
      real_pair(a, (int64_t)a.N2 * half, hA[half], hA[half], rowA[half], rowA[half], &zi, &zmi);
      rowA[half] = zi;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) v[b * RL + r] = mine[tl + SR::T * b + r * (L / RL)];
  fft_inverse<SR>(v, my, a.twr, tl);  // its first exchange waits for the reads above
#pragma unroll
  for (int b = 0; b < B0; ++b)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n1 = tl + SR::T * b + r * (L / R0);
      const float2 w = tw4_fwd(a, (int64_t)n1 * k2);
      row[n1] = cmul(v[b * R0 + r], make_float2(w.x, -w.y));
    }
}

// Inverse transform of recorded spectra (Sec. 2.3, 3.1).  Record s holds
// bins 0 .. L-1 of a 2L-point real FFT as int8 (re, im); the Nyquist bin is
// not recorded and the DC bin's imaginary part is dropped.  Packed as above
// (with w = exp(-i pi / L) and X_L = 0), the record becomes L complex values
// Z_c = (E_c + i O_c), whose inverse DFT (times 1/L) is the record's 2L real
// samples in pairs.  A group of SC::T lanes handles one record; G records
// per workgroup.  The workgroups loop over groups of G records (grid-stride),
// each lane holding the next group's words in registers while the current
// group is transformed and stored, so loads, transforms and stores of
// different groups overlap instead of every workgroup loading, then
// transforming, then storing at the same time.
template <class SC, int G>
__global__ __launch_bounds__(SC::T * G) void gsb_inverse_kernel(
    const uint32_t* __restrict__ spec, float2* __restrict__ out,
    const float2* __restrict__ pre, const float2* __restrict__ tw, int64_t nspec) {
  constexpr int L = SC::N, STRIDE = pair_stride<SC::N, SC::lds_floats()>();
  constexpr int W = L / 2 / SC::T;  // words (two bins each) per lane per record
  static_assert(STRIDE % 4 == 0, "records are staged as float4");
  static_assert(W * SC::T == L / 2, "lanes tile a record's words");
  __shared__ __align__(16) float lds[G * STRIDE];
  constexpr int RI = SC::rad_i(0), BI = L / (RI * SC::T);
  constexpr int R0 = SC::rad_f(0), B0 = L / (R0 * SC::T);
  const int t = threadIdx.x, g = t / SC::T, tl = t % SC::T;
  const int64_t ngroups = (nspec + G - 1) / G;
  float* my = lds + g * STRIDE;
  float4* X4 = (float4*)my;
  const float sc = 0.5f / (float)L;
  uint32_t wd[W];
  auto fetch = [&](int64_t grp) {
    const int64_t s = grp * G + g;
    const bool ok = grp < ngroups && s < nspec;
#pragma unroll
    for (int j = 0; j < W; ++j) wd[j] = ok ? spec[s * (L / 2) + tl + SC::T * j] : 0u;
  };
  fetch(blockIdx.x);
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t s = grp * G + g;
    const bool live = s < nspec;
    __syncthreads();  // the previous group's transform is done with the LDS
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const uint32_t w = wd[j];
      X4[tl + SC::T * j] = make_float4((float)(int8_t)(w & 0xffu),
                                       (float)(int8_t)((w >> 8) & 0xffu),
                                       (float)(int8_t)((w >> 16) & 0xffu),
                                       (float)(int8_t)(w >> 24));
    }
    fetch(grp + gridDim.x);  // in flight during this group's transform
    __syncthreads();
    const float2* X = (const float2*)my;
    float2 v[SC::E];
#pragma unroll
    for (int b = 0; b < BI; ++b)
#pragma unroll
      for (int r = 0; r < RI; ++r) {
        const int c = tl + SC::T * b + r * (L / RI);
        float2 x = X[c];
        float2 m = make_float2(0.f, 0.f);
        if (c == 0)
          x.y = 0.f;
        else
          m = X[L - c];
        const float2 e = make_float2(x.x + m.x, x.y - m.y);                    // 2 E_c
        const float2 o = cmul(make_float2(x.x - m.x, x.y + m.y), pre[c]);      // 2 O_c
        v[b * RI + r] = make_float2(sc * (e.x - o.y), sc * (e.y + o.x));
      }
    fft_inverse<SC>(v, my, tw, tl);  // its first exchange waits for the reads above
    if (live) {
#pragma unroll
      for (int b = 0; b < B0; ++b)
#pragma unroll
        for (int r = 0; r < R0; ++r) out[s * L + tl + SC::T * b + r * (L / R0)] = v[b * R0 + r];
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr int64_t kChunkBytes = (int64_t)512 << 20;  // intermediate spectra per chunk

bool large_supported(int N) { return N >= (1 << 15) && N <= (1 << 26) && (N & (N - 1)) == 0; }

// The fused integration leaves two partial sums per run of G >= 8 samples
// of every item of a chunk in the |y|^2 buffer: at most N bytes per item.
size_t large_partial_bytes(int64_t N, int64_t items) { return (size_t)items * (size_t)N; }

int64_t large_chunk_items(const BeamPlan& p) {
  const int64_t items = (int64_t)p.nchan * p.nblocks;
  const int64_t per = std::max<int64_t>(1, kChunkBytes / ((int64_t)p.N * 8));
  return std::min(items, per);
}

// How an N = 2^LGN point transform is split: N1 = 2^LG1 (rows), and the
// column dimension N2 = A B with A = 2^LGA, B = 2^LGB.  Up to 2^22 points
// two levels; beyond, three, with every sub-transform between 128 and 2048
// points.  Up to 2^22 the columns are 2^(LGN/2) long, except from 2^16 to
// 2^20 points, where columns half as long (rows twice as long) measured
// faster: the column passes then hold half the data per workgroup and more
// workgroups fit on a CU (2^18-point channel transforms 0.175 -> 0.168 ms per
// call on the 2^23-sample single-channel workload; the full band at 2^19,
// 2^20 and 2^21 real points 0.195 -> 0.184, 0.162 -> 0.144 and 0.181 ->
// 0.153 ms, with the row groups below).
template <int LGN>
struct Split {
  static constexpr int LGA = LGN <= 22 ? 0 : (LGN >= 26 ? 8 : 7);
  static constexpr int LGB = LGN > 22 ? 7 : (LGN >= 16 && LGN <= 20) ? LGN / 2 - 1 : LGN / 2;
  static constexpr int LG1 = LGN - LGA - LGB;
  static constexpr int N1 = 1 << LG1, A = 1 << LGA, B = 1 << LGB, N2 = A * B;
  static constexpr bool THREE = LGA > 0;
  using SC = typename SubSched<B>::type;                   // last column sub-transform
  using SA = typename SubSched<THREE ? A : 128>::type;     // middle one (three levels)
  using SR = typename SubSched<N1>::type;                  // rows
  static constexpr int GC = SC::T * 16 <= 1024 ? 16 : 8;
  // The forward column pass of the two-level channel transforms takes 32
  // adjacent columns per workgroup where that stays within 512 threads
  // (columns of up to 256 points): 256-byte runs instead of 128.  Measured
  // on the single-channel workload (2^18 = 1024 x 256): 0.158 -> 0.154 ms
  // per call at 2^23 samples, 1.31 -> 1.28 ms at 2^26.  The inverse pass
  // (0.153 -> 0.158 ms that way) and the full band's forward pass (2048-point
  // rows, 16 KB between the rows of a run) keep GC.
  static constexpr int GW = !THREE && SC::T * GC * 2 <= 512 ? 2 * GC : GC;
  static constexpr int GA = SA::T * 16 <= 1024 ? 16 : 8;
  static_assert(LG1 >= 7 && LG1 <= 11 && N1 % GC == 0 && N1 % GW == 0 && N1 % GA == 0,
                "sub-transforms of 128 .. 2048 points, column groups tiling N1");
};

// Rows per workgroup of the row pass (T threads per row): at most eight and
// at most 256 threads.  Small workgroups let several be resident per CU at
// different phases (loads of one beside the transforms of another); 1024-point
// rows four to a workgroup instead of eight: 0.168 -> 0.158 ms per call on
// the 2^23-sample single-channel workload; 2048-point rows two instead of
// four: 2^22-point channel transforms 1.40 -> 1.37 ms, full band at 2^20
// real points 0.156 -> 0.144 ms.  (With the real series each workgroup holds
// mirror-row pairs, so the count stays even.)
constexpr int rows_per_group(int T) { return T * 8 <= 256 ? 8 : 256 / T; }

// Fill the split-dependent fields of a and its sub-transform twiddles.
template <int LGN>
static int set_split(LargeArgs& a) {
  using SP = Split<LGN>;
  int e = twiddles_of<typename SP::SC>(&a.twc);
  if (!e) e = twiddles_of<typename SP::SR>(&a.twr);
  if (!e && SP::THREE) e = twiddles_of<typename SP::SA>(&a.twm);
  a.N1 = SP::N1;
  a.N2 = SP::N2;
  a.A = SP::A;
  a.lgB = SP::LGB;
  a.lg2 = SP::LGA + SP::LGB;
  a.lgn = LGN;
  return e;
}

// The passes over one chunk of q items (blocks of one or more channels):
// columns forward, rows (chirp; REAL: the mirror-pair filter of the real
// series), columns inverse with the kept window, detection and (fused)
// integration.  GR rows per workgroup.
template <int LGN, int DT, bool REAL, int GR>
static int run_passes(const LargeArgs& a, int64_t q, hipStream_t st) {
  using SP = Split<LGN>;
  using SC = typename SP::SC;
  using SA = typename SP::SA;
  using SR = typename SP::SR;
  constexpr int GC = SP::GC, GA = SP::GA;
  static_assert(SP::N2 % GR == 0 && (!REAL || GR % 2 == 0), "row groups tile N2");
  constexpr int GF = REAL ? GC : SP::GW;
  const int64_t gc = q * SP::A * (SP::N1 / GC), ga = q * SP::B * (SP::N1 / GA);
  const int64_t gf = q * SP::A * (SP::N1 / GF);
  const int64_t gr = q * (SP::N2 / GR);
  if (gc > 0x7fffffffLL || gf > 0x7fffffffLL || ga > 0x7fffffffLL || gr > 0x7fffffffLL)
    return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL((cols_fwd_kernel<SC, GF, DT, SP::THREE>), dim3((unsigned)gf),
                     dim3(SC::T * GF), 0, st, a);
  if constexpr (SP::THREE)
    hipLaunchKernelGGL((cols_mid_kernel<SA, GA, false>), dim3((unsigned)ga), dim3(SA::T * GA), 0,
                       st, a);
  if (REAL)
    hipLaunchKernelGGL((rows_real_kernel<SR, GR>), dim3((unsigned)gr), dim3(SR::T * GR), 0, st,
                       a);
  else
    hipLaunchKernelGGL((rows_kernel<SR, GR>), dim3((unsigned)gr), dim3(SR::T * GR), 0, st, a);
  if constexpr (SP::THREE)
    hipLaunchKernelGGL((cols_mid_kernel<SA, GA, true>), dim3((unsigned)ga), dim3(SA::T * GA), 0,
                       st, a);
  hipLaunchKernelGGL((cols_inv_kernel<SC, GC, SP::THREE>), dim3((unsigned)gc), dim3(SC::T * GC),
                     0, st, a);
  int e = 0;
  if (a.fuse && (e = launch_fixup(a, GC, q, st))) return e;
  return (int)hipGetLastError();
}

template <int LGN>
static int launch_large_t(const BeamPlan& p, const void* xt, double dm, float2* S, float* pbuf,
                          float* P, void* vout, int exact_div, int32_t* cov_fill, int64_t cov_n,
                          void* stream) {
  using SP = Split<LGN>;
  using SR = typename SP::SR;
  constexpr int GR = rows_per_group(SR::T);
  LargeArgs a{};
  int e = set_split<LGN>(a);
  if (e) return e;
  a.x = xt;
  a.S = S;
  a.p = pbuf;
  a.vout = (float2*)vout;
  a.nsamp = p.nsamp;
  a.nblocks = p.nblocks;
  a.nchan = p.nchan;
  a.M = p.M;
  a.nfront = p.nfront;
  a.phase_mode = p.phase_mode;
  a.taper = p.taper;
  a.exact_div = exact_div;
  a.f_lo = p.f_lo;
  a.df = p.df;
  a.dconst = p.dconst;
  a.dm = dm;
  a.P = P;
  a.t_int = p.t_int;
  a.n_int = p.n_int;
  a.fuse = SP::GC % p.n_int == 0 ? 1 : 0;
  a.cov_fill = cov_fill;
  a.cov_n = cov_fill ? cov_n : 0;
  hipStream_t st = (hipStream_t)stream;
  const int64_t items = (int64_t)p.nchan * p.nblocks;
  const int64_t chunk = large_chunk_items(p);
  // the call's chirp table follows the chunk of spectra in the workspace
  constexpr int64_t NP = (int64_t)1 << LGN;
  a.hb = S + chunk * NP;
  const int64_t nt = (std::max<int64_t>(NP * p.nchan, a.cov_n) + 255) / 256;
  if (nt > 0x7fffffffLL) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(chan_chirp_table_kernel, dim3((unsigned)nt), dim3(256), 0, st, a, NP,
                     (float2*)a.hb);
  for (int64_t i0 = 0; i0 < items; i0 += chunk) {
    const int64_t q = std::min(chunk, items - i0);
    a.item0 = i0;
    e = p.dtype == CDD_CI8 ? run_passes<LGN, CDD_CI8, false, GR>(a, q, st)
                           : run_passes<LGN, CDD_CF32, false, GR>(a, q, st);
    if (e) return e;
  }
  return a.fuse ? 0 : launch_integrate(pbuf, P, p.nsamp, p.t_int, p.n_int, p.nchan, st);
}

// exp(+i pi c / L), c < L: the post-twiddle of the packed real inverse.
template <int LG>
static std::vector<float2> make_gsb_pre() {
  const int L = 1 << LG;
  std::vector<float2> t(L);
  for (int c = 0; c < L; ++c) {
    const double ang = M_PI * (double)c / (double)L;
    t[c] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  return t;
}

bool gsb_supported(int nchan) { return nchan >= 128 && nchan <= 2048 && (nchan & (nchan - 1)) == 0; }

template <int LG>
static int launch_gsb_t(const void* spec, int64_t nspec, float* series, void* stream) {
  using SC = typename SubSched<(1 << LG)>::type;
  constexpr int G = SC::T >= 256 ? 1 : 256 / SC::T;
  const float2* tw = nullptr;
  const float2* pre = nullptr;
  int e = twiddles_of<SC>(&tw);
  if (!e) e = cached_table((std::string("gsbpre") + std::to_string(LG)).c_str(),
                           &make_gsb_pre<LG>, &pre);
  if (e) return e;
  const int64_t ngroups = (nspec + G - 1) / G;
  if (ngroups < 1) return (int)hipErrorInvalidValue;
  // as many workgroups as are resident at once (each loops over groups of
  // records): 0.0265 -> 0.0217 ms for the 16,384 records of 512 bins of the
  // 16 MHz full-band workload, against one workgroup per group
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (he == hipSuccess)
    he = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&gsb_inverse_kernel<SC, G>), SC::T * G, 0);
  if (he != hipSuccess) return (int)he;
  const int64_t nb =
      std::min<int64_t>(ngroups, (int64_t)std::max(ncu, 1) * std::max(per_cu, 1));
  hipLaunchKernelGGL((gsb_inverse_kernel<SC, G>), dim3((unsigned)nb), dim3(SC::T * G), 0,
                     (hipStream_t)stream, (const uint32_t*)spec, (float2*)series, pre, tw, nspec);
  return (int)hipGetLastError();
}

int launch_gsb_inverse(const void* spec, int64_t nspec, int32_t nchan, float* series,
                       void* stream) {
  switch (nchan) {
    case 128: return launch_gsb_t<7>(spec, nspec, series, stream);
    case 256: return launch_gsb_t<8>(spec, nspec, series, stream);
    case 512: return launch_gsb_t<9>(spec, nspec, series, stream);
    case 1024: return launch_gsb_t<10>(spec, nspec, series, stream);
    case 2048: return launch_gsb_t<11>(spec, nspec, series, stream);
  }
  return (int)hipErrorInvalidValue;
}

int64_t fullband_chunk_blocks(const FullbandPlan& f) {
  const int64_t per = std::max<int64_t>(1, kChunkBytes / ((int64_t)(f.N / 2) * 8));
  return std::min(f.nblocks, per);
}

template <int LGN>
static int launch_fullband_t(const FullbandPlan& f, const float* series, float2* S, float* pbuf,
                             float2* hb, float* I, float* vout, void* stream) {
  using SP = Split<LGN>;
  using SR = typename SP::SR;
  constexpr int GR = rows_per_group(SR::T);
  LargeArgs a{};
  int e = set_split<LGN>(a);
  if (e) return e;
  a.x = series;
  a.S = S;
  a.p = pbuf;
  a.vout = (float2*)vout;
  a.nsamp = f.nsamp / 2;
  a.nblocks = f.nblocks;
  a.nchan = 1;
  a.M = f.M / 2;
  a.nfront = f.nfront / 2;
  a.phase_mode = CDD_PHASE_FP64_REDUCED;
  a.taper = f.taper;
  a.exact_div = 1;
  a.f_lo = f.f_lo;
  a.bw = f.bw;
  a.df = f.bw;
  a.dconst = f.dconst;
  a.dm = f.dm;
  a.hb = hb;
  a.P = I;
  a.t_int = f.t_int;
  a.n_int = f.n_int / 2;  // pairs of real samples
  a.fuse = SP::GC % (f.n_int / 2) == 0 ? 1 : 0;
  hipStream_t st = (hipStream_t)stream;
  constexpr int64_t NP = (int64_t)1 << LGN;
  hipLaunchKernelGGL(band_chirp_table_kernel, dim3((unsigned)((NP + 256) / 256)), dim3(256), 0,
                     st, a, NP, hb);
  const int64_t chunk = fullband_chunk_blocks(f);
  for (int64_t i0 = 0; i0 < f.nblocks; i0 += chunk) {
    const int64_t q = std::min(chunk, f.nblocks - i0);
    a.item0 = i0;
    if ((e = run_passes<LGN, CDD_CF32, true, GR>(a, q, st))) return e;
  }
  return a.fuse ? 0 : launch_integrate(pbuf, I, f.nsamp / 2, f.t_int, f.n_int / 2, 1, st);
}

int launch_fullband(const FullbandPlan& f, const float* series, void* Sv, float* pbuf,
                    void* Hv, float* I, float* vout, void* stream) {
  float2* S = (float2*)Sv;
  float2* H = (float2*)Hv;
  switch (f.N) {
    case 1 << 16: return launch_fullband_t<15>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 17: return launch_fullband_t<16>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 18: return launch_fullband_t<17>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 19: return launch_fullband_t<18>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 20: return launch_fullband_t<19>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 21: return launch_fullband_t<20>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 22: return launch_fullband_t<21>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 23: return launch_fullband_t<22>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 24: return launch_fullband_t<23>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 25: return launch_fullband_t<24>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 26: return launch_fullband_t<25>(f, series, S, pbuf, H, I, vout, stream);
    case 1 << 27: return launch_fullband_t<26>(f, series, S, pbuf, H, I, vout, stream);
  }
  return (int)hipErrorInvalidValue;
}

int exact_division_needed(const BeamPlan& p, double dm_abs_max);

int launch_large(const BeamPlan& p, const void* xt, double dm, void* Sv, float* pbuf, float* P,
                 void* vout, void* stream, int32_t* cov_fill, int64_t cov_n) {
  float2* S = (float2*)Sv;
  const int ex = exact_division_needed(p, std::fabs(dm));
  switch (p.N) {
    case 1 << 15: return launch_large_t<15>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 16: return launch_large_t<16>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 17: return launch_large_t<17>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 18: return launch_large_t<18>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 19: return launch_large_t<19>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 20: return launch_large_t<20>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 21: return launch_large_t<21>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 22: return launch_large_t<22>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 23: return launch_large_t<23>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 24: return launch_large_t<24>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 25: return launch_large_t<25>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
    case 1 << 26: return launch_large_t<26>(p, xt, dm, S, pbuf, P, vout, ex, cov_fill, cov_n, stream);
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace cdd
