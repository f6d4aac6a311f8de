// Full-band mode (the paper's unchannelised pipeline, Sec. 2.1, 2.3, 3.1):
// declarations shared by the host entry points and the kernels.
#pragma once

#include <cstdint>

#include "cdd_internal.h"

namespace cdd {

// One recorded beam of real-FFT spectra dedispersed as a single band.  All
// lengths are in real samples at the rate 2 bw.
struct FullbandPlan {
  int64_t nspec = 0;                  // records
  int32_t nchan = 0;                  // bins per record (2 nchan-point real FFT)
  int64_t nsamp = 0;                  // real samples, nspec * 2 nchan
  double f_lo = 0, bw = 0, dconst = kDefaultD, dm = 0;
  int32_t n_int = 2;                  // even
  int32_t taper = CDD_TAPER_NONE;
  int32_t N = 0, L = 0, nfront = 0, M = 0;  // N, L, nfront, M = N - L: all even
  int32_t front = 0, back = 0;
  int64_t nblocks = 0, t_int = 0;
};

constexpr int kMinFullband = 1 << 16;  // real points (2^15 packed complex)
constexpr int kMaxFullband = 1 << 27;

bool gsb_supported(int nchan);  // nchan a power of two in [128, 2048]
// Inverse transform of nspec records of nchan int8 (re, im) bins into
// nspec * 2 nchan real samples.  spec 4-byte aligned, series 8-byte aligned.
int launch_gsb_inverse(const void* spec, int64_t nspec, int32_t nchan, float* series,
                       void* stream);
int64_t fullband_chunk_blocks(const FullbandPlan& f);  // blocks per chunk of spectra
// Overlap-save of the real series with the band chirp, y^2 integrated into
// intensity [t_int]; vout (nullable) receives the dedispersed series [nsamp].
// S holds fullband_chunk_blocks * N/2 complex values, pbuf nsamp/2 floats
// (or large_partial_bytes of a chunk, if more),
// H the call's chirp function, N/2 + 1 complex values.
int launch_fullband(const FullbandPlan& f, const float* series, void* S, float* pbuf, void* H,
                    float* intensity, float* vout, void* stream);

}  // namespace cdd
