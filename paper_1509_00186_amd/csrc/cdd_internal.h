// Internal declarations shared by the host API, the planner and the kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "cdd.h"

namespace cdd {

constexpr double kDefaultD = 4.148808e9;  // Eq. 3's D (us MHz^2 cm^3 / pc)
constexpr int kMinFFT = 256;
constexpr int kMaxFFT = 1 << 26;
constexpr int kMaxDmTile = 64;            // DM trials per batched launch
constexpr int64_t kMaxChunks = 12;        // time chunks of the pipelined one-shot path

// Thread-local error message and status (set by every failing call).
cdd_status fail(cdd_status s, const char* fmt, ...);
void clear_error();

// Channel geometry and the overlap-save plan of one beam (all DMs share it).
struct BeamPlan {
  int32_t dtype = CDD_CI8;
  int64_t nsamp = 0;
  int32_t nchan = 0;
  double f_centre = 0, bw = 0, df = 0, f_lo = 0, dconst = kDefaultD;
  int32_t n_int = 1;
  int32_t phase_mode = CDD_PHASE_FP64_REDUCED;
  int32_t taper = CDD_TAPER_NONE;
  int32_t variant = 0;  // block-kernel schedule (autotuner choice)
  int32_t dm_tile = 0;  // DM trials per batched launch (autotuner choice; 0 = as many as fit)
  std::vector<double> dms;
  int32_t N = 0, L = 0, nfront = 0, M = 0;
  int32_t front = 0, back = 0;
  int64_t nblocks = 0, t_int = 0, d_max = 0;
};

// Fill a BeamPlan from the call arguments, applying the length, overlap
// and front-discard rules (Sec. 2.2, 2.3) unless opts->explicit_plan.
cdd_status make_plan(int32_t dtype, int64_t nsamp, int32_t nchan,
                     double f_centre, double bw, const double* dms, int32_t ndm,
                     int32_t fft_len, int32_t n_int, const cdd_opts* opts,
                     BeamPlan* out);

// FP64 channel centre, same operation order as the device code.
double channel_centre(const BeamPlan& p, int c);
// FP64 delay of channel c in integrated samples (Sec. 1.2, Eq. 2).
int64_t channel_delay(const BeamPlan& p, double dm, int c);

// Workspace layout for one beam (one DM tile).
struct WsLayout {
  size_t xt_off = 0, xt_bytes = 0;   // channel-major copy of the input
  size_t p_off = 0, p_bytes = 0;     // per-channel intensities [ndm][C][T_int]
  size_t d_off = 0, d_bytes = 0;     // delays [ndm][C] int32
  size_t s_off = 0, s_bytes = 0;     // long transforms: spectra of one chunk
  size_t pb_off = 0, pb_bytes = 0;   // long transforms: |y|^2 per sample [C][nsamp]
  size_t h_off = 0, h_bytes = 0;     // one DM: chirp table [C][N] complex float
  size_t total = 0;
};
WsLayout ws_layout(const BeamPlan& p, int ndm_tile, bool need_p, bool chirp_table = false);
// Samples between channel rows of the channel-major copy of a record: for
// the block kernels and the incoherent detection nsamp rounded up to 64
// (every row starts on a 128-byte boundary, so the layout change writes
// whole cache lines); for the long transforms nsamp.
int64_t xt_stride(const BeamPlan& p);

// ---------------------------------------------------------------------
// Launchers (defined in the .hip files).  Return hipError_t as int.
// ---------------------------------------------------------------------
struct DmTile {
  int32_t ndm = 0;
  double dm[kMaxDmTile];
};

// Launch-relative coordinates of one beam: block k reads input samples
// k*M - load_off + n (valid in [0, x_len), channel stride x_stride), writes
// integrated samples u = k*M/n_int + ul (u < u_lim) to
// P[dmi*p_dm_stride + c*p_stride + u] and voltages o = k*M + m (o < o_lim) to
// vout[c*v_stride + o].
struct Coords {
  int64_t x_stride = 0, x_len = 0, load_off = 0;
  int64_t p_stride = 0, p_dm_stride = 0, u_lim = 0;
  int64_t v_stride = 0, o_lim = 0;
  int64_t nblocks = 0;
  int32_t accum = 0;  // 1: add the integrated samples to P (second polarisation)
};
Coords offline_coords(const BeamPlan& p);

// Time-major [nsamp][nchan] -> out[c*out_stride + t].
int launch_transpose(const void* in, void* out, int32_t dtype, int64_t nsamp,
                     int32_t nchan, int64_t out_stride, void* stream);
// With one DM trial the block kernel takes the chirp from a table H built
// by launch_chirp_table (chirp_table_bytes of device memory); with several
// it forms the chirp itself and H is ignored.
int launch_block(const BeamPlan& p, const void* xt, const DmTile& dms,
                 float* P, void* vout, const void* H, void* stream);
int launch_block_co(const BeamPlan& p, const Coords& co, const void* xt, const DmTile& dms,
                    float* P, void* vout, const void* H, void* stream);
size_t chirp_table_bytes(const BeamPlan& p);
int launch_chirp_table(const BeamPlan& p, double dm, void* H, void* stream);
// The int8 layout change of a whole record (into [c][xt_stride]) with the
// one-DM chirp table (and, if delays is set, the channel delays at that DM)
// built by the same kernel; possible when the layout change has at least one
// workgroup per channel of the table.
bool transpose_chirp_fits(const BeamPlan& p);
int launch_transpose_chirp(const BeamPlan& p, const void* in, void* out, double dm, void* H,
                           void* stream, int32_t* delays = nullptr);
// One DM, block kernel, record split into time chunks with the layout change
// and the aligned sums on an auxiliary stream (cdd_pipeline.hip).
int run_pipelined(const BeamPlan& p, const void* voltages, double dm, char* xt, float* P,
                  int32_t* d, void* H, void* volt_out, float* I, int32_t* cov, int chunks,
                  int npol, void* stream);
// aux_work(aux stream) and main_work(stream) enqueued so that they run side
// by side: the library's auxiliary stream starts after the work already on
// `stream`, and `stream` goes on past this point only once both are done.
int fork_join(void* stream, const std::function<int(void*)>& aux_work,
              const std::function<int(void*)>& main_work);
// The library's auxiliary stream of the current device, held (one user at a
// time) from aux_open to aux_close: aux_open makes it start after the work
// already on `stream`; aux_mark makes `waiting` wait for everything enqueued
// on it so far; aux_after makes it wait for what `stream` holds so far;
// aux_close makes `stream` wait for all of it and releases it.
struct AuxSession {
  std::unique_lock<std::mutex> lk;
  void* aux = nullptr;   // hipStream_t
  void* impl = nullptr;
};
int aux_open(void* stream, AuxSession* session);
int aux_mark(AuxSession* session, void* waiting);
int aux_after(AuxSession* session, void* stream);  // aux waits for `stream`'s work so far
int aux_close(void* stream, AuxSession* session);
// Batched form: beams, each with its DM tile, in one launch.
struct BatchBeam {
  const BeamPlan* p;
  const void* xt;    // channel-major input
  DmTile dms;
  float* P;          // see Coords
  Coords co;
};
size_t batch_table_bytes(int nbeams);
// Launch kinds of the batched form:
//   kLaunchMixed  beams of any length in [256, 8192] (mixed_supported) in one
//                 persistent launch, each reading its chirp table (H[b]) or,
//                 with H[b] NULL, forming its chirp in the kernel;
//   kLaunchTables one-DM beams of one length, chirps from tables, one
//                 workgroup per (beam, channel, block);
//   kLaunchBatch  beams of one length with DM tiles, chirps in the kernel,
//                 one persistent launch (schedule variant of the first beam,
//                 if batch_variant_ok).
// All beams of a launch share one sample type; they are listed longest work
// per unit first.
enum { kLaunchMixed = 0, kLaunchTables = 1, kLaunchBatch = 2 };
struct LaunchDesc {
  int kind = 0, N = 0, variant = 0, nbeams = 0, multi = 0, dtype = 0;
  int64_t total = 0;  // work units
};
bool mixed_supported(int N);
bool batch_variant_ok(int N, int V);  // schedules the persistent batch kernel has
// Form the per-beam argument table of one launch in host_tab
// (batch_table_bytes(nbeams) bytes); H may be NULL (no tables).
int prepare_launch(int kind, const BatchBeam* beams, const void* const* H, int nbeams,
                   void* host_tab, LaunchDesc* d);
// Copy host_tab (unchanged until the stream has run the copy) to dev_tab and
// launch; counter is a device word for the persistent kinds.
int enqueue_launch(const LaunchDesc& d, const void* host_tab, void* dev_tab,
                   unsigned int* counter, void* stream);
// prepare_launch(kLaunchBatch) + enqueue_launch.
int launch_batch(const BatchBeam* beams, int nbeams, void* host_tab, void* dev_tab,
                 unsigned int* counter, void* stream);
int launch_delays(const BeamPlan& p, const DmTile& dms, int32_t* d, void* stream);
// v[i] = x for i < n (a kernel, not a memset, so the launch is capture-safe).
int launch_fill_i32(int32_t* v, int64_t n, int32_t x, void* stream);
// The whole path for one beam and one tile of DM trials, every launch on the
// one stream (workspace regions per ws_layout; xt_ready = an existing
// channel-major copy or NULL).  timed: record stage events when profiling.
cdd_status run_tile(const BeamPlan& p, const void* voltages, const DmTile& tile,
                    const void* xt_ready, char* ws, const WsLayout& lay, float* chan_P,
                    void* volt_out, float* intensity, int32_t* coverage, int64_t out_stride,
                    void* stream, bool timed);
cdd_status device_fail(const char* what, int err);
// P[c][u] = sum of |x[c][u n_int + r]|^2, r < n_int (channel-major x).
int launch_detect(const BeamPlan& p, const void* xt, float* P, void* stream);
int launch_fold(const float* I, int64_t t_int, double period, double phase0, int32_t nbins,
                float* profile, int32_t* counts, void* stream);
int launch_dsum(const BeamPlan& p, int ndm, const float* P, const int32_t* d,
                float* I, int32_t* cov, int64_t out_stride, void* stream);
// General form: for u in [u_begin, u_begin + u_count),
// I[i*out_stride + u - u_begin] = sum over c with u + d_c < src_lim of
// P[i*p_dm_stride + c*p_stride + u + d_c].
int launch_dsum_range(int nchan, int ndm, const float* P, int64_t p_stride,
                      int64_t p_dm_stride, int64_t src_lim, int64_t u_begin,
                      int64_t u_count, const int32_t* d, float* I, int32_t* cov,
                      int64_t out_stride, void* stream);
bool block_supported(int N);
bool large_supported(int N);
int64_t large_chunk_items(const BeamPlan& p);  // (channel, block) items per chunk
// bytes of the partial integration sums of `items` N-point items (the
// |y|^2 buffer holds them when integration is fused; it must be this large)
size_t large_partial_bytes(int64_t N, int64_t items);
int launch_large(const BeamPlan& p, const void* xt, double dm, void* S, float* pbuf,
                 float* P, void* vout, void* stream, int32_t* cov_fill = nullptr,
                 int64_t cov_n = 0);  // cov_fill: cov_n entries set to 1 as well
int block_variants(int N);  // number of schedules compiled for N

// Stage timing (cdd_profile.hip): no-ops unless profiling is enabled.
bool profiling();
int stage_begin(int stage, void* stream, void** token);
int stage_end(int stage, void* stream, void* token);
enum { kStageTranspose = 0, kStageDelays = 1, kStageBlock = 2, kStageDsum = 3 };
const char* hip_error_string(int err);

}  // namespace cdd
