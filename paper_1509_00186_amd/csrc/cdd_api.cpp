// C-ABI entry points: one-shot dedispersion and batched plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "cdd_internal.h"

using namespace cdd;

namespace cdd {
cdd_status device_fail(const char* what, int err) {
  return fail(CDD_EDEVICE, "%s: %s", what, hip_error_string(err));
}
}  // namespace cdd

namespace {

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

// Layout change with stage timing; with H, the one-DM chirp table (of dm),
// and with delays the channel delays, are built by the same kernel.
int launch_transposed(const BeamPlan& p, const void* in, void* out, void* stream,
                      void* H = nullptr, double dm = 0.0, int32_t* delays = nullptr) {
  void* tok = nullptr;
  int e = stage_begin(kStageTranspose, stream, &tok);
  if (e) return e;
  if ((e = H ? launch_transpose_chirp(p, in, out, dm, H, stream, delays)
             : launch_transpose(in, out, p.dtype, p.nsamp, p.nchan, xt_stride(p), stream)))
    return e;
  return stage_end(kStageTranspose, stream, tok);
}

}  // namespace

namespace cdd {

// Run the path for one beam and one tile of DM trials, every kernel in order
// on the one stream.  With timed, stage timing records events when
// profiling is enabled; without, nothing but kernel launches is issued.
cdd_status run_tile(const BeamPlan& p, const void* voltages, const DmTile& tile,
                    const void* xt_ready, char* ws, const WsLayout& lay, float* chan_P,
                    void* volt_out, float* intensity, int32_t* coverage, int64_t out_stride,
                    void* stream, bool timed) {
  const void* xt = xt_ready;
  void* tok = nullptr;
  int e = 0;
  auto begin = [&](int stage) { return timed ? stage_begin(stage, stream, &tok) : 0; };
  auto end = [&](int stage) { return timed ? stage_end(stage, stream, tok) : 0; };
  // one DM on the block kernel: a chirp table, built by the layout change
  // itself when it can
  const bool table = block_supported(p.N) && tile.ndm == 1;
  if (table && lay.h_bytes < chirp_table_bytes(p))
    return fail(CDD_EINTERNAL, "no chirp table space");
  void* H = table ? ws + lay.h_off : nullptr;
  int32_t* d = (int32_t*)(ws + lay.d_off);
  bool table_built = false;  // the layout change built the table and the delays
  if (xt == nullptr) {
    if (p.nchan > 1) {
      table_built = table && transpose_chirp_fits(p);
      if ((e = begin(kStageTranspose)) ||
          (e = table_built ? launch_transpose_chirp(p, voltages, ws + lay.xt_off, tile.dm[0], H,
                                                    stream, d)
                           : launch_transpose(voltages, ws + lay.xt_off, p.dtype, p.nsamp,
                                              p.nchan, xt_stride(p), stream)) ||
          (e = end(kStageTranspose)))
        return device_fail("transpose launch", e);
      xt = ws + lay.xt_off;
    } else {
      xt = voltages;
    }
  }
  // One channel is its own delay reference (Eq. 2 relative to the top
  // channel for DM >= 0, the bottom one otherwise), so its delay is 0 and the
  // aligned sum is the identity: the transform kernels write the intensities
  // straight into the output (the same [trial][t_int] layout) and every
  // output sample has coverage 1.
  const bool direct = p.nchan == 1 && !chan_P && out_stride == p.t_int;
  float* P = direct ? intensity : chan_P ? chan_P : (float*)(ws + lay.p_off);
  if (!table_built) {
    if ((e = begin(kStageDelays))) return device_fail("event record", e);
    if (!direct && (e = launch_delays(p, tile, d, stream))) return device_fail("delay launch", e);
    if (table && (e = launch_chirp_table(p, tile.dm[0], H, stream)))
      return device_fail("chirp table launch", e);
    if ((e = end(kStageDelays))) return device_fail("event record", e);
  }
  if ((e = begin(kStageBlock))) return device_fail("event record", e);
  if (block_supported(p.N)) {
    if ((e = launch_block(p, xt, tile, P, volt_out, H, stream)))
      return device_fail("block kernel launch", e);
  } else {
    // long transforms: one DM trial at a time through the four-step kernels
    for (int i = 0; i < tile.ndm; ++i) {
      if ((e = launch_large(p, xt, tile.dm[i], ws + lay.s_off, (float*)(ws + lay.pb_off),
                            P + (int64_t)i * p.nchan * p.t_int, tile.ndm == 1 ? volt_out : nullptr,
                            stream, direct && i == 0 ? coverage : nullptr,
                            (int64_t)tile.ndm * p.t_int)))
        return device_fail("long-transform launch", e);
    }
  }
  if ((e = end(kStageBlock))) return device_fail("event record", e);
  if ((e = begin(kStageDsum))) return device_fail("event record", e);
  if (direct) {
    // (the long transforms' chirp-table kernel has set the coverage)
    if (coverage && block_supported(p.N) &&
        (e = launch_fill_i32(coverage, (int64_t)tile.ndm * p.t_int, 1, stream)))
      return device_fail("coverage launch", e);
  } else if ((e = launch_dsum(p, tile.ndm, P, d, intensity, coverage, out_stride, stream))) {
    return device_fail("delay-sum launch", e);
  }
  if ((e = end(kStageDsum))) return device_fail("event record", e);
  return CDD_OK;
}

}  // namespace cdd


struct cdd_plan {
  std::vector<BeamPlan> beams;
  std::vector<cdd_beam> desc;
  std::vector<int> tile;         // DM trials per launch, per beam
  std::vector<WsLayout> lay;     // per-beam workspace regions (offsets from ws_base)
  std::vector<size_t> ws_base;
  size_t tab_off = 0, cnt_off = 0;
  int rounds = 0;
  size_t ws = 0;
  int chirp_in_kernel = 0;       // one-DM beams form their chirp in the kernel
  int single_launch = 0;         // every length up to 8192 in one launch per round
  // Launch tables of every round in pinned host memory, copied into the
  // workspace on each execute.  They are rewritten only when their contents
  // change (another workspace), and then only once the previous execute's
  // copies have run.
  void* host_tab = nullptr;
  size_t host_tab_bytes = 0;
  hipEvent_t tab_done = nullptr;
  bool tab_pending = false;
  ~cdd_plan() {
    if (tab_done) (void)hipEventDestroy(tab_done);
    if (host_tab) (void)hipHostFree(host_tab);
  }
};

namespace {
constexpr size_t kPlanPBudget = (size_t)8 << 30;  // per-channel intensities held at once
// launch kinds of the single-launch form: (lengths up to 8192; 16384 with
// tables; 16384 in-kernel) x (int8, complex float)
constexpr int kGroupKinds = 6;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Whether a beam reads a chirp table built per execute (one DM trial, unless
// the plan forms every chirp in the kernel).
bool table_chirp(const cdd_plan* pl, const BeamPlan& p) {
  return block_supported(p.N) && p.dms.size() == 1 && !pl->chirp_in_kernel;
}

// DM tiles and workspace layout of a plan: each beam gets its own channel-major
// copy, intensity and delay regions (and its chirp table if it reads one);
// then the launch tables of every round and the work counters.
void layout_plan(cdd_plan* pl) {
  const size_t nb = pl->beams.size();
  pl->tile.assign(nb, 1);
  pl->lay.assign(nb, WsLayout());
  pl->ws_base.assign(nb, 0);
  size_t off = 0;
  pl->rounds = 0;
  // DM tiles: as many trials per launch as a beam has (up to kMaxDmTile),
  // scaled down in proportion when the intensities of all tiles would exceed
  // the budget
  double need = 0;
  for (size_t b = 0; b < nb; ++b) {
    const BeamPlan& p = pl->beams[b];
    if (block_supported(p.N))
      need += (double)std::min((int)p.dms.size(), kMaxDmTile) * p.nchan * p.t_int * sizeof(float);
  }
  const double scale = need > (double)kPlanPBudget ? (double)kPlanPBudget / need : 1.0;
  for (size_t b = 0; b < nb; ++b) {
    const BeamPlan& p = pl->beams[b];
    const int ndm = (int)p.dms.size();
    int t = 1;
    if (block_supported(p.N))
      t = std::max(1, (int)std::floor(std::min(ndm, kMaxDmTile) * scale));
    if (p.dm_tile > 0) t = std::min(t, p.dm_tile);
    pl->tile[b] = t;
    pl->lay[b] = ws_layout(p, t, true, table_chirp(pl, p));
    pl->ws_base[b] = off;
    off = align256(off + pl->lay[b].total);
    pl->rounds = std::max(pl->rounds, (ndm + t - 1) / t);
  }
  // launch-table slots: one per beam and round (pipelined form) or one per
  // launch kind and round (single-launch form), each big enough for all beams
  pl->tab_off = off;
  pl->host_tab_bytes = align256(batch_table_bytes((int)nb)) *
                       (size_t)std::max<size_t>(nb, kGroupKinds) *
                       (size_t)std::max(pl->rounds, 1);
  off = align256(off + pl->host_tab_bytes);
  pl->cnt_off = off;
  off = align256(off + 256);
  pl->ws = off;
}
}  // namespace

extern "C" {

cdd_status cdd_dedisperse(const void* voltages, int32_t dtype, int64_t nsamp, int32_t nchan,
                          double f_centre_mhz, double bw_mhz, double dm, int32_t fft_len,
                          int32_t n_int, float* intensity, int32_t* coverage,
                          float* chan_intensity, void* volt_out, const cdd_opts* opts,
                          void* workspace, size_t ws_bytes, void* stream) {
  try {
    if (!voltages) return fail(CDD_EINVAL, "voltages is NULL");
    if (!intensity) return fail(CDD_EINVAL, "intensity is NULL");
    if (opts && opts->time_chunks < 0) return fail(CDD_EINVAL, "time_chunks must be >= 0");
    BeamPlan p;
    cdd_status s = make_plan(dtype, nsamp, nchan, f_centre_mhz, bw_mhz, &dm, 1, fft_len, n_int,
                             opts, &p);
    if (s != CDD_OK) return s;
    if (!block_supported(p.N) && !large_supported(p.N))
      return fail(CDD_ENOTSUP, "fft_len %d is not supported by the library", p.N);
    WsLayout lay = ws_layout(p, 1, true, true);
    if (!workspace || ws_bytes < lay.total)
      return fail(CDD_EINVAL, "workspace too small: need %zu bytes, got %zu", lay.total,
                  workspace ? ws_bytes : (size_t)0);
    if (!aligned256(workspace)) return fail(CDD_EINVAL, "workspace must be 256-byte aligned");
    // time chunks of the overlapped path: one unless asked for more
    int chunks = 1;
    if (opts && opts->time_chunks > 0)
      chunks = (int)std::min<int64_t>({(int64_t)opts->time_chunks, p.nblocks, kMaxChunks});
    const int npol = (opts && opts->npol > 1) ? opts->npol : 1;
    if (opts && (opts->npol < 0 || opts->npol > 2))
      return fail(CDD_EINVAL, "npol must be 0, 1 or 2 (got %d)", opts->npol);
    if (npol == 2 && !(block_supported(p.N) && p.nchan > 1 && chunks == 1 && !volt_out))
      return fail(CDD_ENOTSUP,
                  "two polarisations need fft_len <= 16384, nchan > 1, one time chunk and no "
                  "voltage output");
    if (block_supported(p.N) && p.nchan > 1) {
      char* ws = (char*)workspace;
      int e = run_pipelined(p, voltages, dm, ws + lay.xt_off,
                            chan_intensity ? chan_intensity : (float*)(ws + lay.p_off),
                            (int32_t*)(ws + lay.d_off), ws + lay.h_off, volt_out, intensity,
                            coverage, chunks, npol, stream);
      if (e) return device_fail("pipelined launch", e);
      clear_error();
      return CDD_OK;
    }
    DmTile tile;
    tile.ndm = 1;
    tile.dm[0] = dm;
    s = run_tile(p, voltages, tile, nullptr, (char*)workspace, lay, chan_intensity, volt_out,
                 intensity, coverage, p.t_int, stream, true);
    if (s == CDD_OK) clear_error();
    return s;
  } catch (const std::bad_alloc&) {
    return fail(CDD_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
}

// Incoherent dedispersion: the arguments of cdd_dedisperse that matter
// without a transform (no length rule, so any DM is accepted).
static cdd_status incoherent_plan(int32_t dtype, int64_t nsamp, int32_t nchan, double f_centre,
                                  double bw, double dm, int32_t n_int, const cdd_opts* opts,
                                  BeamPlan* p) {
  if (dtype != CDD_CI8 && dtype != CDD_CF32)
    return fail(CDD_EINVAL, "dtype %d is not CDD_CI8 or CDD_CF32", dtype);
  if (nsamp < 1) return fail(CDD_EINVAL, "nsamp must be >= 1 (got %lld)", (long long)nsamp);
  if (nchan < 1 || nchan > 65535)
    return fail(CDD_EINVAL, "nchan must be in [1, 65535] (got %d)", nchan);
  if (n_int < 1 || n_int > nsamp)
    return fail(CDD_EINVAL, "n_int must be in [1, nsamp] (got %d)", n_int);
  if (!std::isfinite(f_centre) || !std::isfinite(bw) || !std::isfinite(dm))
    return fail(CDD_EINVAL, "frequencies and DM must be finite");
  if (!(bw > 0)) return fail(CDD_EINVAL, "bw must be > 0 (got %g)", bw);
  if (!(f_centre - bw / 2.0 > 0))
    return fail(CDD_EINVAL, "band must lie above 0 MHz (f_centre - bw/2 = %g)",
                f_centre - bw / 2.0);
  p->dtype = dtype;
  p->nsamp = nsamp;
  p->nchan = nchan;
  p->f_centre = f_centre;
  p->bw = bw;
  p->df = bw / nchan;
  p->f_lo = f_centre - bw / 2.0;
  p->n_int = n_int;
  p->dms.assign(1, dm);
  if (opts && opts->dm_const != 0) {
    if (!std::isfinite(opts->dm_const) || opts->dm_const <= 0)
      return fail(CDD_EINVAL, "dm_const must be finite and > 0");
    p->dconst = opts->dm_const;
  }
  p->t_int = nsamp / n_int;
  p->N = 0;  // no transform
  return CDD_OK;
}

extern "C" size_t cdd_incoherent_ws_bytes(int32_t dtype, int64_t nsamp, int32_t nchan,
                                          int32_t n_int) {
  BeamPlan p;
  if (incoherent_plan(dtype, nsamp, nchan, 325.0, 1.0, 0.0, n_int, nullptr, &p) != CDD_OK)
    return 0;
  clear_error();
  return ws_layout(p, 1, true).total;
}

extern "C" cdd_status cdd_incoherent(const void* voltages, int32_t dtype, int64_t nsamp,
                                     int32_t nchan, double f_centre_mhz, double bw_mhz,
                                     double dm, int32_t n_int, float* intensity,
                                     int32_t* coverage, float* chan_intensity,
                                     const cdd_opts* opts, void* workspace, size_t ws_bytes,
                                     void* stream) {
  try {
    if (!voltages) return fail(CDD_EINVAL, "voltages is NULL");
    if (!intensity) return fail(CDD_EINVAL, "intensity is NULL");
    BeamPlan p;
    cdd_status s = incoherent_plan(dtype, nsamp, nchan, f_centre_mhz, bw_mhz, dm, n_int, opts, &p);
    if (s != CDD_OK) return s;
    const WsLayout lay = ws_layout(p, 1, true);
    if (!workspace || ws_bytes < lay.total)
      return fail(CDD_EINVAL, "workspace too small: need %zu bytes, got %zu", lay.total,
                  workspace ? ws_bytes : (size_t)0);
    if (!aligned256(workspace)) return fail(CDD_EINVAL, "workspace must be 256-byte aligned");
    char* ws = (char*)workspace;
    const void* xt = voltages;
    int e = 0;
    if (p.nchan > 1) {
      if ((e = launch_transposed(p, voltages, ws + lay.xt_off, stream)))
        return device_fail("transpose launch", e);
      xt = ws + lay.xt_off;
    }
    float* P = chan_intensity ? chan_intensity : (float*)(ws + lay.p_off);
    int32_t* d = (int32_t*)(ws + lay.d_off);
    DmTile tile;
    tile.ndm = 1;
    tile.dm[0] = dm;
    void* tok = nullptr;
    if ((e = stage_begin(kStageDelays, stream, &tok)) || (e = launch_delays(p, tile, d, stream)) ||
        (e = stage_end(kStageDelays, stream, tok)))
      return device_fail("delay launch", e);
    if ((e = stage_begin(kStageBlock, stream, &tok)) || (e = launch_detect(p, xt, P, stream)) ||
        (e = stage_end(kStageBlock, stream, tok)))
      return device_fail("detect launch", e);
    if ((e = stage_begin(kStageDsum, stream, &tok)) ||
        (e = launch_dsum(p, 1, P, d, intensity, coverage, p.t_int, stream)) ||
        (e = stage_end(kStageDsum, stream, tok)))
      return device_fail("aligned-sum launch", e);
    clear_error();
    return CDD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CDD_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
}

extern "C" cdd_status cdd_fold(const float* intensity, int64_t t_int, double period,
                               double phase0, int32_t nbins, float* profile, int32_t* counts,
                               void* stream) {
  if (!intensity || !profile) return fail(CDD_EINVAL, "intensity or profile is NULL");
  if (t_int < 1) return fail(CDD_EINVAL, "t_int must be >= 1");
  if (nbins < 1) return fail(CDD_EINVAL, "nbins must be >= 1");
  if (!std::isfinite(period) || !std::isfinite(phase0) || !(period > 1.0))
    return fail(CDD_EINVAL, "period must be finite and > 1 sample, phase0 finite");
  const int e = launch_fold(intensity, t_int, period, phase0, nbins, profile, counts, stream);
  if (e) return device_fail("fold launch", e);
  clear_error();
  return CDD_OK;
}

cdd_status cdd_plan_create(const cdd_beam* beams, int32_t nbeam, const cdd_opts* opts,
                           cdd_plan** out) {
  try {
    if (!out) return fail(CDD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!beams || nbeam < 1) return fail(CDD_EINVAL, "no beams");
    cdd_plan* pl = new cdd_plan();
    for (int b = 0; b < nbeam; ++b) {
      const cdd_beam& d = beams[b];
      if (!d.voltages || !d.intensity) {
        delete pl;
        return fail(CDD_EINVAL, "beam %d: voltages or intensity is NULL", b);
      }
      BeamPlan p;
      int32_t fft_len = d.fft_len;
      int32_t tuned_tile = 0;
      cdd_opts o2 = opts ? *opts : cdd_opts{};
      if (opts && opts->autotune && fft_len == 0 && !opts->explicit_plan &&
          d.dtype == CDD_CI8 && d.host_dms && d.ndm > 0) {
        cdd_tune_result tr;
        cdd_status ts = cdd_autotune(d.dtype, d.nchan, d.f_centre_mhz, d.bw_mhz, d.host_dms,
                                     d.ndm, d.n_int, 0, 0, &tr);
        if (ts == CDD_OK) {
          fft_len = tr.fft_len;
          o2.kernel_variant = tr.kernel_variant;
          tuned_tile = tr.dm_tile;
        }
      }
      cdd_status s = make_plan(d.dtype, d.nsamp, d.nchan, d.f_centre_mhz, d.bw_mhz, d.host_dms,
                               d.ndm, fft_len, d.n_int, opts ? &o2 : nullptr, &p);
      if (s != CDD_OK) {
        std::string msg = cdd_last_error();
        delete pl;
        return fail(s, "beam %d: %s", b, msg.c_str());
      }
      if (!block_supported(p.N) && !large_supported(p.N)) {
        delete pl;
        return fail(CDD_ENOTSUP, "beam %d: fft_len %d is not supported", b, p.N);
      }
      p.dm_tile = tuned_tile;
      pl->beams.push_back(p);
      cdd_beam copy = d;
      copy.host_dms = nullptr;
      pl->desc.push_back(copy);
    }
    pl->chirp_in_kernel = (opts && opts->chirp_in_kernel) ? 1 : 0;
    pl->single_launch = (opts && opts->single_launch) ? 1 : 0;
    layout_plan(pl);
    *out = pl;
    clear_error();
    return CDD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CDD_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
}

cdd_status cdd_plan_info_get(const cdd_plan* plan, int32_t beam, cdd_plan_info* info) {
  if (!plan || !info) return fail(CDD_EINVAL, "plan or info is NULL");
  if (beam < 0 || beam >= (int)plan->beams.size())
    return fail(CDD_EINVAL, "beam %d out of range", beam);
  const BeamPlan& p = plan->beams[beam];
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
  info->ws_bytes = plan->ws;
  clear_error();
  return CDD_OK;
}

// Delays and aligned sums of beam b's tile of round r (and, for lengths above
// the block kernel's, its four-step transforms first), on `stream`.
// The tail of beam b's round r on the stream: the long transforms (lengths
// beyond the block kernels), the delays (unless already computed) and the
// aligned sums.
static cdd_status finish_beam(cdd_plan* plan, char* ws, size_t b, int r, const void* xt,
                              void* stream, bool delays_ready = false) {
  const BeamPlan& p = plan->beams[b];
  const cdd_beam& d = plan->desc[b];
  const int i0 = r * plan->tile[b];
  DmTile tile;
  tile.ndm = std::max(0, std::min(plan->tile[b], (int)p.dms.size() - i0));
  if (tile.ndm == 0) return CDD_OK;
  for (int i = 0; i < tile.ndm; ++i) tile.dm[i] = p.dms[i0 + i];
  char* wb = ws + plan->ws_base[b];
  const WsLayout& lay = plan->lay[b];
  float* P = (float*)(wb + lay.p_off);
  void* tok = nullptr;
  int e = 0;
  if (!block_supported(p.N)) {
    if ((e = stage_begin(kStageBlock, stream, &tok))) return device_fail("event record", e);
    for (int i = 0; i < tile.ndm; ++i)
      if ((e = launch_large(p, xt, tile.dm[i], wb + lay.s_off, (float*)(wb + lay.pb_off),
                            P + (int64_t)i * p.nchan * p.t_int, nullptr, stream)))
        return device_fail("long-transform launch", e);
    if ((e = stage_end(kStageBlock, stream, tok))) return device_fail("event record", e);
  }
  int32_t* dl = (int32_t*)(wb + lay.d_off);
  if (!delays_ready) {
    if ((e = stage_begin(kStageDelays, stream, &tok))) return device_fail("event record", e);
    if ((e = launch_delays(p, tile, dl, stream))) return device_fail("delay launch", e);
    if ((e = stage_end(kStageDelays, stream, tok))) return device_fail("event record", e);
  }
  if ((e = stage_begin(kStageDsum, stream, &tok))) return device_fail("event record", e);
  if ((e = launch_dsum(p, tile.ndm, P, dl, d.intensity + (int64_t)i0 * p.t_int,
                       d.coverage ? d.coverage + (int64_t)i0 * p.t_int : nullptr, p.t_int,
                       stream)))
    return device_fail("delay-sum launch", e);
  if ((e = stage_end(kStageDsum, stream, tok))) return device_fail("event record", e);
  return CDD_OK;
}

cdd_status cdd_plan_execute(cdd_plan* plan, void* workspace, size_t ws_bytes, void* stream) {
  try {
    if (!plan) return fail(CDD_EINVAL, "plan is NULL");
    if (!workspace || ws_bytes < plan->ws)
      return fail(CDD_EINVAL, "workspace too small: need %zu bytes", plan->ws);
    if (!aligned256(workspace)) return fail(CDD_EINVAL, "workspace must be 256-byte aligned");
    char* ws = (char*)workspace;
    const size_t nb = plan->beams.size();
    const size_t slot_bytes = align256(batch_table_bytes((int)nb));
    const size_t slots_per_round = std::max<size_t>(nb, kGroupKinds);
    int e = 0;
    if (!plan->host_tab) {
      hipError_t he = hipHostMalloc(&plan->host_tab, plan->host_tab_bytes);
      if (he != hipSuccess) {
        plan->host_tab = nullptr;
        return device_fail("pinned launch tables", (int)he);
      }
      std::memset(plan->host_tab, 0, plan->host_tab_bytes);
      if ((he = hipEventCreateWithFlags(&plan->tab_done, hipEventDisableTiming)) != hipSuccess)
        return device_fail("event create", (int)he);
    }
    std::vector<const void*> xt(nb, nullptr);
    std::vector<void*> H(nb, nullptr);
    for (size_t b = 0; b < nb; ++b) {
      const BeamPlan& p = plan->beams[b];
      xt[b] = p.nchan > 1 ? (const void*)(ws + plan->ws_base[b] + plan->lay[b].xt_off)
                          : plan->desc[b].voltages;
      if (table_chirp(plan, p)) H[b] = ws + plan->ws_base[b] + plan->lay[b].h_off;
    }
    auto tile_of = [&](size_t b, int r, BatchBeam* bb) {
      const BeamPlan& p = plan->beams[b];
      const int i0 = r * plan->tile[b];
      const int ndm = std::max(0, std::min(plan->tile[b], (int)p.dms.size() - i0));
      bb->p = &p;
      bb->xt = xt[b];
      bb->dms.ndm = ndm;
      for (int i = 0; i < ndm; ++i) bb->dms.dm[i] = p.dms[i0 + i];
      bb->P = (float*)(ws + plan->ws_base[b] + plan->lay[b].p_off);
      bb->co = offline_coords(p);
      return ndm;
    };
    // Every block-kernel launch of the execute with its argument table, formed
    // on the host first.  Pipelined form (default): one launch per beam and
    // round, the specialised kernel of the beam's length.  Single-launch form:
    // per round, every beam of length <= 8192 and one sample type in one
    // persistent launch, the 16384-point beams in one more per kind.
    struct Launch {
      LaunchDesc d;
      size_t slot = 0;
      int round = 0;
      size_t beam = 0;   // pipelined form
      bool direct = false;  // one beam, one DM: the one-shot block kernel
      BatchBeam bb;
      const void* h = nullptr;
    };
    std::vector<Launch> launches;
    std::vector<char> staged(plan->host_tab_bytes, 0);
    // beams in the order their inputs are ready: shortest layout change first
    std::vector<size_t> order(nb);
    for (size_t b = 0; b < nb; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
      auto bytes = [&](size_t b) {
        const BeamPlan& p = plan->beams[b];
        return p.nchan > 1 ? (double)p.nchan * p.nsamp * (p.dtype == CDD_CI8 ? 2 : 8) : 0.0;
      };
      return bytes(x) < bytes(y);
    });
    for (int r = 0; r < plan->rounds; ++r) {
      if (!plan->single_launch) {
        for (size_t j = 0; j < nb; ++j) {
          const size_t b = order[j];
          BatchBeam bb;
          if (!block_supported(plan->beams[b].N) || tile_of(b, r, &bb) == 0) continue;
          Launch L;
          L.round = r;
          L.beam = b;
          L.slot = slot_bytes * ((size_t)r * slots_per_round + j);
          const void* h = H[b];
          if (h) {
            // a beam with its chirp table: the one-shot call's own kernel,
            // its arguments passed by value
            L.direct = true;
            L.bb = bb;
            L.h = h;
          } else if ((e = prepare_launch(kLaunchBatch, &bb, &h, 1, staged.data() + L.slot,
                                         &L.d))) {
            return device_fail("launch table", e);
          }
          launches.push_back(L);
        }
        continue;
      }
      std::vector<BatchBeam> group[kGroupKinds];
      std::vector<const void*> gh[kGroupKinds];
      // when every beam of a sample type shares one length and one chirp
      // form, that length's own kernel takes them all; otherwise the mixed
      // kernel does (one launch either way)
      int len[2] = {0, 0}, form[2] = {0, 0};
      for (size_t b = 0; b < nb; ++b) {
        const BeamPlan& p = plan->beams[b];
        BatchBeam bb;
        if (!block_supported(p.N) || tile_of(b, r, &bb) == 0) continue;
        const int t = p.dtype == CDD_CI8 ? 0 : 1, f = H[b] ? 1 : 2;
        len[t] = len[t] == 0 ? p.N : (len[t] == p.N ? len[t] : -1);
        form[t] = form[t] == 0 ? f : (form[t] == f ? f : -1);
      }
      for (size_t b = 0; b < nb; ++b) {
        const BeamPlan& p = plan->beams[b];
        BatchBeam bb;
        if (!block_supported(p.N) || tile_of(b, r, &bb) == 0) continue;
        const int t = p.dtype == CDD_CI8 ? 0 : 1;
        const bool uniform = len[t] == p.N && form[t] > 0;
        const int kind = (mixed_supported(p.N) && !uniform)
                             ? kLaunchMixed
                             : (H[b] ? kLaunchTables : kLaunchBatch);
        const int k = kind * 2 + (p.dtype == CDD_CI8 ? 0 : 1);
        group[k].push_back(bb);
        gh[k].push_back(H[b]);
      }
      for (int k = 0; k < kGroupKinds; ++k) {
        if (group[k].empty()) continue;
        Launch L;
        L.round = r;
        L.slot = slot_bytes * ((size_t)r * slots_per_round + k);
        if ((e = prepare_launch(k / 2, group[k].data(), gh[k].data(), (int)group[k].size(),
                                staged.data() + L.slot, &L.d)))
          return device_fail("launch table", e);
        launches.push_back(L);
      }
    }
    // Publish the tables into the pinned buffer if they changed; a rewrite
    // first waits for the previous execute's copies out of it.
    if (std::memcmp(plan->host_tab, staged.data(), plan->host_tab_bytes) != 0) {
      if (plan->tab_pending) {
        hipError_t he = hipEventSynchronize(plan->tab_done);
        if (he != hipSuccess) return device_fail("launch table wait", (int)he);
      }
      std::memcpy(plan->host_tab, staged.data(), plan->host_tab_bytes);
    }
    unsigned int* counter = (unsigned int*)(ws + plan->cnt_off);  // launches share one stream
    auto enqueue = [&](const Launch& L) -> cdd_status {
      void* tok = nullptr;
      int err = 0;
      if ((err = stage_begin(kStageBlock, stream, &tok))) return device_fail("event record", err);
      if (L.direct)
        err = launch_block_co(*L.bb.p, L.bb.co, L.bb.xt, L.bb.dms, L.bb.P, nullptr, L.h, stream);
      else
        err = enqueue_launch(L.d, (char*)plan->host_tab + L.slot, ws + plan->tab_off + L.slot,
                             counter, stream);
      if (err) return device_fail("batched launch", err);
      if ((err = stage_end(kStageBlock, stream, tok))) return device_fail("event record", err);
      return CDD_OK;
    };
    // Round 0.  A one-DM beam whose layout change can carry them has its
    // chirp table and delays built by that kernel; the tables and first-tile
    // delays of the other beams are built on the auxiliary stream while the
    // caller's stream changes the layout of the first beam (the auxiliary
    // stream is not used at all when there are none).  In the pipelined form
    // each beam then takes its layout change, its launches and its aligned
    // sums in turn on the caller's stream (running the layout changes of
    // later beams beside the transforms of earlier ones slows both down on
    // this GPU as much as it hides); the single-launch form changes every
    // layout first.
    auto fused = [&](size_t b) { return H[b] && transpose_chirp_fits(plan->beams[b]); };
    auto d_of = [&](size_t b) { return (int32_t*)(ws + plan->ws_base[b] + plan->lay[b].d_off); };
    bool use_aux = false;
    for (size_t b = 0; b < nb; ++b) use_aux = use_aux || !fused(b);
    AuxSession aux;
    if (use_aux && (e = aux_open(stream, &aux))) return device_fail("auxiliary stream", e);
    size_t li = 0;
    cdd_status st = CDD_OK;
    bool aux_waited = !use_aux;
    for (size_t j = 0; j < nb && st == CDD_OK; ++j) {
      const size_t b = order[j];
      const BeamPlan& p = plan->beams[b];
      if (fused(b)) continue;
      DmTile t0;
      t0.ndm = std::min(plan->tile[b], (int)p.dms.size());
      for (int i = 0; i < t0.ndm; ++i) t0.dm[i] = p.dms[i];
      int err = 0;
      void* tok = nullptr;
      if ((err = stage_begin(kStageDelays, aux.aux, &tok)) ||
          (H[b] && (err = launch_chirp_table(p, p.dms[0], H[b], aux.aux))) ||
          (err = launch_delays(p, t0, d_of(b), aux.aux)) ||
          (err = stage_end(kStageDelays, aux.aux, tok)))
        st = device_fail("chirp table or delay launch", err);
    }
    for (size_t j = 0; j < nb && st == CDD_OK; ++j) {
      const size_t b = order[j];
      const BeamPlan& p = plan->beams[b];
      int err = 0;
      if (p.nchan > 1 &&
          (err = launch_transposed(p, plan->desc[b].voltages, (void*)xt[b], stream,
                                   fused(b) ? H[b] : nullptr, p.dms[0],
                                   fused(b) ? d_of(b) : nullptr))) {
        st = device_fail("transpose launch", err);
        break;
      }
      if (plan->single_launch) continue;
      if (!aux_waited) {
        if ((err = aux_mark(&aux, stream))) {
          st = device_fail("stream wait", err);
          break;
        }
        aux_waited = true;
      }
      while (st == CDD_OK && li < launches.size() && launches[li].round == 0 &&
             launches[li].beam == b)
        st = enqueue(launches[li++]);
      if (st == CDD_OK) st = finish_beam(plan, ws, b, 0, xt[b], stream, true);
    }
    const int ce = use_aux ? aux_close(stream, &aux) : 0;
    if (st != CDD_OK) return st;
    if (ce) return device_fail("auxiliary stream", ce);
    for (int r = plan->single_launch ? 0 : 1; r < plan->rounds; ++r) {
      while (li < launches.size() && launches[li].round == r)
        if ((st = enqueue(launches[li++])) != CDD_OK) return st;
      for (size_t j = 0; j < nb; ++j)  // round 0: delays already computed (see above)
        if ((st = finish_beam(plan, ws, order[j], r, xt[order[j]], stream, r == 0)) != CDD_OK)
          return st;
    }
    hipError_t he = hipEventRecord(plan->tab_done, (hipStream_t)stream);
    if (he != hipSuccess) return device_fail("event record", (int)he);
    plan->tab_pending = true;
    clear_error();
    return CDD_OK;
  } catch (const std::bad_alloc&) {
    return fail(CDD_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
}

void cdd_plan_destroy(cdd_plan* plan) { delete plan; }

}  // extern "C"
