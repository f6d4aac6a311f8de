// C-ABI entry points: one-shot dedispersion and batched plans.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "cdd_internal.h"

using namespace cdd;

namespace {

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

cdd_status device_fail(const char* what, int err) {
  return fail(CDD_EDEVICE, "%s: %s", what, hip_error_string(err));
}

// Layout change with stage timing.
int launch_transposed(const BeamPlan& p, const void* in, void* out, void* stream) {
  void* tok = nullptr;
  int e = stage_begin(stream, &tok);
  if (e) return e;
  if ((e = launch_transpose(in, out, p.dtype, p.nsamp, p.nchan, stream))) return e;
  return stage_end(kStageTranspose, stream, tok);
}

// Run the path for one beam and one tile of DM trials.
cdd_status run_tile(const BeamPlan& p, const void* voltages, const DmTile& tile,
                    const void* xt_ready, char* ws, const WsLayout& lay, float* chan_P,
                    void* volt_out, float* intensity, int32_t* coverage, int64_t out_stride,
                    void* stream) {
  const void* xt = xt_ready;
  void* tok = nullptr;
  int e = 0;
  if (xt == nullptr) {
    if (p.nchan > 1) {
      if ((e = launch_transposed(p, voltages, ws + lay.xt_off, stream))) return device_fail("transpose launch", e);
      xt = ws + lay.xt_off;
    } else {
      xt = voltages;
    }
  }
  float* P = chan_P ? chan_P : (float*)(ws + lay.p_off);
  int32_t* d = (int32_t*)(ws + lay.d_off);
  if ((e = stage_begin(stream, &tok))) return device_fail("event record", e);
  if ((e = launch_delays(p, tile, d, stream))) return device_fail("delay launch", e);
  if ((e = stage_end(kStageDelays, stream, tok))) return device_fail("event record", e);
  if ((e = stage_begin(stream, &tok))) return device_fail("event record", e);
  if (block_supported(p.N)) {
    if ((e = launch_block(p, xt, tile, P, volt_out, stream)))
      return device_fail("block kernel launch", e);
  } else {
    // long transforms: one DM trial at a time through the four-step kernels
    for (int i = 0; i < tile.ndm; ++i) {
      if ((e = launch_large(p, xt, tile.dm[i], ws + lay.s_off, (float*)(ws + lay.pb_off),
                            P + (int64_t)i * p.nchan * p.t_int, tile.ndm == 1 ? volt_out : nullptr,
                            stream)))
        return device_fail("long-transform launch", e);
    }
  }
  if ((e = stage_end(kStageBlock, stream, tok))) return device_fail("event record", e);
  if ((e = stage_begin(stream, &tok))) return device_fail("event record", e);
  if ((e = launch_dsum(p, tile.ndm, P, d, intensity, coverage, out_stride, stream)))
    return device_fail("delay-sum launch", e);
  if ((e = stage_end(kStageDsum, stream, tok))) return device_fail("event record", e);
  return CDD_OK;
}

}  // namespace

struct cdd_plan {
  std::vector<BeamPlan> beams;
  std::vector<cdd_beam> desc;
  size_t ws = 0;
};

extern "C" {

cdd_status cdd_dedisperse(const void* voltages, int32_t dtype, int64_t nsamp, int32_t nchan,
                          double f_centre_mhz, double bw_mhz, double dm, int32_t fft_len,
                          int32_t n_int, float* intensity, int32_t* coverage,
                          float* chan_intensity, void* volt_out, const cdd_opts* opts,
                          void* workspace, size_t ws_bytes, void* stream) {
  try {
    if (!voltages) return fail(CDD_EINVAL, "voltages is NULL");
    if (!intensity) return fail(CDD_EINVAL, "intensity is NULL");
    BeamPlan p;
    cdd_status s = make_plan(dtype, nsamp, nchan, f_centre_mhz, bw_mhz, &dm, 1, fft_len, n_int,
                             opts, &p);
    if (s != CDD_OK) return s;
    if (!block_supported(p.N) && !large_supported(p.N))
      return fail(CDD_ENOTSUP, "fft_len %d is not supported by this build", p.N);
    WsLayout lay = ws_layout(p, 1, true);
    if (!workspace || ws_bytes < lay.total)
      return fail(CDD_EINVAL, "workspace too small: need %zu bytes, got %zu", lay.total,
                  workspace ? ws_bytes : (size_t)0);
    if (!aligned256(workspace)) return fail(CDD_EINVAL, "workspace must be 256-byte aligned");
    DmTile tile;
    tile.ndm = 1;
    tile.dm[0] = dm;
    s = run_tile(p, voltages, tile, nullptr, (char*)workspace, lay, chan_intensity, volt_out,
                 intensity, coverage, p.t_int, stream);
    if (s == CDD_OK) clear_error();
    return s;
  } catch (const std::bad_alloc&) {
    return fail(CDD_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
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
      cdd_status s = make_plan(d.dtype, d.nsamp, d.nchan, d.f_centre_mhz, d.bw_mhz, d.host_dms,
                               d.ndm, d.fft_len, d.n_int, opts, &p);
      if (s != CDD_OK) {
        std::string msg = cdd_last_error();
        delete pl;
        return fail(s, "beam %d: %s", b, msg.c_str());
      }
      if (!block_supported(p.N) && !large_supported(p.N)) {
        delete pl;
        return fail(CDD_ENOTSUP, "beam %d: fft_len %d is not supported", b, p.N);
      }
      int tile = std::min<int>((int)p.dms.size(), kMaxDmTile);
      pl->ws = std::max(pl->ws, ws_layout(p, tile, true).total);
      pl->beams.push_back(p);
      cdd_beam copy = d;
      copy.host_dms = nullptr;
      pl->desc.push_back(copy);
    }
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

cdd_status cdd_plan_execute(cdd_plan* plan, void* workspace, size_t ws_bytes, void* stream) {
  try {
    if (!plan) return fail(CDD_EINVAL, "plan is NULL");
    if (!workspace || ws_bytes < plan->ws)
      return fail(CDD_EINVAL, "workspace too small: need %zu bytes", plan->ws);
    if (!aligned256(workspace)) return fail(CDD_EINVAL, "workspace must be 256-byte aligned");
    char* ws = (char*)workspace;
    for (size_t b = 0; b < plan->beams.size(); ++b) {
      const BeamPlan& p = plan->beams[b];
      const cdd_beam& d = plan->desc[b];
      const int ndm = (int)p.dms.size();
      const int tmax = std::min(ndm, kMaxDmTile);
      WsLayout lay = ws_layout(p, tmax, true);
      const void* xt = nullptr;
      if (p.nchan > 1) {
        int e = launch_transposed(p, d.voltages, ws + lay.xt_off, stream);
        if (e) return device_fail("transpose launch", e);
        xt = ws + lay.xt_off;
      } else {
        xt = d.voltages;
      }
      for (int i0 = 0; i0 < ndm; i0 += kMaxDmTile) {
        DmTile tile;
        tile.ndm = std::min(kMaxDmTile, ndm - i0);
        for (int i = 0; i < tile.ndm; ++i) tile.dm[i] = p.dms[i0 + i];
        cdd_status s = run_tile(p, d.voltages, tile, xt, ws, lay, nullptr, nullptr,
                                d.intensity + (int64_t)i0 * p.t_int,
                                d.coverage ? d.coverage + (int64_t)i0 * p.t_int : nullptr,
                                p.t_int, stream);
        if (s != CDD_OK) return s;
      }
    }
    clear_error();
    return CDD_OK;
  } catch (...) {
    return fail(CDD_EINTERNAL, "unexpected exception");
  }
}

void cdd_plan_destroy(cdd_plan* plan) { delete plan; }

}  // extern "C"
