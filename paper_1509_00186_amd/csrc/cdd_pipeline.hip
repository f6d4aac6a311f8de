// One-shot path with the memory-bound stages overlapped with compute.
//
// The layout change runs on an auxiliary HIP stream while the caller's stream
// builds the chirp table and the channel delays.  With several time chunks
// the auxiliary stream also changes the layout of chunk i+1 while the
// caller's stream transforms chunk i, and sums every output range whose
// delayed inputs are complete as soon as they are.  Events order the two
// streams, and the caller's stream waits for the auxiliary one at the end, so
// the call stays asynchronous and stream-ordered.  (Each chunk boundary costs
// a partly filled last round of workgroups and the overlapped kernels slow
// the block kernel down, so one chunk is the default.)
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "cdd_internal.h"

namespace cdd {

namespace {
constexpr int kEvents = 64;
static_assert(kEvents >= 2 * kMaxChunks + 3, "one call takes 2 C + 3 events");

// Blocks of the first time chunk = nblocks / kFirstDiv (rounded up): its
// layout change is the only one not hidden behind block work, and the layout
// change of a block column is about four times faster than its transforms.
constexpr int64_t kFirstDiv = 5;
// Consecutive chunks alternate between the caller's stream and a second
// compute stream, so one chunk's last workgroups overlap the next chunk's
// first ones instead of draining the machine at every chunk boundary.
constexpr bool kTwoCompute = true;

struct Aux {
  hipStream_t s = nullptr;   // layout changes and aligned sums
  hipStream_t s2 = nullptr;  // every other block chunk
  hipEvent_t ev[kEvents];
  int next = 0;
};
std::mutex g_aux_mu;
std::map<int, Aux> g_aux;

hipEvent_t take(Aux& a) {
  hipEvent_t e = a.ev[a.next];
  a.next = (a.next + 1) % kEvents;
  return e;
}
}  // namespace

// Library-owned auxiliary streams and events of the current device.
static int aux_of(Aux** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  Aux& ax = g_aux[dev];
  if (!ax.s) {
    if ((e = hipStreamCreateWithFlags(&ax.s, hipStreamNonBlocking)) != hipSuccess) return (int)e;
    if ((e = hipStreamCreateWithFlags(&ax.s2, hipStreamNonBlocking)) != hipSuccess) return (int)e;
    for (int i = 0; i < kEvents; ++i)
      if ((e = hipEventCreateWithFlags(&ax.ev[i], hipEventDisableTiming)) != hipSuccess)
        return (int)e;
  }
  *out = &ax;
  return 0;
}

// One chunk: the layout change, the block kernel and the aligned sum run in
// order on the caller's stream.  For int8 records with at least one layout
// workgroup per channel the layout-change kernel also builds the chirp table
// and the channel delays, so the call is those three kernels on one stream
// and nothing else; otherwise the table and the delays run beside the
// layout change on the auxiliary stream, which the caller's stream waits
// for before the block kernel.
static int run_single(Aux& ax, const BeamPlan& p, const void* voltages, double dm, char* xt,
                      float* P, int32_t* d, void* H, void* volt_out, float* I, int32_t* cov,
                      int npol, hipStream_t S) {
  hipStream_t A = ax.s;
  hipError_t e;
  int err = 0;
  void* tok = nullptr;
  DmTile tile;
  tile.ndm = 1;
  tile.dm[0] = dm;
  const bool fused = H != nullptr && transpose_chirp_fits(p);
  hipEvent_t eA = nullptr;
  if (!fused) {
    // fork after the caller's earlier work (a previous call may still read H)
    hipEvent_t e0 = take(ax);
    if ((e = hipEventRecord(e0, S)) != hipSuccess) return (int)e;
    if ((e = hipStreamWaitEvent(A, e0, 0)) != hipSuccess) return (int)e;
    if ((err = stage_begin(kStageDelays, A, &tok))) return err;
    if (H && (err = launch_chirp_table(p, dm, H, A))) return err;
    if ((err = launch_delays(p, tile, d, A))) return err;
    if ((err = stage_end(kStageDelays, A, tok))) return err;
    eA = take(ax);
    if ((e = hipEventRecord(eA, A)) != hipSuccess) return (int)e;
  }
  // polarisation records back to back; the second adds its intensities
  const size_t rec = (size_t)p.nsamp * p.nchan * (p.dtype == CDD_CI8 ? 2 : 8);
  Coords co = offline_coords(p);
  for (int pol = 0; pol < npol; ++pol) {
    if ((err = stage_begin(kStageTranspose, S, &tok))) return err;
    if (pol == 0 && fused)
      err = launch_transpose_chirp(p, voltages, xt, dm, H, S, d);
    else
      err = launch_transpose((const char*)voltages + pol * rec, xt, p.dtype, p.nsamp, p.nchan,
                             xt_stride(p), S);
    if (err) return err;
    if ((err = stage_end(kStageTranspose, S, tok))) return err;
    if (pol == 0 && eA && (e = hipStreamWaitEvent(S, eA, 0)) != hipSuccess) return (int)e;
    co.accum = pol > 0;
    if ((err = stage_begin(kStageBlock, S, &tok))) return err;
    if ((err = launch_block_co(p, co, xt, tile, P, volt_out, H, S))) return err;
    if ((err = stage_end(kStageBlock, S, tok))) return err;
  }
  if ((err = stage_begin(kStageDsum, S, &tok))) return err;
  if ((err = launch_dsum(p, 1, P, d, I, cov, p.t_int, S))) return err;
  return stage_end(kStageDsum, S, tok);
}

int fork_join(void* stream, const std::function<int(void*)>& aux_work,
              const std::function<int(void*)>& main_work) {
  std::lock_guard<std::mutex> lk(g_aux_mu);
  Aux* axp = nullptr;
  int err = aux_of(&axp);
  if (err) return err;
  Aux& ax = *axp;
  hipStream_t S = (hipStream_t)stream, A = ax.s;
  hipError_t e;
  hipEvent_t e0 = take(ax);
  if ((e = hipEventRecord(e0, S)) != hipSuccess) return (int)e;
  if ((e = hipStreamWaitEvent(A, e0, 0)) != hipSuccess) return (int)e;
  if ((err = aux_work((void*)A))) return err;
  hipEvent_t eA = take(ax);
  if ((e = hipEventRecord(eA, A)) != hipSuccess) return (int)e;
  if ((err = main_work((void*)S))) return err;
  if ((e = hipStreamWaitEvent(S, eA, 0)) != hipSuccess) return (int)e;
  return 0;
}

int aux_open(void* stream, AuxSession* session) {
  session->lk = std::unique_lock<std::mutex>(g_aux_mu);
  Aux* axp = nullptr;
  int err = aux_of(&axp);
  if (err) {
    session->lk.unlock();
    return err;
  }
  session->impl = axp;
  session->aux = (void*)axp->s;
  hipEvent_t e0 = take(*axp);
  hipError_t e = hipEventRecord(e0, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(axp->s, e0, 0);
  return (int)e;
}

int aux_mark(AuxSession* session, void* waiting) {
  Aux& ax = *(Aux*)session->impl;
  hipEvent_t ev = take(ax);
  hipError_t e = hipEventRecord(ev, ax.s);
  if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)waiting, ev, 0);
  return (int)e;
}

int aux_after(AuxSession* session, void* stream) {
  Aux& ax = *(Aux*)session->impl;
  hipEvent_t ev = take(ax);
  hipError_t e = hipEventRecord(ev, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(ax.s, ev, 0);
  return (int)e;
}

int aux_close(void* stream, AuxSession* session) {
  int err = session->impl ? aux_mark(session, stream) : 0;
  session->impl = nullptr;
  session->aux = nullptr;
  if (session->lk.owns_lock()) session->lk.unlock();
  return err;
}

int run_pipelined(const BeamPlan& p, const void* voltages, double dm, char* xt, float* P,
                  int32_t* d, void* H, void* volt_out, float* I, int32_t* cov, int chunks,
                  int npol, void* stream) {
  std::lock_guard<std::mutex> lk(g_aux_mu);
  Aux* axp = nullptr;
  int aerr = aux_of(&axp);
  if (aerr) return aerr;
  Aux& ax = *axp;
  hipError_t e = hipSuccess;
  if (chunks <= 1)
    return run_single(ax, p, voltages, dm, xt, P, d, H, volt_out, I, cov, npol,
                      (hipStream_t)stream);
  if (npol != 1) return (int)hipErrorInvalidValue;
  hipStream_t S = (hipStream_t)stream, A = ax.s, S2 = ax.s2;
  const size_t elem = p.dtype == CDD_CI8 ? 2 : 8;
  const int C = chunks;
  std::vector<int64_t> kb(C + 1), tr(C + 1);
  kb[0] = 0;
  if (C >= 2) {
    kb[1] = std::max<int64_t>(1, (p.nblocks + kFirstDiv - 1) / kFirstDiv);
    for (int i = 2; i <= C; ++i) kb[i] = kb[1] + (p.nblocks - kb[1]) * (i - 1) / (C - 1);
  }
  kb[C] = p.nblocks;
  tr[0] = 0;
  for (int i = 1; i <= C; ++i)
    tr[i] = std::max(tr[i - 1],
                     std::min<int64_t>(p.nsamp, kb[i] * p.M - p.nfront + p.N));
  tr[C] = p.nsamp;
  DmTile tile;
  tile.ndm = 1;
  tile.dm[0] = dm;
  // fork: the auxiliary stream starts after everything already on the caller's
  hipEvent_t e0 = take(ax);
  if ((e = hipEventRecord(e0, S)) != hipSuccess) return (int)e;
  if ((e = hipStreamWaitEvent(A, e0, 0)) != hipSuccess) return (int)e;
  const bool two = kTwoCompute && C >= 2;
  if (two && (e = hipStreamWaitEvent(S2, e0, 0)) != hipSuccess) return (int)e;
  int err = 0;
  void* tok = nullptr;
  if ((err = stage_begin(kStageDelays, S, &tok))) return err;
  if ((err = launch_delays(p, tile, d, S))) return err;
  if ((err = launch_chirp_table(p, dm, H, S))) return err;
  if ((err = stage_end(kStageDelays, S, tok))) return err;
  std::vector<hipEvent_t> evT(C), evB(C);
  for (int i = 0; i < C; ++i) {
    const int64_t rows = tr[i + 1] - tr[i];
    if (rows > 0) {
      if ((err = stage_begin(kStageTranspose, A, &tok))) return err;
      if ((err = launch_transpose((const char*)voltages + tr[i] * p.nchan * elem,
                                  xt + tr[i] * elem, p.dtype, rows, p.nchan, xt_stride(p),
                                  A)))
        return err;
      if ((err = stage_end(kStageTranspose, A, tok))) return err;
    }
    evT[i] = take(ax);
    if ((e = hipEventRecord(evT[i], A)) != hipSuccess) return (int)e;
  }
  // compute: chunk i of blocks once its rows are in place
  const Coords full = offline_coords(p);
  // the chirp table and delays (on S) come before every chunk
  hipEvent_t eS = nullptr;
  if (two) {
    eS = take(ax);
    if ((e = hipEventRecord(eS, S)) != hipSuccess) return (int)e;
    if ((e = hipStreamWaitEvent(S2, eS, 0)) != hipSuccess) return (int)e;
  }
  for (int i = 0; i < C; ++i) {
    hipStream_t Q = (two && (i & 1)) ? S2 : S;
    if ((e = hipStreamWaitEvent(Q, evT[i], 0)) != hipSuccess) return (int)e;
    const int64_t k0 = kb[i], nb = kb[i + 1] - kb[i];
    if (nb > 0) {
      Coords co = full;
      co.load_off = p.nfront - k0 * p.M;
      const int64_t u0 = k0 * (p.M / p.n_int);
      co.u_lim = p.t_int - u0;
      co.o_lim = p.nsamp - k0 * p.M;
      co.nblocks = nb;
      if ((err = stage_begin(kStageBlock, Q, &tok))) return err;
      if ((err = launch_block_co(p, co, xt, tile, P + u0,
                                 volt_out ? (char*)volt_out + k0 * p.M * 8 : nullptr, H, Q)))
        return err;
      if ((err = stage_end(kStageBlock, Q, tok))) return err;
    }
    evB[i] = take(ax);
    if ((e = hipEventRecord(evB[i], Q)) != hipSuccess) return (int)e;
  }
  // the caller's stream continues after every chunk (those on S2 included)
  if (two)
    for (int i = 1; i < C; i += 2)
      if ((e = hipStreamWaitEvent(S, evB[i], 0)) != hipSuccess) return (int)e;
  // aligned sums: u is final once every channel's P[u + d_c] is computed;
  // the last range runs on the caller's stream, right after the last chunk
  int64_t u_done = 0;
  for (int i = 0; i < C; ++i) {
    const bool last = i == C - 1;
    hipStream_t Q = last ? S : A;
    if (!last && (e = hipStreamWaitEvent(A, evB[i], 0)) != hipSuccess) return (int)e;
    int64_t upto = last ? p.t_int
                        : std::min<int64_t>(p.t_int, kb[i + 1] * (p.M / p.n_int) - p.d_max);
    if (upto > u_done) {
      if ((err = stage_begin(kStageDsum, Q, &tok))) return err;
      if ((err = launch_dsum_range(p.nchan, 1, P, p.t_int, (int64_t)p.nchan * p.t_int, p.t_int,
                                   u_done, upto - u_done, d, I + u_done,
                                   cov ? cov + u_done : nullptr, p.t_int, Q)))
        return err;
      if ((err = stage_end(kStageDsum, Q, tok))) return err;
      u_done = upto;
    }
  }
  // join
  hipEvent_t eA = take(ax);
  if ((e = hipEventRecord(eA, A)) != hipSuccess) return (int)e;
  if ((e = hipStreamWaitEvent(S, eA, 0)) != hipSuccess) return (int)e;
  return 0;
}

}  // namespace cdd
