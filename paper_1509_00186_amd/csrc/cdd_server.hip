// Real-time serving: streams of voltage blocks, continuous batching.
//
// Per stream, device memory holds
//   pend[2]  channel-major input samples [pbase, E) (ping-pong for compaction):
//            the overlap tail of the previous blocks plus newly arrived data;
//            the block grid is anchored at absolute sample 0, so the output
//            equals the whole-record computation (the first block sees zeros
//            before sample 0, as offline);
//   Pb[2]    per-channel intensities [ubase, U) still needed by the aligned
//            sum (the dispersion sweep d_max plus one batch);
//   d        channel delays; Iout staging for finished I[u];
//   slots    device staging for pushed blocks (time-major).
// A scheduler thread forms batches: every stream with consumed data gets its
// complete overlap-save blocks folded into one persistent launch (every
// transform length up to 8192 together, one launch per longer length);
// aligned sums and copies to the host follow on the same
// HIP stream.  Pushes copy into pinned slots and start the host-to-device
// copy on a second HIP stream; the compute stream waits on its event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "cdd_internal.h"
#include "cdd_sched.h"

namespace cdd {
namespace {

constexpr int kBatchRing = 4;  // batches in flight at once
constexpr int kMaxGroups = 16;  // transform lengths per batch (one counter each)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

enum SlotState { FREE = 0, PUSHED = 1, TAKEN = 2 };

struct Slot {
  void* host = nullptr;  // pinned
  void* dev = nullptr;
  int64_t nsamp = 0;
  uint64_t seq = 0;
  int64_t zeros = 0;  // lost samples to insert (as zeros) before this block
  double t_arrive = 0;
  hipEvent_t h2d = nullptr;
  SlotState state = FREE;
};

struct Stream {
  int id = -1;
  bool closing = false, flushed = false, released = false, releasing = false;
  BeamPlan p;
  StreamGeom g;
  Timeline tl;
  int64_t max_block = 0;
  int64_t block_len = 0;    // declared length of every push but the last (0: any)
  bool short_seen = false;  // a push shorter than block_len (must be the last)
  size_t elem = 2;
  char* pend[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t cap = 0;
  float* Pb[2] = {nullptr, nullptr};
  int pcur = 0;
  int64_t pcap = 0;
  int32_t* d = nullptr;
  float* Iout = nullptr;
  int64_t icap = 0;
  float* Ihost = nullptr;  // pinned, icap floats per batch ring entry
  std::vector<Slot> slots;
  size_t bytes = 0;
  // host results
  std::deque<float> ready;
  int64_t ready_first = 0;
  int64_t polled = 0;
  int64_t total_int = -1;  // set at close: E / n_int
};

struct BatchRec {
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<std::pair<int, std::pair<int64_t, int64_t>>> outs;  // stream, (u_first, count)
  std::vector<std::pair<int, int>> slots;                          // stream, slot index
  std::vector<double> arrivals;
  void* tab_dev = nullptr;
  unsigned int* counter = nullptr;
  std::vector<std::vector<char>> host_tabs;
  std::vector<float*> host_outs;
};

}  // namespace
}  // namespace cdd

struct cdd_server {
  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
  int device = 0;
  hipStream_t compute = nullptr, h2d = nullptr;
  size_t budget = 0, used = 0;
  int max_streams = 64, depth = 4;
  std::map<int, std::unique_ptr<cdd::Stream>> streams;
  int next_id = 0;
  cdd::BatchRec ring[cdd::kBatchRing];
  int ring_next = 0;
  std::vector<double> lat;
  cdd_server_stats st{};
  double t_first = -1, t_last = 0;
  int pending_work = 0;  // pushed blocks not yet completed
  std::string thread_error;
};

namespace cdd {
namespace {

hipError_t free_stream_mem(Stream* s) {
  for (int i = 0; i < 2; ++i) {
    if (s->pend[i]) (void)hipFree(s->pend[i]);
    if (s->Pb[i]) (void)hipFree(s->Pb[i]);
    s->pend[i] = nullptr;
    s->Pb[i] = nullptr;
  }
  if (s->d) (void)hipFree(s->d);
  if (s->Iout) (void)hipFree(s->Iout);
  if (s->Ihost) (void)hipHostFree(s->Ihost);
  s->d = nullptr;
  s->Iout = nullptr;
  s->Ihost = nullptr;
  for (auto& sl : s->slots) {
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.h2d) (void)hipEventDestroy(sl.h2d);
    sl.host = sl.dev = nullptr;
    sl.h2d = nullptr;
  }
  return hipSuccess;
}

// Issue the work of one batch on the compute stream (scheduler thread, lock
// held for the host-side bookkeeping).
int issue_batch(cdd_server* sv, BatchRec& br) {
  int e = 0;
  hipStream_t cs = sv->compute;
  struct Work {
    Stream* s;
    int64_t nproc;
    int64_t u_fin;
  };
  std::vector<Work> work;
  // 1. append consumed slots to each stream's pending input
  for (auto& kv : sv->streams) {
    Stream* s = kv.second.get();
    if (s->released || s->flushed) continue;
    bool any = false;
    Timeline& tl = s->tl;
    while (true) {
      // consume in sequence order, as far as the pending buffer has room
      int best = -1;
      for (size_t q = 0; q < s->slots.size(); ++q)
        if (s->slots[q].state == PUSHED && (best < 0 || s->slots[q].seq < s->slots[best].seq))
          best = (int)q;
      if (best < 0) break;
      Slot& sl = s->slots[best];
      if (sl.zeros > 0) {
        // lost blocks of a stream with a declared block length: zeros at
        // their true position, as much as fits now
        const int64_t z = std::min<int64_t>(sl.zeros, s->cap - (tl.E - tl.pbase));
        if (z > 0) {
          if ((e = (int)hipMemset2DAsync(s->pend[s->cur] + (tl.E - tl.pbase) * s->elem,
                                         (size_t)s->cap * s->elem, 0, (size_t)z * s->elem,
                                         (size_t)s->p.nchan, cs)))
            return e;
          tl.E += z;
          sl.zeros -= z;
          any = true;
        }
        if (sl.zeros > 0) break;  // the rest after this batch's compaction
      }
      const int64_t off = tl.E - tl.pbase;
      if (off + sl.nsamp > s->cap) break;  // next batch, after compaction
      if ((e = (int)hipStreamWaitEvent(cs, sl.h2d, 0))) return e;
      if ((e = launch_transpose(sl.dev, s->pend[s->cur] + off * s->elem, s->p.dtype, sl.nsamp,
                                s->p.nchan, s->cap, cs)))
        return e;
      tl.E += sl.nsamp;
      sl.state = TAKEN;
      br.slots.push_back({s->id, best});
      br.arrivals.push_back(sl.t_arrive);
      any = true;
    }
    const bool flush = s->closing && !any && s->slots.end() == std::find_if(
        s->slots.begin(), s->slots.end(), [](const Slot& x) { return x.state != FREE; });
    if (!any && !flush) continue;
    // complete blocks: block k reads [k M - nfront, k M - nfront + N)
    const int64_t nproc = blocks_ready(s->tl, s->g, flush);
    work.push_back({s, nproc, 0});
    if (flush) s->flushed = true;
  }
  if (work.empty()) return 0;
  // 2. one persistent launch for every stream of a sample type whose length
  //    the mixed-length kernel takes, one per length above that
  auto group_key = [&](size_t w) {
    const BeamPlan& p = work[w].s->p;
    return (mixed_supported(p.N) ? 0 : p.N) * 2 + p.dtype;
  };
  std::vector<BatchBeam> group;
  std::vector<bool> done(work.size(), false);
  size_t tab_used = 0;
  int ngroup = 0;
  for (size_t w0 = 0; w0 < work.size(); ++w0) {
    if (done[w0] || work[w0].nproc == 0) continue;
    group.clear();
    for (size_t w = w0; w < work.size(); ++w) {
      if (done[w] || work[w].nproc == 0 || group_key(w) != group_key(w0)) continue;
      done[w] = true;
      Stream* s = work[w].s;
      BatchBeam bb;
      bb.p = &s->p;
      bb.xt = s->pend[s->cur];
      bb.dms.ndm = 1;
      bb.dms.dm[0] = s->p.dms[0];
      bb.P = s->Pb[s->pcur] + (s->tl.U - s->tl.ubase);
      Coords co;
      co.x_stride = s->cap;
      co.x_len = s->tl.E - s->tl.pbase;
      co.load_off = 0;
      co.p_stride = s->pcap;
      co.p_dm_stride = (int64_t)s->p.nchan * s->pcap;
      co.u_lim = s->closing ? s->tl.E / s->p.n_int - s->tl.U
                            : s->pcap - (s->tl.U - s->tl.ubase);
      co.v_stride = 0;
      co.o_lim = 0;
      co.nblocks = work[w].nproc;
      bb.co = co;
      group.push_back(bb);
    }
    std::stable_sort(group.begin(), group.end(), [](const BatchBeam& x, const BatchBeam& y) {
      return (int64_t)x.p->nchan * x.co.nblocks > (int64_t)y.p->nchan * y.co.nblocks;
    });
    br.host_tabs.emplace_back(batch_table_bytes((int)group.size()), 0);
    void* tok = nullptr;
    if ((e = stage_begin(kStageBlock, cs, &tok))) return e;
    LaunchDesc ld;
    const int kind = mixed_supported(group[0].p->N) ? kLaunchMixed : kLaunchBatch;
    if ((e = prepare_launch(kind, group.data(), nullptr, (int)group.size(),
                            br.host_tabs.back().data(), &ld)))
      return e;
    if ((e = enqueue_launch(ld, br.host_tabs.back().data(), (char*)br.tab_dev + tab_used,
                            br.counter + 64 * ngroup, cs)))
      return e;
    if ((e = stage_end(kStageBlock, cs, tok))) return e;
    tab_used += batch_table_bytes((int)group.size());
    if (++ngroup >= kMaxGroups) return (int)hipErrorInvalidValue;
  }
  // 3. aligned sums of the newly finished samples, copies to the host,
  //    compaction of the pending input and intensities
  for (auto& w : work) {
    Stream* s = w.s;
    const BeamPlan& p = s->p;
    Timeline& tl = s->tl;
    const int64_t U_old = tl.U, ub_old = tl.ubase;
    const Advance adv = timeline_advance(&tl, s->g, w.nproc, s->closing, s->flushed);
    (void)U_old;
    const int64_t cnt = adv.count;
    if (cnt > 0) {
      if (cnt > s->icap) return (int)hipErrorInvalidValue;
      void* tok = nullptr;
      if ((e = stage_begin(kStageDsum, cs, &tok))) return e;
      if ((e = launch_dsum_range(p.nchan, 1, s->Pb[s->pcur], s->pcap, (int64_t)p.nchan * s->pcap,
                                 tl.U - ub_old, adv.u_first - ub_old, cnt, s->d, s->Iout,
                                 nullptr, cnt, cs)))
        return e;
      if ((e = stage_end(kStageDsum, cs, tok))) return e;
      float* hout = s->Ihost + (size_t)(&br - sv->ring) * s->icap;
      if ((e = (int)hipMemcpyAsync(hout, s->Iout, cnt * sizeof(float), hipMemcpyDeviceToHost,
                                   cs)))
        return e;
      br.outs.push_back({s->id, {adv.u_first, cnt}});
      br.host_outs.push_back(hout);
    }
    // compaction: keep input from the next block's start, intensities from
    // the first output not yet final
    const int64_t keep = tl.E - adv.pb_new;
    if (adv.pb_new != tl.pbase && !s->flushed) {
      char* src = s->pend[s->cur] + (adv.pb_new - tl.pbase) * s->elem;
      char* dst = s->pend[s->cur ^ 1];
      if (keep > 0 &&
          (e = (int)hipMemcpy2DAsync(dst, s->cap * s->elem, src, s->cap * s->elem,
                                     keep * s->elem, p.nchan, hipMemcpyDeviceToDevice, cs)))
        return e;
      s->cur ^= 1;
      tl.pbase = adv.pb_new;
    }
    if (adv.ub_new != tl.ubase && !s->flushed) {
      const int64_t pk = tl.U - adv.ub_new;
      if (pk > 0 &&
          (e = (int)hipMemcpy2DAsync(s->Pb[s->pcur ^ 1], s->pcap * 4,
                                     s->Pb[s->pcur] + (adv.ub_new - tl.ubase), s->pcap * 4, pk * 4,
                                     p.nchan, hipMemcpyDeviceToDevice, cs)))
        return e;
      s->pcur ^= 1;
      tl.ubase = adv.ub_new;
    }
    if (s->flushed) s->total_int = tl.E / p.n_int;
  }
  return (int)hipEventRecord(br.done, cs);
}

// Completed batches: hand results to the streams, free slots, latencies.
// Batches are taken round the ring from the oldest (the entry after the last
// issued one) and in issue order only, so a stream's intensities are appended
// in time order even when several batches complete between two visits.
void reap(cdd_server* sv, bool wait) {
  for (int j = 0; j < kBatchRing; ++j) {
    BatchRec& br = sv->ring[(sv->ring_next + j) % kBatchRing];
    if (!br.busy) continue;
    hipError_t q = wait ? hipEventSynchronize(br.done) : hipEventQuery(br.done);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) {
      sv->thread_error = hipGetErrorString(q);
      br.busy = false;
      continue;
    }
    const double t = now_s();
    for (size_t k = 0; k < br.outs.size(); ++k) {
      auto it = sv->streams.find(br.outs[k].first);
      if (it == sv->streams.end()) continue;
      Stream* s = it->second.get();
      const int64_t u0 = br.outs[k].second.first, n = br.outs[k].second.second;
      if (s->ready.empty()) s->ready_first = u0;
      const float* h = br.host_outs[k];
      s->ready.insert(s->ready.end(), h, h + n);
    }
    for (auto& ps : br.slots) {
      auto it = sv->streams.find(ps.first);
      if (it == sv->streams.end()) continue;
      Stream* s = it->second.get();
      Slot& sl = s->slots[ps.second];
      sl.state = FREE;
      sv->st.blocks_done++;
      sv->st.data_s += (double)sl.nsamp / (s->p.df * 1e6);
      sv->pending_work--;
    }
    for (double ta : br.arrivals) sv->lat.push_back((t - ta) * 1e3);
    sv->t_last = t;
    br.outs.clear();
    br.slots.clear();
    br.arrivals.clear();
    br.host_tabs.clear();
    br.host_outs.clear();
    br.busy = false;
  }
}

bool has_work(cdd_server* sv) {
  for (auto& kv : sv->streams) {
    Stream* s = kv.second.get();
    if (s->released || s->flushed) continue;
    for (auto& sl : s->slots)
      if (sl.state == PUSHED) return true;
    if (s->closing) {
      bool idle = true;
      for (auto& sl : s->slots)
        if (sl.state != FREE) idle = false;
      if (idle) return true;
    }
  }
  return false;
}

void scheduler(cdd_server* sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    reap(sv, false);
    if (sv->stop && !has_work(sv)) {
      bool busy = false;
      for (auto& br : sv->ring) busy |= br.busy;
      if (!busy) break;
    }
    BatchRec& br = sv->ring[sv->ring_next];
    if (has_work(sv) && !br.busy) {
      const int e = issue_batch(sv, br);
      if (e) {
        sv->thread_error = hipGetErrorString((hipError_t)e);
      } else if (!br.slots.empty() || !br.outs.empty()) {
        br.busy = true;
        sv->st.batches++;
        sv->ring_next = (sv->ring_next + 1) % kBatchRing;
      } else {
        // nothing launched (e.g. a flush with no output): still ordered
        (void)hipEventRecord(br.done, sv->compute);
        br.busy = true;
        sv->ring_next = (sv->ring_next + 1) % kBatchRing;
      }
      sv->cv.notify_all();
      continue;
    }
    sv->cv.notify_all();
    sv->cv.wait_for(lk, std::chrono::microseconds(200));
  }
  sv->cv.notify_all();
}

}  // namespace
}  // namespace cdd

using namespace cdd;

extern "C" {

cdd_status cdd_server_create(const cdd_server_opts* opts, cdd_server** out) {
  if (!out) return fail(CDD_EINVAL, "out is NULL");
  *out = nullptr;
  try {
    std::unique_ptr<cdd_server> sv(new cdd_server());
    sv->budget = (opts && opts->hbm_budget) ? opts->hbm_budget : ((size_t)8 << 30);
    sv->max_streams = (opts && opts->max_streams > 0) ? opts->max_streams : 64;
    sv->depth = (opts && opts->queue_depth > 0) ? opts->queue_depth : 4;
    hipError_t e = hipGetDevice(&sv->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->compute, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->h2d, hipStreamNonBlocking);
    const size_t tab = al256(batch_table_bytes(sv->max_streams)) * 2;
    for (int i = 0; i < kBatchRing && e == hipSuccess; ++i) {
      e = hipEventCreateWithFlags(&sv->ring[i].done, hipEventDisableTiming);
      if (e == hipSuccess) e = hipMalloc(&sv->ring[i].tab_dev, tab);
      if (e == hipSuccess) e = hipMalloc((void**)&sv->ring[i].counter, 256 * kMaxGroups);
    }
    if (e != hipSuccess) return fail(CDD_EDEVICE, "server create: %s", hipGetErrorString(e));
    sv->th = std::thread(scheduler, sv.get());
    *out = sv.release();
    clear_error();
    return CDD_OK;
  } catch (...) {
    return fail(CDD_ENOMEM, "server create failed");
  }
}

void cdd_server_destroy(cdd_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  if (sv->th.joinable()) sv->th.join();
  (void)hipStreamSynchronize(sv->compute);
  (void)hipStreamSynchronize(sv->h2d);
  for (auto& kv : sv->streams) free_stream_mem(kv.second.get());
  for (auto& br : sv->ring) {
    if (br.done) (void)hipEventDestroy(br.done);
    if (br.tab_dev) (void)hipFree(br.tab_dev);
    if (br.counter) (void)hipFree(br.counter);
  }
  (void)hipStreamDestroy(sv->compute);
  (void)hipStreamDestroy(sv->h2d);
  delete sv;
}

cdd_status cdd_stream_open(cdd_server* sv, const cdd_stream_desc* d, int32_t* id) {
  if (!sv || !d || !id) return fail(CDD_EINVAL, "NULL argument");
  if (d->max_block < 1) return fail(CDD_EINVAL, "max_block must be >= 1");
  cdd_opts o{};
  o.phase_mode = d->phase_mode;
  o.taper = d->taper;
  BeamPlan p;
  cdd_status s = make_plan(d->dtype, d->max_block, d->nchan, d->f_centre_mhz, d->bw_mhz, &d->dm,
                           1, d->fft_len, d->n_int, &o, &p);
  if (s != CDD_OK) return s;
  if (!block_supported(p.N))
    return fail(CDD_ENOTSUP, "streams support fft_len up to 16384 (got %d)", p.N);
  if (d->block_len < 0 || d->block_len > d->max_block)
    return fail(CDD_EINVAL, "block_len must be in [0, max_block]");
  std::unique_ptr<Stream> st(new Stream());
  st->p = p;
  st->max_block = d->max_block;
  st->block_len = d->block_len;
  st->elem = p.dtype == CDD_CI8 ? 2 : 8;
  st->g.N = p.N;
  st->g.M = p.M;
  st->g.nfront = p.nfront;
  st->g.n_int = p.n_int;
  st->g.front = p.front;
  st->g.back = p.back;
  st->g.d_max = p.d_max;
  st->g.nchan = p.nchan;
  st->g.elem = (int64_t)st->elem;
  const Footprint fp = stream_footprint(st->g, d->max_block, sv->depth);
  st->cap = fp.cap;
  st->pcap = fp.pcap;
  st->icap = fp.icap;
  const size_t bytes = fp.bytes;
  timeline_start(&st->tl, st->g);
  std::lock_guard<std::mutex> lk(sv->mu);
  int open = 0;
  for (auto& kv : sv->streams)
    if (!kv.second->released) ++open;
  if (!admit(sv->used, sv->budget, open, sv->max_streams, bytes)) {
    sv->st.refused++;
    return fail(CDD_EAGAIN, "stream needs %zu bytes; %zu of %zu in use, %d streams open", bytes,
                sv->used, sv->budget, open);
  }
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipMalloc((void**)&st->pend[i], (size_t)p.nchan * st->cap * st->elem);
    if (e == hipSuccess) e = hipMalloc((void**)&st->Pb[i], (size_t)p.nchan * st->pcap * 4);
  }
  if (e == hipSuccess) e = hipMalloc((void**)&st->d, (size_t)p.nchan * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&st->Iout, (size_t)st->icap * 4);
  if (e == hipSuccess) e = hipHostMalloc((void**)&st->Ihost, (size_t)st->icap * 4 * kBatchRing);
  st->slots.resize(sv->depth);
  for (auto& sl : st->slots) {
    const size_t b = (size_t)d->max_block * p.nchan * st->elem;
    if (e == hipSuccess) e = hipHostMalloc(&sl.host, b);
    if (e == hipSuccess) e = hipMalloc(&sl.dev, b);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.h2d, hipEventDisableTiming);
  }
  if (e == hipSuccess)
    e = hipMemsetAsync(st->pend[0], 0, (size_t)p.nchan * st->cap * st->elem, sv->compute);
  DmTile t;
  t.ndm = 1;
  t.dm[0] = d->dm;
  if (e == hipSuccess) e = (hipError_t)launch_delays(p, t, st->d, sv->compute);
  if (e != hipSuccess) {
    free_stream_mem(st.get());
    return fail(e == hipErrorOutOfMemory ? CDD_ENOMEM : CDD_EDEVICE, "stream open: %s",
                hipGetErrorString(e));
  }
  st->bytes = bytes;
  st->id = sv->next_id++;
  sv->used += bytes;
  sv->st.admitted++;
  *id = st->id;
  sv->streams[st->id] = std::move(st);
  clear_error();
  return CDD_OK;
}

cdd_status cdd_stream_push(cdd_server* sv, int32_t id, const void* host_block, int64_t nsamp,
                           uint64_t seq) {
  if (!sv || !host_block) return fail(CDD_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->streams.find(id);
  if (it == sv->streams.end() || it->second->released)
    return fail(CDD_EINVAL, "no open stream %d", id);
  Stream* s = it->second.get();
  if (s->closing) return fail(CDD_EINVAL, "stream %d is closed", id);
  if (nsamp < 1 || nsamp > s->max_block)
    return fail(CDD_EINVAL, "block of %lld samples outside [1, %lld]", (long long)nsamp,
                (long long)s->max_block);
  if (s->block_len > 0 && (nsamp > s->block_len || s->short_seen))
    return fail(CDD_EINVAL, "stream %d declared blocks of %lld samples; only the last may be "
                "shorter", id, (long long)s->block_len);
  if (classify_push(s->tl.next_seq, seq) == kPushStale) {
    sv->st.rejected++;
    return fail(CDD_EINVAL, "sequence %llu already seen (next is %llu)", (unsigned long long)seq,
                (unsigned long long)s->tl.next_seq);
  }
  int free_slot = -1;
  for (size_t q = 0; q < s->slots.size(); ++q)
    if (s->slots[q].state == FREE) {
      free_slot = (int)q;
      break;
    }
  if (free_slot < 0) return fail(CDD_EAGAIN, "stream %d queue full", id);
  Slot& sl = s->slots[free_slot];
  const size_t bytes = (size_t)nsamp * s->p.nchan * s->elem;
  std::memcpy(sl.host, host_block, bytes);
  hipError_t e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, sv->h2d);
  if (e == hipSuccess) e = hipEventRecord(sl.h2d, sv->h2d);
  if (e != hipSuccess) return fail(CDD_EDEVICE, "push copy: %s", hipGetErrorString(e));
  sl.nsamp = nsamp;
  sl.seq = seq;
  if (timeline_push(&s->tl, s->g, seq, nsamp, s->block_len, &sl.zeros) == kPushGap)
    sv->st.gaps++;
  if (s->block_len > 0 && nsamp < s->block_len) s->short_seen = true;
  sl.t_arrive = now_s();
  if (sv->t_first < 0) sv->t_first = sl.t_arrive;
  sl.state = PUSHED;
  sv->st.blocks_in++;
  sv->pending_work++;
  sv->cv.notify_all();
  clear_error();
  return CDD_OK;
}

cdd_status cdd_stream_poll(cdd_server* sv, int32_t id, float* host_out, int64_t cap, int64_t* n,
                           int64_t* u_first) {
  if (!sv || !n || !u_first || (cap > 0 && !host_out)) return fail(CDD_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->streams.find(id);
  if (it == sv->streams.end()) return fail(CDD_EINVAL, "no stream %d", id);
  Stream* s = it->second.get();
  const int64_t k = std::min<int64_t>(cap, (int64_t)s->ready.size());
  *u_first = s->ready_first;
  for (int64_t i = 0; i < k; ++i) host_out[i] = s->ready[i];
  s->ready.erase(s->ready.begin(), s->ready.begin() + k);
  s->ready_first += k;
  s->polled += k;
  *n = k;
  bool release = false;
  if (s->flushed && s->total_int >= 0 && s->polled >= s->total_int && !s->released &&
      !s->releasing) {
    bool idle = true;
    for (auto& sl : s->slots)
      if (sl.state != FREE) idle = false;
    for (auto& br : sv->ring)
      if (br.busy)
        for (auto& o : br.outs)
          if (o.first == id) idle = false;
    release = idle;
  }
  if (release) {
    // the stream's memory is freed without the server lock held: the
    // scheduler skips a flushed stream, and `releasing` keeps other callers off
    s->releasing = true;
    lk.unlock();
    (void)hipStreamSynchronize(sv->compute);
    free_stream_mem(s);
    lk.lock();
    s->released = true;
    sv->used -= s->bytes;
  }
  clear_error();
  return CDD_OK;
}

cdd_status cdd_stream_invalid(cdd_server* sv, int32_t id, int64_t* spans, int64_t cap,
                              int64_t* n) {
  if (!sv || !n || (cap > 0 && !spans)) return fail(CDD_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->streams.find(id);
  if (it == sv->streams.end()) return fail(CDD_EINVAL, "no stream %d", id);
  const auto& inv = it->second->tl.invalid;
  const int64_t k = std::min<int64_t>(cap, (int64_t)inv.size());
  for (int64_t i = 0; i < k; ++i) {
    spans[2 * i] = inv[i].first;
    spans[2 * i + 1] = inv[i].second;
  }
  *n = (int64_t)inv.size();
  clear_error();
  return CDD_OK;
}

cdd_status cdd_stream_close(cdd_server* sv, int32_t id) {
  if (!sv) return fail(CDD_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->streams.find(id);
  if (it == sv->streams.end() || it->second->released)
    return fail(CDD_EINVAL, "no open stream %d", id);
  it->second->closing = true;
  sv->cv.notify_all();
  clear_error();
  return CDD_OK;
}

cdd_status cdd_server_sync(cdd_server* sv) {
  if (!sv) return fail(CDD_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool busy = has_work(sv) || sv->pending_work > 0;
    for (auto& br : sv->ring) busy |= br.busy;
    if (!busy) break;
    if (!sv->thread_error.empty()) break;
    sv->cv.wait_for(lk, std::chrono::milliseconds(1));
  }
  if (!sv->thread_error.empty())
    return fail(CDD_EDEVICE, "scheduler: %s", sv->thread_error.c_str());
  clear_error();
  return CDD_OK;
}

cdd_status cdd_server_stats_get(cdd_server* sv, cdd_server_stats* out) {
  if (!sv || !out) return fail(CDD_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->st;
  if (!sv->lat.empty()) {
    out->lat_p50_ms = percentile(sv->lat, 0.50);
    out->lat_p99_ms = percentile(sv->lat, 0.99);
    out->lat_max_ms = percentile(sv->lat, 1.0);
  }
  out->wall_s = sv->t_first >= 0 ? sv->t_last - sv->t_first : 0;
  out->hbm_used = sv->used;
  out->hbm_budget = sv->budget;
  clear_error();
  return CDD_OK;
}

}  // extern "C"
