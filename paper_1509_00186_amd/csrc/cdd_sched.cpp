// Host bookkeeping of the serving loop (see cdd_sched.h).
#include "cdd_sched.h"

#include <algorithm>

namespace cdd {

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

static int64_t floor_div(int64_t a, int64_t b) {
  const int64_t q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

Footprint stream_footprint(const StreamGeom& g, int64_t max_block, int depth) {
  Footprint f;
  f.cap = g.N + max_block;
  const int64_t per_batch = (max_block + g.N) / g.n_int + g.M / g.n_int + 2;
  f.pcap = g.d_max + 2 + per_batch;
  f.icap = per_batch + g.d_max + 2;
  f.bytes = 2 * al256((size_t)g.nchan * f.cap * g.elem) + 2 * al256((size_t)g.nchan * f.pcap * 4) +
            al256((size_t)g.nchan * 4) + al256((size_t)f.icap * 4) +
            (size_t)depth * al256((size_t)max_block * g.nchan * g.elem);
  return f;
}

bool admit(size_t used, size_t budget, int open, int max_streams, size_t bytes) {
  return open < max_streams && used <= budget && bytes <= budget - used;
}

PushVerdict classify_push(uint64_t next_seq, uint64_t seq) {
  if (seq < next_seq) return kPushStale;
  return seq == next_seq ? kPushNext : kPushGap;
}

void timeline_start(Timeline* tl, const StreamGeom& g) {
  *tl = Timeline();
  tl->pbase = -g.nfront;  // the first block sees nfront zeros before sample 0
}

std::pair<int64_t, int64_t> invalid_span(const StreamGeom& g, int64_t t0, int64_t t1) {
  // output y[t] depends on input within the filter's reach on either side;
  // P[u] on y over [u n_int, (u + 1) n_int); I[u] on P[u + d_c], d_c in [0, d_max]
  const int64_t R = g.front + g.back;
  const int64_t lo = floor_div(t0 - R, g.n_int) - g.d_max;
  const int64_t hi = floor_div(t1 + R + g.n_int - 1, g.n_int) + 1;
  return {std::max<int64_t>(0, lo), std::max<int64_t>(0, hi)};
}

PushVerdict timeline_push(Timeline* tl, const StreamGeom& g, uint64_t seq, int64_t nsamp,
                          int64_t block_len, int64_t* zeros_before) {
  *zeros_before = 0;
  const PushVerdict v = classify_push(tl->next_seq, seq);
  if (v == kPushStale) return v;
  if (v == kPushGap) {
    const int64_t t0 = tl->accepted;
    const int64_t lost = block_len > 0 ? (int64_t)(seq - tl->next_seq) * block_len : 0;
    *zeros_before = lost;
    tl->accepted += lost;
    tl->invalid.push_back(invalid_span(g, t0, t0 + lost));
  }
  tl->accepted += nsamp;
  tl->next_seq = seq + 1;
  return v;
}

int64_t blocks_ready(const Timeline& tl, const StreamGeom& g, bool flush) {
  int64_t n = 0;
  if (flush) {
    while ((tl.kn + n) * g.M < tl.E) ++n;
  } else {
    while ((tl.kn + n) * g.M - g.nfront + g.N <= tl.E) ++n;
  }
  return n;
}

Advance timeline_advance(Timeline* tl, const StreamGeom& g, int64_t nproc, bool closing,
                         bool flushed) {
  Advance a;
  const int64_t step = g.M / g.n_int;
  int64_t U_new = tl->U + nproc * step;
  if (closing) U_new = std::min<int64_t>(U_new, tl->E / g.n_int);
  tl->kn += nproc;
  tl->U = U_new;
  const int64_t u_fin = flushed ? tl->U : std::max<int64_t>(tl->Inext, tl->U - g.d_max);
  a.u_first = tl->Inext;
  a.count = std::max<int64_t>(0, u_fin - tl->Inext);
  tl->Inext = std::max(tl->Inext, u_fin);
  a.pb_new = tl->kn * g.M - g.nfront;
  a.ub_new = tl->Inext;
  return a;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const size_t i = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
  return v[i];
}

}  // namespace cdd
