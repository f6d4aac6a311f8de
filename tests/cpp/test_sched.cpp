// CPU tests of the serving bookkeeping (cdd_sched.h) against a fake
// executor: a host model of the scheduler loop in which the pending buffer
// holds sample indices instead of voltages, every "launched" block checks
// that its whole input window is in the buffer, and every finished aligned
// sum is recorded.  No device is involved.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "cdd_sched.h"

using namespace cdd;

static int g_fail = 0;
#define CHECK(cond, ...)                                      \
  do {                                                        \
    if (!(cond)) {                                            \
      std::printf("FAIL %s:%d: %s -- ", __FILE__, __LINE__, #cond); \
      std::printf(__VA_ARGS__);                               \
      std::printf("\n");                                      \
      ++g_fail;                                               \
    }                                                         \
  } while (0)

struct Push {
  int64_t nsamp;
  uint64_t seq;
};

// The scheduler's decisions for one stream, replayed on the host: pushes are
// consumed in order into a pending buffer of `cap` samples (lost samples as
// zeros, marked -1), complete blocks run, outputs become final, the buffers
// compact.  Returns the outputs in the order they were finalised.
struct FakeExec {
  StreamGeom g;
  int64_t cap, block_len;
  Timeline tl;
  std::vector<int64_t> buf;      // sample index held at pend[i] (i = t - pbase), -1 = zero
  std::vector<int64_t> emitted;  // finalised aligned-sum outputs, in order
  int64_t next_index = 0;        // index of the next pushed sample
  int batches = 0;

  FakeExec(const StreamGeom& g_, int64_t max_block, int64_t block_len_)
      : g(g_), block_len(block_len_) {
    cap = stream_footprint(g, max_block, 1).cap;
    timeline_start(&tl, g);
    buf.assign(cap, -1);
  }

  // one push through the timeline, then consumed as the scheduler does
  // (zeros first, as much as fits, processing and compacting in between)
  void push(const Push& p) {
    int64_t zeros = 0;
    const PushVerdict v = timeline_push(&tl, g, p.seq, p.nsamp, block_len, &zeros);
    if (v == kPushStale) return;
    while (zeros > 0) {
      const int64_t z = std::min<int64_t>(zeros, cap - (tl.E - tl.pbase));
      for (int64_t i = 0; i < z; ++i) buf[tl.E - tl.pbase + i] = -1;
      tl.E += z;
      zeros -= z;
      if (zeros > 0) batch(false);
    }
    while (tl.E - tl.pbase + p.nsamp > cap) batch(false);
    for (int64_t i = 0; i < p.nsamp; ++i) buf[tl.E - tl.pbase + i] = next_index + i;
    next_index += p.nsamp;
    tl.E += p.nsamp;
    batch(false);
  }

  void batch(bool flush) {
    ++batches;
    const int64_t nproc = blocks_ready(tl, g, flush);
    for (int64_t k = tl.kn; k < tl.kn + nproc; ++k) {
      const int64_t t0 = k * g.M - g.nfront, t1 = t0 + g.N;
      CHECK(t0 >= tl.pbase, "block %lld starts at %lld before the buffer (%lld)", (long long)k,
            (long long)t0, (long long)tl.pbase);
      if (!flush) CHECK(t1 <= tl.E, "block %lld reads past the data", (long long)k);
      // the data part of the window (past E the kernel reads zeros) is held
      CHECK(std::min(t1, tl.E) - tl.pbase <= cap, "block %lld reads past the buffer",
            (long long)k);
    }
    const Advance a = timeline_advance(&tl, g, nproc, flush, flush);
    for (int64_t u = a.u_first; u < a.u_first + a.count; ++u) emitted.push_back(u);
    // every finalised output has all channels' delayed intensities computed
    if (!flush && a.count > 0)
      CHECK(a.u_first + a.count + g.d_max <= tl.U, "output finalised before its inputs");
    if (!flush && a.pb_new != tl.pbase) {
      CHECK(a.pb_new >= tl.pbase, "compaction goes backwards");
      std::vector<int64_t> nb(cap, -1);
      for (int64_t t = a.pb_new; t < tl.E; ++t) nb[t - a.pb_new] = buf[t - tl.pbase];
      buf.swap(nb);
      tl.pbase = a.pb_new;
    }
    if (!flush) tl.ubase = a.ub_new;
  }

  void close() {
    batch(true);
  }
};

static StreamGeom geom(int64_t N, int64_t L, int64_t nfront, int64_t n_int, int64_t d_max,
                       int64_t front, int64_t back) {
  StreamGeom g;
  g.N = N;
  g.M = N - L;
  g.nfront = nfront;
  g.n_int = n_int;
  g.d_max = d_max;
  g.front = front;
  g.back = back;
  g.nchan = 16;
  g.elem = 2;
  return g;
}

// outputs emitted exactly once each, in order, covering [0, total / n_int)
static void check_outputs(const FakeExec& fx, int64_t total, const char* what) {
  const int64_t want = total / fx.g.n_int;
  CHECK((int64_t)fx.emitted.size() == want, "%s: %zu outputs, want %lld", what,
        fx.emitted.size(), (long long)want);
  for (size_t i = 0; i < fx.emitted.size(); ++i)
    if (fx.emitted[i] != (int64_t)i) {
      CHECK(false, "%s: output %zu is %lld", what, i, (long long)fx.emitted[i]);
      break;
    }
}

static void test_random_blocks() {
  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t N = 1 << (8 + trial % 6), L = N / 8 + (trial % 3) * 4;
    const int64_t n_int = 1 + trial % 5;
    int64_t Lr = L;
    while ((N - Lr) % n_int) ++Lr;
    const StreamGeom g = geom(N, Lr, Lr / 2, n_int, trial * 13 % 200, Lr / 2, Lr / 3);
    const int64_t max_block = 50 + (int64_t)(rng() % 5000);
    FakeExec fx(g, max_block, 0);
    int64_t total = 0;
    const int nblk = 5 + (int)(rng() % 40);
    for (int i = 0; i < nblk; ++i) {
      const int64_t n = 1 + (int64_t)(rng() % max_block);
      fx.push({n, (uint64_t)i});
      total += n;
    }
    fx.close();
    check_outputs(fx, total, "random blocks");
    CHECK(fx.tl.invalid.empty(), "no gap, no invalid span");
  }
}

// with a declared block length, lost blocks come back as zeros at their
// position: the timeline equals the whole record, and the invalid span
// holds every output whose dependency reaches the lost samples
static void test_gap_with_block_length() {
  const StreamGeom g = geom(2048, 128, 64, 4, 37, 60, 50);
  const int64_t B = 1500;
  FakeExec fx(g, B, B);
  int64_t total = 0;
  const std::vector<uint64_t> seqs = {0, 1, 2, 5, 6, 7, 8};  // 3 and 4 lost
  for (uint64_t s : seqs) fx.push({B, s});
  total = 9 * B;
  fx.close();
  check_outputs(fx, total, "gap with block length");
  CHECK(fx.tl.invalid.size() == 1, "one span, got %zu", fx.tl.invalid.size());
  // brute force: I[u] reads P_c[u + d], d in [0, d_max]; P[v] reads y over
  // [v n_int, (v + 1) n_int); y[t] reads x over [t - back, t + front]
  const int64_t lost0 = 3 * B, lost1 = 5 * B;
  const auto span = fx.tl.invalid[0];
  for (int64_t u = 0; u < total / g.n_int; ++u) {
    const int64_t x_lo = u * g.n_int - g.back - g.front;
    const int64_t x_hi = (u + g.d_max + 1) * g.n_int + g.front + g.back;
    const bool reaches = x_lo < lost1 && x_hi > lost0;
    if (reaches) CHECK(u >= span.first && u < span.second, "u %lld not marked", (long long)u);
  }
  CHECK(span.first >= 0 && span.second > span.first, "span");
  // lost samples are zeros, every other sample is its own index
  CHECK(fx.next_index == 7 * B, "pushed samples");
}

// without a block length the block joins the data before the gap; the
// junction's reach is marked
static void test_gap_without_block_length() {
  const StreamGeom g = geom(1024, 64, 32, 2, 20, 30, 25);
  FakeExec fx(g, 3000, 0);
  fx.push({3000, 0});
  fx.push({2000, 3});  // 1 and 2 lost, length unknown
  fx.push({1000, 4});
  fx.close();
  check_outputs(fx, 6000, "junction");
  CHECK(fx.tl.invalid.size() == 1, "one span");
  const auto span = fx.tl.invalid[0];
  const int64_t j = 3000;
  for (int64_t u = 0; u < 3000; ++u) {
    const int64_t x_lo = u * g.n_int - g.back - g.front;
    const int64_t x_hi = (u + g.d_max + 1) * g.n_int + g.front + g.back;
    if (x_lo < j && x_hi > j) CHECK(u >= span.first && u < span.second, "junction u %lld",
                                    (long long)u);
  }
}

static void test_sequence_rules() {
  CHECK(classify_push(0, 0) == kPushNext, "first");
  CHECK(classify_push(3, 2) == kPushStale, "duplicate");
  CHECK(classify_push(3, 7) == kPushGap, "gap");
  const StreamGeom g = geom(512, 64, 32, 4, 10, 20, 20);
  Timeline tl;
  timeline_start(&tl, g);
  int64_t z = -1;
  CHECK(timeline_push(&tl, g, 0, 100, 100, &z) == kPushNext && z == 0, "push 0");
  CHECK(timeline_push(&tl, g, 0, 100, 100, &z) == kPushStale && tl.accepted == 100, "stale");
  CHECK(timeline_push(&tl, g, 3, 100, 100, &z) == kPushGap && z == 200, "gap zeros %lld",
        (long long)z);
  CHECK(tl.accepted == 400 && tl.next_seq == 4, "accepted %lld", (long long)tl.accepted);
}

static void test_admission() {
  const StreamGeom g = geom(2048, 128, 64, 4, 100, 60, 60);
  const size_t one = stream_footprint(g, 4096, 4).bytes;
  CHECK(one > 0, "footprint");
  CHECK(stream_footprint(g, 8192, 4).bytes > one, "footprint grows with the block");
  CHECK(stream_footprint(g, 4096, 8).bytes > one, "footprint grows with the queue");
  // a budget for one and a half streams: the second is refused until the
  // first is gone; the stream limit refuses too
  const size_t budget = one + one / 2;
  size_t used = 0;
  int open = 0;
  CHECK(admit(used, budget, open, 64, one), "first");
  used += one;
  ++open;
  CHECK(!admit(used, budget, open, 64, one), "second over budget");
  used -= one;
  --open;
  CHECK(admit(used, budget, open, 64, one), "after release");
  CHECK(!admit(0, budget, 2, 2, one), "stream limit");
  CHECK(!admit(budget + 1, budget, 0, 64, 1), "used over budget");
}

static void test_percentile() {
  CHECK(percentile({}, 0.5) == 0.0, "empty");
  std::vector<double> v;
  for (int i = 100; i >= 1; --i) v.push_back(i);
  CHECK(percentile(v, 0.0) == 1.0 && percentile(v, 1.0) == 100.0, "ends");
  CHECK(percentile(v, 0.5) == 51.0, "p50 %g", percentile(v, 0.5));
  CHECK(percentile(v, 0.99) == 99.0, "p99 %g", percentile(v, 0.99));
}

static void test_invalid_span_edges() {
  const StreamGeom g = geom(1024, 64, 32, 4, 10, 8, 8);
  const auto s = invalid_span(g, 0, 0);
  CHECK(s.first == 0 && s.second >= 1, "clamped at zero");
  const auto t = invalid_span(g, 4000, 4400);
  CHECK(t.first <= (4000 - 16) / 4 - 10 && t.second >= (4400 + 16) / 4, "covers the reach");
}

int main() {
  test_random_blocks();
  test_gap_with_block_length();
  test_gap_without_block_length();
  test_sequence_rules();
  test_admission();
  test_percentile();
  test_invalid_span_edges();
  if (g_fail) {
    std::printf("%d failures\n", g_fail);
    return 1;
  }
  std::printf("all passed\n");
  return 0;
}
