// Host bookkeeping of the serving loop, free of device calls: admission by
// device-memory budget, the sequence rules of pushed blocks, and the
// timeline of one stream (which overlap-save blocks can run, which aligned
// sums are final, what the pending buffers keep, and which outputs include
// lost input).  The server issues its device work from these decisions; the
// CPU tests drive them directly.
#pragma once

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

namespace cdd {

// Plan figures of a stream that the timeline needs (samples per channel).
struct StreamGeom {
  int64_t N = 0, M = 0, nfront = 0, n_int = 1;
  int64_t front = 0, back = 0;  // reach of the filter's impulse response
  int64_t d_max = 0;            // largest channel delay (integrated samples)
  int64_t nchan = 1;
  int64_t elem = 2;             // bytes per input sample
};

// Device bytes a stream holds and the sizes of its buffers: pending input
// (cap samples per channel, two for compaction), per-channel intensities
// (pcap, two), delays, finished-output staging (icap) and `depth` push slots.
struct Footprint {
  size_t bytes = 0;
  int64_t cap = 0, pcap = 0, icap = 0;
};
Footprint stream_footprint(const StreamGeom& g, int64_t max_block, int depth);
// Whether a stream of `bytes` may open next to `open` others holding `used`.
bool admit(size_t used, size_t budget, int open, int max_streams, size_t bytes);

// Sequence rules: seq below the next expected is refused (stale); above it,
// blocks were lost (gap).
enum PushVerdict { kPushNext = 0, kPushGap = 1, kPushStale = 2 };
PushVerdict classify_push(uint64_t next_seq, uint64_t seq);

// The timeline of one stream, in absolute samples (per channel) and
// integrated samples.  Block k of the overlap-save grid reads input samples
// [k M - nfront, k M - nfront + N) and yields outputs [k M, k M + M).
struct Timeline {
  int64_t accepted = 0; // samples of accepted pushes, plus lost samples re-inserted
  int64_t E = 0;        // input samples appended to the pending buffer so far
  int64_t kn = 0;       // blocks processed
  int64_t pbase = 0;    // first sample held in the pending input buffer
  int64_t U = 0;        // integrated samples computed per channel
  int64_t ubase = 0;    // first integrated sample held per channel
  int64_t Inext = 0;    // first aligned-sum output not yet final
  uint64_t next_seq = 0;
  std::vector<std::pair<int64_t, int64_t>> invalid;  // [begin, end) of I with lost input
};
void timeline_start(Timeline* tl, const StreamGeom& g);  // pbase = -nfront
// A pushed block of nsamp samples with sequence seq >= next_seq is accepted.
// When blocks were lost and the stream declared its block length, their
// samples are to be inserted as zeros at their true position, before this
// block (*zeros_before); otherwise the block joins the data before the gap.
// Either way the aligned-sum outputs whose inputs include the lost span (or
// the junction) are recorded in tl->invalid.  Returns the verdict (nothing
// changes for a stale block).
PushVerdict timeline_push(Timeline* tl, const StreamGeom& g, uint64_t seq, int64_t nsamp,
                          int64_t block_len, int64_t* zeros_before);
// Blocks whose whole input window is in (or, at the end of the stream,
// past the data, zero-padded).
int64_t blocks_ready(const Timeline& tl, const StreamGeom& g, bool flush);
// After nproc blocks have run: per-channel intensities advance, and the
// aligned sums [u_first, u_first + count) become final (every channel's
// delayed input known; at the end of the stream, all of them).  Also the
// new starts of the pending input and intensity buffers after compaction.
struct Advance {
  int64_t u_first = 0, count = 0;
  int64_t pb_new = 0, ub_new = 0;
};
Advance timeline_advance(Timeline* tl, const StreamGeom& g, int64_t nproc, bool closing,
                         bool flushed);
// Aligned-sum outputs [begin, end) whose inputs include samples [t0, t1)
// (t1 == t0: a junction of data across a gap), clamped at 0.
std::pair<int64_t, int64_t> invalid_span(const StreamGeom& g, int64_t t0, int64_t t1);
// Value at fraction q of the sorted samples (nearest rank); 0 if empty.
double percentile(std::vector<double> v, double q);

}  // namespace cdd
