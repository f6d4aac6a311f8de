/*
 * cdd.h -- C ABI of the MI355X coherent-dedispersion library (libcdd.so).
 *
 * The library implements overlap-save coherent dedispersion of channelised
 * complex voltage beams as described by De & Gupta, "A Real-time Coherent
 * Dedispersion Pipeline for the Giant Metrewave Radio Telescope":
 *
 *   per channel: forward FFT of N-sample blocks at stride M = N - L
 *                (Sec. 2.2, Sec. 2.3), multiply by the all-pass chirp of
 *                Eq. 3 (Sec. 2.1), inverse FFT keeping M samples per block
 *                (overlap-save, Sec. 2.2 and Sec. 4.3), detect |y|^2 and
 *                integrate n_int samples (Sec. 3.1, write-to-disk routine);
 *   then:        delay-align the channels and sum them (Sec. 1.2, the
 *                linear term of Eq. 2; sub-band alignment of Sec. 1.3).
 *
 * Conventions shared by every call:
 *   - Channel c of a beam centred at f_centre with bandwidth bw (MHz, > 0)
 *     covers [f_c - df/2, f_c + df/2), df = bw / nchan,
 *     f_c = (f_centre - bw/2) + (c + 0.5) * df; channels ascend in frequency.
 *   - The forward transform uses exp(-2 pi i j n / N), the inverse carries
 *     1/N.  Bin j < N/2 sits at +j*df/N from f_c, bin j >= N/2 at (j-N)*df/N.
 *   - The dedispersing filter is exp(-2 pi i q_j), q_j = D*DM*f_j^2 /
 *     (f_c^2 (f_c + f_j)) turns (Eq. 3 with its sign read as the inverse of
 *     the dispersive term of Eq. 2); D defaults to 4.148808e9.
 *   - Block k of a channel transforms input samples [k*M - nfront,
 *     k*M - nfront + N) (zeros outside the data) and yields output samples
 *     [k*M, k*M + M) from its inverse-transform samples [nfront, nfront + M).
 *   - Intensities are |y|^2 summed over samples [u*n_int, (u+1)*n_int),
 *     u < T_int = nsamp / n_int, in (input units)^2.
 *   - Channel delay d_c = floor(D*DM*(1/f_c^2 - 1/f_ref^2)*df/n_int + 0.5)
 *     integrated samples, computed in FP64; f_ref is the top channel centre
 *     for DM >= 0 and the bottom one for DM < 0.
 *     I[u] = sum over c (ascending) with u + d_c < T_int of P_c[u + d_c];
 *     coverage[u] is the number of channels in that sum.
 *
 * Memory: every data pointer is a DEVICE pointer owned by the caller, unless
 * named host_*.  Calls that take a stream enqueue work on it and return
 * without waiting (the stream is a hipStream_t passed as void*, NULL = the
 * null stream).  The library owns only plan and server objects and a cache
 * of FP64-derived twiddle tables per device.
 *
 * Errors: every call returns a cdd_status; no C++ exception, abort or exit
 * crosses the ABI.  cdd_last_error() gives a message for the last failing
 * call on the calling thread.
 */
#ifndef CDD_H
#define CDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDD_ABI_VERSION 1

typedef enum {
  CDD_OK = 0,
  CDD_EINVAL = -1,    /* invalid argument; see cdd_last_error()            */
  CDD_ENOMEM = -2,    /* host or device allocation failed                  */
  CDD_EDEVICE = -3,   /* a HIP call failed; the message holds HIP's string  */
  CDD_EBUSY = -4,     /* object in use (e.g. a stream with work in flight)  */
  CDD_EAGAIN = -5,    /* admission refused now (over budget); retry later   */
  CDD_EINTERNAL = -6, /* invariant broken inside the library               */
  CDD_ENOTSUP = -7    /* valid request the library does not support        */
} cdd_status;

/* Input sample formats (time-major, as a voltage-beam recorder writes
 * them; Sec. 1.1 and Sec. 2.3 describe 8-bit real/imag FFT outputs). */
typedef enum {
  CDD_CI8 = 0,  /* [nsamp][nchan][2] int8: re, im                        */
  CDD_CF32 = 1  /* [nsamp][nchan] complex float (re, im interleaved)       */
} cdd_dtype;

/* How the chirp phase is evaluated on the GPU. */
typedef enum {
  CDD_PHASE_FP64_REDUCED = 0, /* q in FP64, r = q - rint(q), FP32 sin/cos   */
  CDD_PHASE_FP32 = 1          /* q and sin/cos in FP32 (precision study)     */
} cdd_phase_mode;

/* Taper of the chirp function over each channel (Sec. 2.2: the window that
 * multiplies the inverse transfer function; it trades the ripple of the
 * rectangular band edge for sensitivity at the edges).  x = the bin's offset
 * from the channel centre over the channel width, in [-1/2, 1/2). */
typedef enum {
  CDD_TAPER_NONE = 0,  /* rectangular: |H| = 1                               */
  CDD_TAPER_HANN = 1,  /* Hanning: (1 + cos 2 pi x) / 2                      */
  CDD_TAPER_WELCH = 2  /* Welch: 1 - (2 x)^2                                 */
} cdd_taper;

/*
 * cdd_incoherent -- incoherent dedispersion (Sec. 1.2): the same detection,
 * integration and delay-aligned channel sum as cdd_dedisperse, without the
 * coherent (chirp) step, so each channel keeps its intra-channel dispersion
 * smear.  The baseline the coherent path improves on (Sec. 1.2, Fig. 1).
 *   voltages, dtype, nsamp, nchan, f_centre_mhz, bw_mhz, dm, n_int,
 *   intensity, coverage, chan_intensity: as cdd_dedisperse
 *   workspace    device scratch of at least cdd_incoherent_ws_bytes(...)
 *                bytes, 256-byte aligned
 * Errors: EINVAL as cdd_dedisperse (no transform length is involved), short
 * or misaligned workspace; EDEVICE if a launch fails.
 */
size_t cdd_incoherent_ws_bytes(int32_t dtype, int64_t nsamp, int32_t nchan, int32_t n_int);

/* Options.  Zero-initialise; zero fields take the rule-based defaults. */
typedef struct {
  int32_t explicit_plan;   /* 1: use fft_len/overlap/nfront as given        */
  int32_t fft_len;         /* N (power of two); 0 = length rule (Sec. 2.3)  */
  int32_t overlap;         /* L (explicit_plan only)                        */
  int32_t nfront;          /* front discard (explicit_plan only)            */
  double dm_const;         /* D of Eq. 3; 0 = 4.148808e9                    */
  int32_t phase_mode;      /* cdd_phase_mode                                */
  int32_t kernel_variant;  /* block-kernel schedule for this N; 0 = default,
                              1.. = alternatives (cdd_kernel_variants)     */
  int32_t autotune;        /* cdd_plan_create: beams with fft_len 0 get N and
                              schedule from cdd_autotune (2^11 .. 2^14)    */
  int32_t time_chunks;     /* cdd_dedisperse: split the record into this many
                              time chunks so the layout change and aligned
                              sums overlap the block kernel; 0 = automatic,
                              1 = no split                                 */
  int32_t taper;           /* cdd_taper; the plan (N, L, nfront) is the same
                              with or without a taper                      */
  int32_t npol;            /* cdd_dedisperse: polarisations in the record
                              (0 or 1 = one; 2 = two records of the same
                              shape back to back, [2][nsamp][nchan]...):
                              their detected intensities are summed before
                              the delay-aligned sum (Sec. 4.3 and 4.5, one
                              polarisation per host, summed); N <= 16384,
                              nchan > 1, one time chunk, no voltages out   */
  int32_t chirp_in_kernel; /* cdd_plan_*: beams with one DM trial form their
                              chirp inside the batched kernel like beams
                              with several, instead of reading a table built
                              per execute                                  */
  int32_t single_launch;   /* cdd_plan_*: per round of DM tiles, every beam
                              of length <= 8192 (per sample type) in one
                              launch after all layout changes, instead of
                              one launch per beam, each after its own
                              layout change                                */
} cdd_opts;

/* Plan figures for one beam (filled by cdd_query / cdd_plan_info). */
typedef struct {
  int32_t fft_len;     /* N                                                 */
  int32_t overlap;     /* L                                                 */
  int32_t nfront;      /* front discard                                     */
  int32_t step;        /* M = N - L                                         */
  int64_t nblocks;     /* blocks per channel, ceil(nsamp / M)               */
  int64_t t_int;       /* nsamp / n_int                                     */
  int32_t front;       /* ceil of the impulse response's forward reach      */
  int32_t back;        /* ceil of its backward reach                        */
  int64_t d_max;       /* largest channel delay (integrated samples)        */
  size_t ws_bytes;     /* workspace the call needs                          */
} cdd_plan_info;

/*
 * cdd_query -- plan figures and workspace size for cdd_dedisperse.  Host
 * only; touches no device.  Arguments as cdd_dedisperse.  Rules (Sec. 2.2,
 * 2.3): front/back = ceil of the largest forward/backward reach of the
 * chirp's impulse response over the channels, from its group delay at the
 * channel edges; L = next power of two >= front + back (>= 1), raised until
 * n_int divides N - L; nfront = front + (L - front - back) / 2, moved down
 * to a multiple of 16 if that stays >= front; N (if 0) =
 * max(smallest power of two > 2 x the widest channel's dispersion samples,
 * 2L, 256).  EINVAL if N is not a power of two in [256, 2^26], if
 * L >= N ("DM too large for fft_len"), or on any invalid argument below.
 */
cdd_status cdd_query(int32_t dtype, int64_t nsamp, int32_t nchan,
                     double f_centre_mhz, double bw_mhz, double dm,
                     int32_t fft_len, int32_t n_int, int32_t want_voltages,
                     const cdd_opts* opts, cdd_plan_info* info);

/*
 * cdd_dedisperse -- the whole path for one beam and one DM.
 *   voltages     [nsamp][nchan][2] int8 or [nsamp][nchan] complex float
 *   intensity    out, float [t_int]: the delay-aligned sum I
 *   coverage     out, int32 [t_int] or NULL
 *   chan_intensity out, float [nchan][t_int] (P_c) or NULL
 *   volt_out     out, complex float [nchan][nsamp] dedispersed voltages,
 *                channel-major, or NULL
 *   workspace    device scratch of at least info.ws_bytes (cdd_query with
 *                want_voltages = (volt_out != NULL)); 256-byte aligned
 * Errors: EINVAL for nsamp < 1, nchan < 1, n_int < 1, n_int > nsamp,
 * bw <= 0, f_centre - bw/2 <= 0, non-finite DM or frequency, bad dtype or
 * phase mode, a plan rejected by cdd_query, a short or misaligned
 * workspace, NULL voltages or intensity; EDEVICE if a launch fails.
 * Negative DM is allowed (it disperses).
 */
cdd_status cdd_dedisperse(const void* voltages, int32_t dtype, int64_t nsamp,
                          int32_t nchan, double f_centre_mhz, double bw_mhz,
                          double dm, int32_t fft_len, int32_t n_int,
                          float* intensity, int32_t* coverage,
                          float* chan_intensity, void* volt_out,
                          const cdd_opts* opts, void* workspace,
                          size_t ws_bytes, void* stream);
/*
 * cdd_dedisperse_noalloc -- cdd_dedisperse for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation): the same path and results, with the workspace in
 * a static device array of CDD_NOALLOC_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends.  A call issues kernel
 * launches on `stream` only (no auxiliary stream, no stage timing) and
 * never allocates device memory; its first call on a device looks the
 * array up and uploads the transform's FP64-built twiddle tables (into a
 * static table pool).
 *   arguments    as cdd_dedisperse without workspace/ws_bytes; opts may be
 *                NULL; npol and time_chunks above 1 are not taken
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents (nothing needs to start at zero): calls that overlap in time on
 * one GPU race and must be serialised by the caller.
 * Errors: as cdd_dedisperse; EINVAL when the call's workspace (cdd_query's
 * ws_bytes) exceeds CDD_NOALLOC_SCRATCH_BYTES, checked before any launch;
 * ENOTSUP for npol > 1 or time_chunks > 1.
 */
#define CDD_NOALLOC_SCRATCH_BYTES (512u << 20)
cdd_status cdd_dedisperse_noalloc(const void* voltages, int32_t dtype, int64_t nsamp,
                                  int32_t nchan, double f_centre_mhz, double bw_mhz,
                                  double dm, int32_t fft_len, int32_t n_int,
                                  float* intensity, int32_t* coverage,
                                  float* chan_intensity, void* volt_out,
                                  const cdd_opts* opts, void* stream);
cdd_status cdd_incoherent(const void* voltages, int32_t dtype, int64_t nsamp,
                          int32_t nchan, double f_centre_mhz, double bw_mhz,
                          double dm, int32_t n_int, float* intensity,
                          int32_t* coverage, float* chan_intensity,
                          const cdd_opts* opts, void* workspace,
                          size_t ws_bytes, void* stream);

/*
 * cdd_fold -- fold an intensity series at a known period into phase bins
 * (the folded profiles the paper compares in Sec. 4.5).  Sample u goes to bin
 * floor(frac(u / period + phase0) * nbins) (clamped to nbins - 1),
 * frac(x) = x - floor(x), all in FP64; profile[b] is the sum of its samples
 * in ascending u (accumulated in FP64, stored as FP32) and counts[b] their
 * number.
 *   intensity  device float [t_int] (e.g. the output of cdd_dedisperse)
 *   period     in samples of the series, > 1; phase0 in turns, finite
 *   profile    device float [nbins]; counts device int32 [nbins] or NULL
 * Errors: EINVAL for NULL intensity or profile, t_int < 1, nbins < 1,
 * period <= 1 or non-finite period/phase0; EDEVICE if the launch fails.
 */
cdd_status cdd_fold(const float* intensity, int64_t t_int, double period, double phase0,
                    int32_t nbins, float* profile, int32_t* counts, void* stream);

/* ---------------------------------------------------------------------
 * Full-band mode: the paper's own pipeline without sub-banding (Sec. 2.1,
 * 2.3, 3.1).  The recorded voltage beam is a sequence of records, each the
 * first nchan bins (DC upward) of a 2 nchan-point real FFT of the real
 * sampled voltage, as int8 (re, im): [nspec][nchan][2].  The records are
 * inverse transformed back into one real series of nsamp = nspec * 2 nchan
 * samples at 2 bw samples per microsecond (upper sideband: baseband
 * frequency f is sky frequency f_lo + f, f_lo = f_centre - bw/2), which is
 * dedispersed as one band by overlap-save with real transforms of N points:
 * bin j (0 .. N/2) lies f = j bw / (N/2) above f_lo and takes exp(-2 pi i q),
 * q = D*DM*f^2 / (f_lo^2 (f_lo + f)) turns (Eq. 3 about the lower band edge,
 * so the output is referenced to the arrival time at f_lo), times the taper
 * over the band at x = f/bw - 1/2 and 1/N; the imaginary parts at DC and
 * Nyquist are dropped (the series is real).  Block k transforms samples
 * [k M - nfront, k M - nfront + N) and keeps [nfront, nfront + M), M = N - L.
 * Output: y^2 summed over n_int samples, I[u], u < t_int = nsamp / n_int.
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t fft_len;     /* N, real points                                    */
  int32_t overlap;     /* L                                                 */
  int32_t nfront;      /* front discard                                     */
  int32_t step;        /* M = N - L                                         */
  int64_t nsamp;       /* real samples, nspec * 2 nchan                     */
  int64_t nblocks;     /* ceil(nsamp / M)                                   */
  int64_t t_int;       /* nsamp / n_int                                     */
  int32_t front;       /* ceil of the impulse response's forward reach      */
  int32_t back;        /* the same backward (DM < 0)                        */
  size_t ws_bytes;     /* workspace cdd_fullband_dedisperse needs           */
} cdd_fullband_info;

/*
 * cdd_gsb_inverse -- the inverse transform alone (Sec. 3.1, the inverse
 * transform routine; Eq. 4 counts its cost).
 *   spectra  device int8 [nspec][nchan][2], 4-byte aligned
 *   series   device float [nspec * 2 nchan], 8-byte aligned: record t gives
 *            samples [2 nchan t, 2 nchan (t + 1)) = its real inverse DFT with
 *            1/(2 nchan); the Nyquist bin is taken as zero and the imaginary
 *            part of the DC bin is dropped
 * Errors: EINVAL for NULL or misaligned pointers, nspec < 1, nchan not a
 * power of two in [128, 2048]; EDEVICE if the launch fails.
 */
cdd_status cdd_gsb_inverse(const void* spectra, int64_t nspec, int32_t nchan, float* series,
                           void* stream);

/*
 * cdd_fullband_query -- plan figures and workspace size (host only).  Rules
 * in real samples (Sec. 2.2, 2.3): front = ceil of the dispersion samples
 * across the band, D*|DM|*(f_lo^-2 - f_hi^-2) * 2 bw, for DM >= 0 (back = 0;
 * swapped for DM < 0); L = the power of two >= front + back (>= 2), raised
 * until n_int divides N - L; nfront = front + (L - front - back)/2, moved
 * down to a multiple of 32 if that stays >= front, else to
 * the even neighbour inside [front, L - back]; N (if 0) = max(smallest power
 * of two > 2 x the dispersion samples, 2L, 2^16).  opts: dm_const, taper and
 * explicit_plan (fft_len, overlap, nfront even) apply.
 * Errors: EINVAL for nspec < 1, nchan not a power of two in [128, 2048],
 * n_int odd or < 2 or above nsamp, bw <= 0, f_centre - bw/2 <= 0, non-finite
 * values, fft_len not a power of two in [2^16, 2^27], an overlap shorter
 * than the impulse response; ENOTSUP when the rule asks for more than 2^27
 * points, for CDD_PHASE_FP32, npol, kernel_variant or time_chunks.
 */
cdd_status cdd_fullband_query(int64_t nspec, int32_t nchan, double f_centre_mhz, double bw_mhz,
                              double dm, int32_t fft_len, int32_t n_int, const cdd_opts* opts,
                              cdd_fullband_info* info);

/*
 * cdd_fullband_dedisperse -- inverse transform, full-band dedispersion,
 * detection and integration of one recorded beam.
 *   spectra    device int8 [nspec][nchan][2], 4-byte aligned
 *   intensity  out, device float [t_int]
 *   volt_out   out, device float [nsamp], the dedispersed real series, or
 *              NULL (8-byte aligned)
 *   workspace  device scratch of info.ws_bytes, 256-byte aligned (the real
 *              series, one chunk of block spectra and the per-pair y^2)
 * Errors: as cdd_fullband_query, plus NULL or misaligned pointers and a short
 * workspace (EINVAL); EDEVICE if a launch fails.
 */
cdd_status cdd_fullband_dedisperse(const void* spectra, int64_t nspec, int32_t nchan,
                                   double f_centre_mhz, double bw_mhz, double dm,
                                   int32_t fft_len, int32_t n_int, float* intensity,
                                   float* volt_out, const cdd_opts* opts, void* workspace,
                                   size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Batched form: many DM trials on several beams in one launch.  The
 * forward transform of each (beam, channel, block) is computed once and
 * every DM trial reuses it; the chirp is generated on the fly per trial.
 * All trials of a beam share one (N, L, nfront), planned for the largest
 * |DM| of the beam (overlap rules as cdd_query over all its DMs).  By
 * default each beam takes, in turn on the caller's stream, its layout
 * change, its launch (the kernel specialised for its length: a persistent
 * one over its DM tile, or one workgroup per block for a single DM) and
 * its delays and aligned sums; the chirp tables of one-DM beams are built
 * on an auxiliary stream beside the first layout change.  With
 * opts->single_launch, every beam of length 256 .. 8192 (and one sample
 * type) shares one launch per round of DM tiles instead: that length's own
 * kernel when all share one length and chirp form, else one persistent
 * launch, longest work per workgroup first, of a kernel that holds the
 * largest length's register budget (which lowers the occupancy of the
 * short lengths).  A beam with a
 * single DM reads its chirp from a table built once per execute unless
 * opts->chirp_in_kernel asks for the in-kernel chirp.
 * Precision: with the FP64-reduced phase, a tile of three or more trials
 * spaced evenly (DM_i = DM_0 + i step to within 1e-13 of the largest |DM|)
 * at N <= 4096 advances each bin's chirp from trial to trial by a fixed
 * rotation exp(-2 pi i step Q) (Eq. 3 is linear in DM), formed in FP64 and
 * rounded to FP32 once: the chirp of the k-th trial of a tile is then off by
 * up to about k * 1e-7 relative (6e-6 at the 64th), against about 2e-7 when
 * each trial's phase is formed on its own (uneven trials, longer transforms).
 * ------------------------------------------------------------------- */
typedef struct {
  const void* voltages;   /* device, layout as cdd_dedisperse               */
  int32_t dtype;
  int32_t nchan;
  int64_t nsamp;
  double f_centre_mhz;
  double bw_mhz;
  const double* host_dms; /* host array of ndm DMs, copied at create        */
  int32_t ndm;
  int32_t n_int;
  int32_t fft_len;        /* 0 = rule / autotuner                           */
  int32_t reserved;
  float* intensity;       /* device out, float [ndm][t_int]                 */
  int32_t* coverage;      /* device out, int32 [ndm][t_int] or NULL         */
} cdd_beam;

typedef struct cdd_plan cdd_plan;

/* Create a plan (host work only, unless opts->autotune asks the autotuner
 * for beams with fft_len 0; twiddle tables are uploaded on first execute).
 * EINVAL as cdd_query for each beam; ENOMEM. */
cdd_status cdd_plan_create(const cdd_beam* beams, int32_t nbeam,
                           const cdd_opts* opts, cdd_plan** out);
/* Plan figures of one beam (ws_bytes is the whole plan's workspace). */
cdd_status cdd_plan_info_get(const cdd_plan* plan, int32_t beam,
                             cdd_plan_info* info);
/* Enqueue the whole batch on stream.  workspace as for cdd_dedisperse,
 * sized by cdd_plan_info_get().ws_bytes.  The plan may be executed again
 * (same buffers); it must not be executed concurrently with itself. */
cdd_status cdd_plan_execute(cdd_plan* plan, void* workspace, size_t ws_bytes,
                            void* stream);
void cdd_plan_destroy(cdd_plan* plan);

/* ---------------------------------------------------------------------
 * Real-time serving.  A server accepts many concurrent streams, each a
 * voltage beam that arrives in blocks of any size (the paper's pipeline reads
 * consecutive blocks from a ring and must not lose any, Sec. 4.3 and 4.5).
 * Per stream the server keeps, in device memory, the overlap tail of the
 * input (the samples a block loses to overlap-save are prefixed to the next
 * block, Sec. 4.3) and the per-channel intensities still needed by the
 * delay-aligned sum.  A scheduler thread folds every block that is ready,
 * from every stream, into the next launch (one persistent launch for every
 * transform length up to 8192, one per longer length), so streams that
 * arrive while others are on the GPU are
 * served as slots and memory free up, and their work overlaps on the device.
 * The result of a stream depends only on its own data and plan: the same
 * alone or in any mix, and equal to cdd_dedisperse on the whole record.
 * Host pointers below are host memory; the server owns all device memory.
 * ------------------------------------------------------------------- */
typedef struct cdd_server cdd_server;

typedef struct {
  size_t hbm_budget;      /* device bytes open streams may hold; 0 = 8 GiB   */
  int32_t max_streams;    /* 0 = 64                                          */
  int32_t queue_depth;    /* blocks per stream pushed but not yet consumed;
                             0 = 4                                           */
  int32_t reserved[6];
} cdd_server_opts;

typedef struct {
  int32_t dtype;          /* cdd_dtype; blocks are time-major as for
                             cdd_dedisperse                                  */
  int32_t nchan;
  double f_centre_mhz;
  double bw_mhz;
  double dm;
  int32_t fft_len;        /* 0 = length rule; must be <= 16384             */
  int32_t n_int;
  int64_t max_block;      /* largest block a push may carry (samples/chan)   */
  int32_t phase_mode;
  int32_t taper;          /* cdd_taper                                      */
  int64_t block_len;      /* samples per channel of every push but the last
                             (0: pushes of any size).  With it, blocks lost
                             before a push are re-inserted as zeros at their
                             true position, so later outputs keep their
                             absolute indices                               */
  int32_t reserved[2];
} cdd_stream_desc;

typedef struct {
  int64_t blocks_in;      /* blocks accepted                                 */
  int64_t blocks_done;    /* blocks whose results are on the host            */
  int64_t rejected;       /* duplicate or out-of-order pushes refused        */
  int64_t gaps;           /* pushes that skipped sequence numbers            */
  int64_t admitted;       /* streams opened                                  */
  int64_t refused;        /* stream opens refused for budget or slots        */
  int64_t batches;        /* launches formed by the scheduler                */
  double lat_p50_ms;      /* block arrival -> its results on the host        */
  double lat_p99_ms;
  double lat_max_ms;
  double data_s;          /* seconds of data consumed, summed over streams   */
  double wall_s;          /* wall seconds from first push to last completion */
  size_t hbm_used;        /* device bytes held by admitted streams           */
  size_t hbm_budget;
} cdd_server_stats;

/* Create a server on the current device.  ENOMEM, EDEVICE. */
cdd_status cdd_server_create(const cdd_server_opts* opts, cdd_server** out);
/* Finish all queued work, then free everything. */
void cdd_server_destroy(cdd_server* server);
/* Admit a stream (plan as cdd_query with nsamp = max_block).  EAGAIN when
 * its device memory would exceed the budget or all slots are taken; EINVAL
 * as cdd_query; ENOTSUP for fft_len > 16384. */
cdd_status cdd_stream_open(cdd_server* server, const cdd_stream_desc* desc,
                           int32_t* stream_id);
/* Queue the next block: host_block [nsamp][nchan] (time-major), copied
 * before return.  seq must be the stream's next sequence number (first 0):
 * a smaller seq is refused (EINVAL, counted as rejected); a larger one means
 * blocks were lost -- it is accepted and counted as a gap.  With the
 * stream's block_len set, the lost blocks' samples are inserted as zeros at
 * their true position (the result is that of the record with those samples
 * zero); without it the block joins the data before the gap.  Either way the
 * aligned-sum outputs whose inputs include the lost span (or the junction)
 * are reported by cdd_stream_invalid (the paper's real-time check is that
 * no block is lost, Sec. 4.5).  EAGAIN when queue_depth blocks are already
 * waiting (retry later); EINVAL for nsamp < 1 or > max_block (or >
 * block_len, or any push after one shorter than block_len), or a closed
 * stream. */
cdd_status cdd_stream_push(cdd_server* server, int32_t stream_id,
                           const void* host_block, int64_t nsamp, uint64_t seq);
/* Copy up to cap finished samples of the stream's aligned sum I[u] (FP32,
 * in order) to host_out; *n receives the count and *u_first the absolute
 * index of the first.  Samples are finished once every channel's delayed
 * intensity is known (after the dispersion sweep), or at close. */
cdd_status cdd_stream_poll(cdd_server* server, int32_t stream_id, float* host_out,
                           int64_t cap, int64_t* n, int64_t* u_first);
/* Output spans [begin, end) (aligned-sum indices, absolute) whose inputs
 * include lost samples or a junction across lost blocks, in the order the
 * gaps arrived: up to cap pairs into spans[2 i], spans[2 i + 1]; *n receives
 * the number recorded so far.  The span covers every output the lost input
 * can reach through the filter's impulse response, the integration and the
 * channel delays. */
cdd_status cdd_stream_invalid(cdd_server* server, int32_t stream_id, int64_t* spans,
                              int64_t cap, int64_t* n);
/* End of stream: the tail is processed with zeros after the last sample and
 * every I[u], u < total/n_int, becomes available (with partial coverage at
 * the end, as cdd_dedisperse).  The stream's memory is returned to the
 * budget once its last sample has been polled. */
cdd_status cdd_stream_close(cdd_server* server, int32_t stream_id);
/* Wait until every pushed block is finished. */
cdd_status cdd_server_sync(cdd_server* server);
cdd_status cdd_server_stats_get(cdd_server* server, cdd_server_stats* out);

/* ---------------------------------------------------------------------
 * Stage timing.  When enabled, every call records a pair of HIP events on
 * its stream around each kernel it launches; cdd_profile_read waits for the
 * recorded events, returns the accumulated time per stage and starts over.
 * Stages: 0 layout change (time-major -> channel-major), 1 channel delays
 * (and, with one DM, the per-channel chirp table of the block kernel),
 * 2 fused FFT/chirp/IFFT/detect/integrate block kernel, 3 delay-aligned sum.
 * ------------------------------------------------------------------- */
#define CDD_NSTAGES 4
typedef struct {
  double ms[CDD_NSTAGES];     /* summed elapsed milliseconds per stage      */
  int64_t count[CDD_NSTAGES]; /* number of launches timed per stage         */
} cdd_profile;
cdd_status cdd_profile_enable(int32_t on);  /* process-wide switch          */
/* Which stages are timed while enabled: bit s = stage s (default all).  Each
 * timed stage adds two event records to its stream, which cost the device a
 * few microseconds each; timing only the stage of interest keeps a measured
 * run close to an untimed one.  EINVAL for 0 or bits beyond CDD_NSTAGES. */
cdd_status cdd_profile_select(uint32_t stage_mask);
cdd_status cdd_profile_read(cdd_profile* out);

/* ---------------------------------------------------------------------
 * Autotuner: transform length, block-kernel schedule and DM tile for a beam
 * shape, timed in the form a plan runs them.  Every N in [n_min, n_max]
 * (powers of two; 0 = 2^11 and 2^14; at most 2^14, the longest transform a
 * workgroup holds: beyond it the four-step kernels take several passes over
 * HBM per block) for which the overlap fits is timed on the current device
 * on a random int8 record of the beam's channel count.  With one DM trial:
 * the per-execute chirp table and the one-workgroup-per-block kernel.  With
 * several: the persistent batched kernel in each schedule it is compiled
 * for, over tiles of 16, 32 and 64 trials (no more than the beam has).  Two
 * sweeps; the best time per candidate counts; the fastest in input samples
 * x DM trials per second wins.  Results are cached per device and shape in
 * memory, and appended to the text file named by the environment variable
 * CDD_TUNE_CACHE (read back on first use).  Allocates and frees its own
 * device memory and waits for the device.  ENOTSUP for complex-float
 * records.
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t fft_len;
  int32_t kernel_variant;  /* schedule of the kernel that won               */
  double ms;               /* one launch over the timing record              */
  double msamples_per_s;   /* input samples x DM trials per second           */
  int32_t dm_tile;         /* DM trials per launch that won (1 for one DM)   */
  int32_t reserved;
} cdd_tune_result;
cdd_status cdd_autotune(int32_t dtype, int32_t nchan, double f_centre_mhz, double bw_mhz,
                        const double* host_dms, int32_t ndm, int32_t n_int,
                        int32_t n_min, int32_t n_max, cdd_tune_result* best);

/* ---------------------------------------------------------------------
 * Host-side helpers (no device needed)
 * ------------------------------------------------------------------- */
const char* cdd_last_error(void);         /* thread-local, never NULL      */
const char* cdd_status_str(cdd_status s); /* static string                 */
int32_t cdd_abi_version(void);            /* CDD_ABI_VERSION               */
/* Number of block-kernel schedules compiled for transform length N (0 if
 * N is not supported); valid kernel_variant values are 0 .. count-1. */
int32_t cdd_kernel_variants(int32_t fft_len);

#ifdef __cplusplus
}
#endif
#endif /* CDD_H */
