"""FP64 CPU oracle for overlap-save coherent dedispersion of channelised voltages.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or constants); it reads only numpy.

It is written from De & Gupta, "A Real-time Coherent Dedispersion Pipeline
for the Giant Metrewave Radio Telescope" (Experimental Astronomy), as plainly
as possible: every quantity is computed in float64 with no reduction, no
blocking beyond what overlap-save itself prescribes, and no fusion.  Library
primitives used as steps: ``numpy.fft.fft`` / ``numpy.fft.ifft`` and, for
real series, ``numpy.fft.rfft`` / ``numpy.fft.irfft``.

Readings of the paper that it follows (each is listed with its reason in the
design notes of the repository):

* Chirp (Sec. 2.1, Eq. 3): in turns, q(f) = D*DM*f^2 / (f0^2 (f0 + f)), with
  f0 the reference frequency of the band and f the offset from it, in MHz,
  D = 4.148808e9 (us MHz^2 cm^3 / pc, so q is dimensionless).  The reference
  f0 is the centre of each channel (complex baseband) rather than the lower
  edge of a real-sampled band; the two differ by a delay and a constant phase.
* Sign: the forward FFT uses exp(-2 pi i j n / N); the correcting filter is
  the inverse of the third term of Eq. 2 (Sec. 2.1), i.e. exp(-2 pi i q);
  exp(+2 pi i q) disperses.
* Overlap-save (Sec. 2.2, Sec. 4.3): blocks of N samples at stride M = N - L;
  block k starts at k*M - nfront; of its inverse transform the samples
  [nfront, nfront + M) are kept, the rest (front and end wrap-around) dropped.
* Detection and integration (Sec. 3.1, the write-to-disk routine): |y|^2
  summed over non-overlapping groups of n_int samples starting at sample 0.
* Taper (Sec. 2.2): the chirp function is the inverse transfer function
  multiplied by a window over the band the transform covers (here one
  channel): none (rectangular), Hanning 1/2 (1 + cos 2 pi x) or Welch
  1 - (2 x)^2, with x = f / df the bin's offset from the channel centre as a
  fraction of the channel width, x in [-1/2, 1/2).
* Full-band mode (Sec. 2.1, 2.3, 3.1): the recorded spectra are real-FFT
  outputs; their inverse transforms give back the real series (sampled at
  twice the band), which is dedispersed as one band with the filter of
  Eq. 3 about the lower band edge, by overlap-save with real transforms.
* Incoherent alignment of channels (Sec. 1.2; the linear term of Eq. 2):
  per-channel delay d_c = floor(D*DM*(f_c^-2 - f_ref^-2)*df/n_int + 0.5)
  integrated samples, f_ref the highest channel centre (lowest for DM < 0);
  I[u] = sum over c with u + d_c < T_int of P_c[u + d_c], plus the count.
"""
from __future__ import annotations

import math

import numpy as np

# Sec. 2.1, the constant below Eq. 3 (us MHz^2 cm^3 / pc).
D_PAPER = 4.148808e9


# --------------------------------------------------------------------------
# Frequencies
# --------------------------------------------------------------------------
def channel_centres(f_centre: float, bw: float, nchan: int):
    """Centre frequency (MHz) of each channel and the channel width.

    Channels tile [f_centre - bw/2, f_centre + bw/2) in ascending order
    (upper sideband).  The paper does not state the channel placement
    (Sec. 1.1 describes the FFT channels only); this is the reading used.
    """
    df = bw / nchan
    c = np.arange(nchan, dtype=np.float64)
    return (f_centre - bw / 2.0) + (c + 0.5) * df, df


def bin_offsets(n: int, df: float) -> np.ndarray:
    """Offset from the channel centre (MHz) of each bin of an n-point DFT of
    samples taken at rate df (MHz): bin j < n/2 is +j*df/n, else (j-n)*df/n."""
    j = np.arange(n)
    s = np.where(j < n // 2, j, j - n).astype(np.float64)
    return s * df / n


# --------------------------------------------------------------------------
# Chirp (Sec. 2.1, Eq. 3)
# --------------------------------------------------------------------------
def chirp_turns(f: np.ndarray, f0: float, dm: float, dconst: float = D_PAPER):
    """Dispersive phase of Eq. 3 in turns (cycles): D*DM*f^2/(f0^2 (f0+f))."""
    f = np.asarray(f, dtype=np.float64)
    return dconst * dm * f * f / (f0 * f0 * (f0 + f))


TAPERS = ("none", "hann", "welch")


def taper(n: int, kind: str = "none") -> np.ndarray:
    """Window over the n bins of a channel transform (Sec. 2.2, the taper
    that turns the inverse transfer function into the chirp function).
    x = offset / df in [-1/2, 1/2) for bin j (j < n/2: j/n, else j/n - 1)."""
    j = np.arange(n)
    x = np.where(j < n // 2, j, j - n).astype(np.float64) / n
    if kind == "none":
        return np.ones(n)
    if kind == "hann":
        return 0.5 * (1.0 + np.cos(2.0 * np.pi * x))
    if kind == "welch":
        return 1.0 - (2.0 * x) ** 2
    raise ValueError("unknown taper %r" % kind)


def transfer(n: int, f0: float, df: float, dm: float, dconst: float = D_PAPER,
             sign: int = -1, window: str = "none") -> np.ndarray:
    """The filter on the n bins: exp(sign * 2 pi i q), times the taper.
    sign=-1 dedisperses, sign=+1 disperses.  Evaluated directly in float64;
    without a taper it is all-pass."""
    q = chirp_turns(bin_offsets(n, df), f0, dm, dconst)
    return np.exp(sign * 2j * np.pi * q) * taper(n, window)


# --------------------------------------------------------------------------
# Impulse-response extent, overlap and FFT-length rules (Sec. 2.2, 2.3)
# --------------------------------------------------------------------------
def group_delay_us(f: np.ndarray, f0: float, dm: float, dconst: float = D_PAPER):
    """Delay (us) that the dedispersing filter applies at offset f from f0:
    the derivative of the chirp phase in turns, d q / d f, which equals
    D*DM*(f0^-2 - (f0+f)^-2).  High frequencies are delayed, low advanced."""
    f = np.asarray(f, dtype=np.float64)
    return dconst * dm * (1.0 / (f0 * f0) - 1.0 / ((f0 + f) * (f0 + f)))


def wrap_extent(fc: np.ndarray, df: float, dm: float, dconst: float = D_PAPER):
    """Largest number of samples that the impulse response reaches forward
    (corrupting the front of a block) and backward (corrupting its end), over
    the given channel centres: (front, back), both >= 0, real-valued."""
    fc = np.atleast_1d(np.asarray(fc, dtype=np.float64))
    lo = group_delay_us(-df / 2.0, fc, dm, dconst) * df
    hi = group_delay_us(+df / 2.0, fc, dm, dconst) * df
    front = max(0.0, float(np.max(np.maximum(lo, hi))))
    back = max(0.0, float(np.max(-np.minimum(lo, hi))))
    return front, back


def dispersion_samples(f_lo: float, f_hi: float, rate_mhz: float, dm: float,
                       dconst: float = D_PAPER) -> float:
    """Dispersion time across [f_lo, f_hi] (Sec. 2.2) in samples at the given
    sample rate: D*DM*(f_lo^-2 - f_hi^-2) us times rate (MHz)."""
    return dconst * abs(dm) * (1.0 / (f_lo * f_lo) - 1.0 / (f_hi * f_hi)) * rate_mhz


def next_pow2(x: float) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


def fft_len_rule(disp_samples: float) -> int:
    """Sec. 2.3: the smallest power of two greater than twice the number of
    samples spanned by the dispersion time."""
    p = 1
    while not p > 2.0 * disp_samples:
        p *= 2
    return p


def overlap_plan(f_centre: float, bw: float, nchan: int, dms, n_int: int,
                 fft_len: int | None = None, dconst: float = D_PAPER):
    """(N, L, nfront) shared by a set of DM trials on one beam.

    front/back = ceil of the largest forward/backward reach of the impulse
    response over all channels and DMs; L = the power of two at or above
    front + back (at least 1), raised until n_int divides N - L; nfront =
    front + floor((L - front - back) / 2) (the spare margin centred), then
    moved down to a multiple of 16 if that stays >= front.
    N defaults to the Sec. 2.3 rule on the widest channel dispersion, raised
    to 2L and to 256 if either is larger.
    """
    fc, df = channel_centres(f_centre, bw, nchan)
    dms = np.atleast_1d(np.asarray(dms, dtype=np.float64))
    front = back = 0
    disp = 0.0
    for dm in dms:
        fr, bk = wrap_extent(fc, df, float(dm), dconst)
        front = max(front, math.ceil(fr))
        back = max(back, math.ceil(bk))
        disp = max(disp, float(np.max(
            [dispersion_samples(f - df / 2.0, f + df / 2.0, df, float(dm), dconst)
             for f in (fc[0], fc[-1])])))
    L = next_pow2(max(1, front + back))
    if fft_len is None:
        fft_len = max(fft_len_rule(disp), 2 * L, 256)
    N = int(fft_len)
    while L < N and (N - L) % n_int != 0:
        L += 1
    if L >= N:
        raise ValueError("fft_len too short for this DM: need N > %d" % L)
    nfront = front + (L - front - back) // 2
    if nfront - nfront % 16 >= front:
        nfront -= nfront % 16
    return N, L, nfront


# --------------------------------------------------------------------------
# Overlap-save dedispersion of one channel (Sec. 2.2, 2.3, 4.3)
# --------------------------------------------------------------------------
def overlap_save(x: np.ndarray, H: np.ndarray, L: int, nfront: int) -> np.ndarray:
    """Filter x (complex, [T]) with the N-bin transfer function H by overlap-save.

    Block k holds x[k*M - nfront + n], n < N, with zeros outside [0, T); its
    spectrum is multiplied by H and inverse transformed (with 1/N); samples
    [nfront, nfront + M) of the result become y[k*M : k*M + M).
    """
    x = np.asarray(x, dtype=np.complex128)
    N = H.shape[0]
    M = N - L
    T = x.shape[0]
    y = np.zeros(T, dtype=np.complex128)
    nblk = -(-T // M)
    for k in range(nblk):
        start = k * M - nfront
        s = np.zeros(N, dtype=np.complex128)
        lo = max(0, start)
        hi = min(T, start + N)
        if hi > lo:
            s[lo - start:hi - start] = x[lo:hi]
        z = np.fft.ifft(np.fft.fft(s) * H)
        take = min(M, T - k * M)
        y[k * M:k * M + take] = z[nfront:nfront + take]
    return y


def detect_integrate(y: np.ndarray, n_int: int) -> np.ndarray:
    """|y|^2 summed over consecutive groups of n_int samples from sample 0;
    a trailing partial group is dropped (Sec. 3.1)."""
    p = (y.real * y.real + y.imag * y.imag).astype(np.float64)
    t_int = p.shape[-1] // n_int
    return p[..., :t_int * n_int].reshape(p.shape[:-1] + (t_int, n_int)).sum(-1)


def channel_delays(f_centre: float, bw: float, nchan: int, dm: float, n_int: int,
                   dconst: float = D_PAPER) -> np.ndarray:
    """Integer delay of each channel in integrated samples (Sec. 1.2, linear
    term of Eq. 2): floor(D*DM*(1/f_c^2 - 1/f_ref^2)*df/n_int + 0.5), with
    f_ref the highest channel centre for DM >= 0 and the lowest for DM < 0,
    so every delay is >= 0."""
    fc, df = channel_centres(f_centre, bw, nchan)
    fref = fc[-1] if dm >= 0 else fc[0]
    out = np.empty(nchan, dtype=np.int64)
    for c in range(nchan):
        x = dconst * dm * (1.0 / (fc[c] * fc[c]) - 1.0 / (fref * fref)) * df / n_int
        out[c] = math.floor(x + 0.5)
    return out


def delay_sum(P: np.ndarray, d: np.ndarray):
    """I[u] = sum over channels c with u + d_c < T_int of P[c][u + d_c], in
    channel order, and the number of channels that contributed."""
    nchan, t_int = P.shape
    I = np.zeros(t_int, dtype=np.float64)
    cov = np.zeros(t_int, dtype=np.int64)
    for c in range(nchan):
        dc = int(d[c])
        if dc < t_int:
            I[:t_int - dc] += P[c, dc:]
            cov[:t_int - dc] += 1
    return I, cov


# --------------------------------------------------------------------------
# Whole path
# --------------------------------------------------------------------------
def as_complex(voltages: np.ndarray) -> np.ndarray:
    """[T][C][2] int8 (re, im) or [T][C] / [T] complex -> complex128 [T][C]."""
    v = np.asarray(voltages)
    if v.dtype == np.int8:
        return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)
    v = v.astype(np.complex128)
    return v[:, None] if v.ndim == 1 else v


def dedisperse(voltages, f_centre: float, bw: float, dm: float, n_int: int,
               fft_len: int | None = None, overlap: int | None = None,
               nfront: int | None = None, dconst: float = D_PAPER,
               channels=None, want_voltages: bool = False, sign: int = -1,
               window: str = "none"):
    """Coherent dedispersion of every channel, detection, integration and
    the delay-aligned channel sum.

    voltages: [T][C][2] int8 or [T][C] complex (time-major).  (N, L, nfront)
    default to ``overlap_plan``.  ``channels`` restricts the per-channel work
    to a subset (then I and cov are not formed).  ``window`` selects the
    taper ("none", "hann", "welch").  Returns a dict with
    N, L, nfront, P [C][T_int], and, over all channels, I, cov, d; and y
    [C][T] if asked.
    """
    x = as_complex(voltages)
    T, nchan = x.shape
    if fft_len is None or overlap is None or nfront is None:
        N, L, nf = overlap_plan(f_centre, bw, nchan, [dm], n_int, fft_len, dconst)
        fft_len = fft_len or N
        overlap = L if overlap is None else overlap
        nfront = nf if nfront is None else nfront
    fc, df = channel_centres(f_centre, bw, nchan)
    chans = range(nchan) if channels is None else list(channels)
    out = {"N": fft_len, "L": overlap, "nfront": nfront}
    P = np.zeros((len(chans), T // n_int))
    Y = np.zeros((len(chans), T), dtype=np.complex128) if want_voltages else None
    for i, c in enumerate(chans):
        H = transfer(fft_len, fc[c], df, dm, dconst, sign, window)
        y = overlap_save(x[:, c], H, overlap, nfront)
        P[i] = detect_integrate(y, n_int)
        if want_voltages:
            Y[i] = y
    out["P"] = P
    if want_voltages:
        out["y"] = Y
    if channels is None:
        d = channel_delays(f_centre, bw, nchan, dm, n_int, dconst)
        out["d"] = d
        out["I"], out["cov"] = delay_sum(P, d)
    return out


def incoherent(voltages, f_centre: float, bw: float, dm: float, n_int: int,
               dconst: float = D_PAPER):
    """Incoherent dedispersion (Sec. 1.2): each channel detected and
    integrated as recorded (its intra-channel dispersion left in place),
    then the same delay-aligned sum.  Returns P, I, cov, d."""
    x = as_complex(voltages)
    P = detect_integrate(x.T, n_int)
    nchan = x.shape[1]
    d = channel_delays(f_centre, bw, nchan, dm, n_int, dconst)
    I, cov = delay_sum(P, d)
    return {"P": P, "I": I, "cov": cov, "d": d}


def fold(I: np.ndarray, period: float, phase0: float, nbins: int):
    """Fold a series at a known period (the folded profiles compared in
    Sec. 4.5): sample u goes to bin floor(frac(u / period + phase0) * nbins),
    frac(x) = x - floor(x), clamped to nbins - 1.  Returns the per-bin sums
    (float64, ascending u) and counts."""
    prof = np.zeros(nbins)
    cnt = np.zeros(nbins, dtype=np.int64)
    for u in range(len(I)):
        x = u / period + phase0
        b = min(int(math.floor((x - math.floor(x)) * nbins)), nbins - 1)
        prof[b] += I[u]
        cnt[b] += 1
    return prof, cnt


# --------------------------------------------------------------------------
# Full-band mode: the recorded spectra back to one real series, then one
# long real transform over the whole band (Sec. 2.1, 2.3, 3.1)
# --------------------------------------------------------------------------
def gsb_inverse(spectra) -> np.ndarray:
    """Inverse transform of voltage-beam records (Sec. 2.3; the inverse
    transform routine of Sec. 3.1).  Record t holds bins 0 .. nchan-1 (DC
    first) of a 2*nchan-point real FFT of the real sampled voltage; its
    Nyquist bin is not recorded (taken as zero) and the imaginary part of
    its DC bin is dropped (a real series has a real DC term).  Each record
    is inverse transformed with 1/(2 nchan), so a record made by a forward
    real FFT gives its samples back, and the records are laid end to end.

    spectra: [T][nchan][2] int8 or [T][nchan] complex -> float64 [T*2*nchan].
    """
    X = as_complex(spectra)
    T, nchan = X.shape
    full = np.zeros((T, nchan + 1), dtype=np.complex128)
    full[:, :nchan] = X
    full[:, 0] = full[:, 0].real
    return np.fft.irfft(full, n=2 * nchan, axis=1).reshape(-1)


def band_window(x: np.ndarray, kind: str = "none") -> np.ndarray:
    """The taper of Sec. 2.2 at x = position in the band, in [-1/2, 1/2]."""
    x = np.asarray(x, dtype=np.float64)
    if kind == "none":
        return np.ones_like(x)
    if kind == "hann":
        return 0.5 * (1.0 + np.cos(2.0 * np.pi * x))
    if kind == "welch":
        return 1.0 - (2.0 * x) ** 2
    raise ValueError("unknown taper %r" % kind)


def fullband_transfer(n: int, f_lo: float, bw: float, dm: float, dconst: float = D_PAPER,
                      sign: int = -1, window: str = "none") -> np.ndarray:
    """Filter on the n/2 + 1 bins of an n-point real FFT of the band
    [f_lo, f_lo + bw] sampled at 2 bw (Sec. 2.1: real-sampled band, offsets
    f_l from its lower edge f_o): bin j lies f = j*bw/(n/2) above f_lo and
    takes exp(sign 2 pi i q(f)) with q of Eq. 3 about f_lo; the taper spans
    the band, x = f/bw - 1/2."""
    j = np.arange(n // 2 + 1, dtype=np.float64)
    f = j * (bw / (n // 2))
    q = chirp_turns(f, f_lo, dm, dconst)
    return np.exp(sign * 2j * np.pi * q) * band_window(f / bw - 0.5, window)


def fullband_plan(f_lo: float, bw: float, dm: float, n_int: int,
                  fft_len: int | None = None, dconst: float = D_PAPER):
    """(N, L, nfront) in real samples at rate 2 bw for the full-band filter
    about the lower band edge.  The filter delays every frequency above f_lo
    to f_lo's arrival, so for DM >= 0 its impulse response reaches forward
    only, by the dispersion time across the band (Sec. 2.2): front = ceil of
    it, back = 0 (the other way round for DM < 0).  L = the power of two at or
    above front + back (at least 2), raised until n_int divides N - L; nfront
    = front + floor((L - front - back)/2), moved down to a multiple of 32 if
    that stays >= front, else to an even value inside [front, L - back].  N defaults to the Sec. 2.3 rule, raised to 2L and to
    2^16 (the mode is for long transforms; shorter ones are the channel
    form's).  n_int must be even (integration over pairs of real samples)."""
    if n_int < 2 or n_int % 2:
        raise ValueError("n_int must be even")
    reach = dispersion_samples(f_lo, f_lo + bw, 2.0 * bw, dm, dconst)
    front, back = (math.ceil(reach), 0) if dm >= 0 else (0, math.ceil(reach))
    L = next_pow2(max(2, front + back))
    if fft_len is None:
        fft_len = max(fft_len_rule(reach), 2 * L, 1 << 16)
    N = int(fft_len)
    while L < N and (N - L) % n_int != 0:
        L += 1
    if L >= N:
        raise ValueError("fft_len too short for this DM: need N > %d" % L)
    nf = front + (L - front - back) // 2
    if nf - nf % 32 >= front:
        nf -= nf % 32
    elif nf % 2:
        nf = nf + 1 if nf + 1 <= L - back else nf - 1
    return N, L, nf


def overlap_save_real(x: np.ndarray, H: np.ndarray, N: int, L: int, nfront: int) -> np.ndarray:
    """overlap_save for a real series: each block's real FFT (N/2 + 1 bins)
    is multiplied by H and inverse real transformed (the imaginary parts a
    real series cannot carry at DC and Nyquist are dropped)."""
    x = np.asarray(x, dtype=np.float64)
    M = N - L
    T = x.shape[0]
    y = np.zeros(T)
    for k in range(-(-T // M)):
        start = k * M - nfront
        s = np.zeros(N)
        lo, hi = max(0, start), min(T, start + N)
        if hi > lo:
            s[lo - start:hi - start] = x[lo:hi]
        z = np.fft.irfft(np.fft.rfft(s) * H, n=N)
        take = min(M, T - k * M)
        y[k * M:k * M + take] = z[nfront:nfront + take]
    return y


def fullband_dedisperse(spectra, f_centre: float, bw: float, dm: float, n_int: int,
                        fft_len: int | None = None, overlap: int | None = None,
                        nfront: int | None = None, dconst: float = D_PAPER,
                        window: str = "none", sign: int = -1, want_voltages: bool = False):
    """The paper's unchannelised mode: recorded spectra -> real series
    (gsb_inverse) -> overlap-save with the full-band chirp about the lower
    band edge (real samples at 2 bw) -> y^2 integrated over n_int samples.
    ``spectra`` may also be a real float series (then taken as is).
    Returns N, L, nfront, P [T/n_int], and x, y if asked."""
    a = np.asarray(spectra)
    x = a.astype(np.float64) if a.ndim == 1 and not np.iscomplexobj(a) else gsb_inverse(a)
    f_lo = f_centre - bw / 2.0
    if fft_len is None or overlap is None or nfront is None:
        N, L, nf = fullband_plan(f_lo, bw, dm, n_int, fft_len, dconst)
        fft_len = fft_len or N
        overlap = L if overlap is None else overlap
        nfront = nf if nfront is None else nfront
    H = fullband_transfer(fft_len, f_lo, bw, dm, dconst, sign, window)
    y = overlap_save_real(x, H, fft_len, overlap, nfront)
    t_int = y.shape[0] // n_int
    P = (y[:t_int * n_int] ** 2).reshape(t_int, n_int).sum(-1)
    out = {"N": fft_len, "L": overlap, "nfront": nfront, "P": P}
    if want_voltages:
        out["x"], out["y"] = x, y
    return out


def dft_direct(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """O(N^2) discrete Fourier transform by explicit sums (small N only)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    out = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        acc = 0j
        for m in range(n):
            acc += x[m] * complex(math.cos(2 * math.pi * k * m / n),
                                  sign * math.sin(2 * math.pi * k * m / n))
        out[k] = acc
    return out
