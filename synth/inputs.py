"""Seeded synthetic voltage beams for tests and benchmarks.

This module draws random numbers and lays samples out; it holds none of the
dedispersion arithmetic (no chirp, no transform, no delay law).  Where a
dispersed pulse is wanted, the caller passes the arrival-time law in as a
function, and the pulse is built from narrow sub-band wave packets, each
centred on the arrival time of its own frequency.

Workload shapes follow the observing set-ups of De & Gupta (GMRT 16 and
32 MHz bands, 8-bit voltage samples; Sec. 1.1, 2.3) and the upgraded 200 MHz
band discussed in Sec. 5.  No recorded data is used: these stand in for it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 150900186


@dataclass
class Beam:
    """One channelised voltage beam: centre frequency and bandwidth (MHz),
    channel count, duration in samples per channel, DM and the run options."""
    f_centre: float
    bw: float
    nchan: int
    nsamp: int
    dm: float
    fft_len: int = 0
    n_int: int = 4
    int8: bool = True
    # pulse model
    period_s: float = 0.089
    fwhm_s: float = 0.5e-3
    amp_sigma: float = 0.5
    sigma: float = 20.0
    dms: list = field(default_factory=list)

    @property
    def df(self) -> float:
        return self.bw / self.nchan


def config(k: int) -> Beam:
    """The five workloads by number (1-based)."""
    if k == 1:   # single-channel 16 MHz complex baseband at 610 MHz
        return Beam(610.0, 16.0, 1, 1 << 23, 10.0, fft_len=1 << 18, n_int=16,
                    int8=False, period_s=0.0, fwhm_s=20e-6, amp_sigma=2.7,
                    sigma=1.0)
    if k == 2:   # 32 MHz at 325 MHz, 512 channels of 62.5 kHz, 4 s
        return Beam(325.0, 32.0, 512, 250_000, 67.9, fft_len=8192, n_int=4)
    if k == 3:   # 200 MHz at 400 MHz, 4096 channels, 2 s
        return Beam(400.0, 200.0, 4096, 97_656, 120.0, fft_len=8192, n_int=4)
    if k == 4:   # 64 DM trials on the config-2 beam
        b = config(2)
        b.dms = [60.0 + 0.254 * i for i in range(64)]
        return b
    raise ValueError("no such config")


def extra_beams():
    """The four beams of uneven bandwidth that share one batched launch."""
    return [Beam(610.0, 16.0, 512, 31_250, 10.0),
            Beam(325.0, 32.0, 512, 125_000, 67.9),
            Beam(325.0, 32.0, 1024, 93_750, 67.9),
            Beam(400.0, 200.0, 4096, 195_312, 120.0)]


def scaled(beam: Beam, nchan: int | None = None, nsamp: int | None = None) -> Beam:
    """The same band set-up with fewer channels or samples (same channel
    width when nchan shrinks: the band narrows around the same centre)."""
    b = Beam(**{k: getattr(beam, k) for k in beam.__dataclass_fields__})
    if nchan is not None:
        b.bw = beam.bw * nchan / beam.nchan
        b.nchan = nchan
    if nsamp is not None:
        b.nsamp = nsamp
    return b


def rng_for(k: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k + 1000 * salt)


# --------------------------------------------------------------------------
# Noise
# --------------------------------------------------------------------------
def quantise_int8(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Round half to even, clip to [-127, 127], pack as [..., 2] int8."""
    out = np.empty(re.shape + (2,), dtype=np.int8)
    out[..., 0] = np.clip(np.rint(re), -127, 127)
    out[..., 1] = np.clip(np.rint(im), -127, 127)
    return out


def noise_int8(rng, nsamp: int, nchan: int, sigma: float, chunk: int = 1 << 14):
    """[nsamp][nchan][2] int8 Gaussian voltages (sigma per component)."""
    out = np.empty((nsamp, nchan, 2), dtype=np.int8)
    for t0 in range(0, nsamp, chunk):
        t1 = min(nsamp, t0 + chunk)
        g = rng.standard_normal((t1 - t0, nchan, 2), dtype=np.float32) * sigma
        out[t0:t1] = np.clip(np.rint(g), -127, 127).astype(np.int8)
    return out


def noise_cf32(rng, nsamp: int, sigma: float = 1.0) -> np.ndarray:
    g = rng.standard_normal((nsamp, 2), dtype=np.float32) * sigma
    return (g[:, 0] + 1j * g[:, 1]).astype(np.complex64)


# --------------------------------------------------------------------------
# Pulses built from sub-band wave packets
# --------------------------------------------------------------------------
def pulse_channel(rng, nsamp: int, rate_mhz: float, f_lo: float, t_pulses_us,
                  arrival_us, fwhm_us: float, amp: float, nsub: int) -> np.ndarray:
    """Complex samples of a pulsed signal in one channel [f_lo, f_lo + rate).

    The channel is split into nsub sub-bands.  Sub-band s contributes, per
    pulse p, amp/sqrt(nsub) * g(t - t_p - arrival(f_s)) * n_s(t)
    * exp(2 pi i nu_s t):
    g a Gaussian of the given FWHM, n_s complex noise smoothed by a boxcar of
    nsub samples (bandwidth about rate/nsub, unit variance), nu_s the sub-band
    centre relative to the channel centre, t in samples of this channel.
    """
    y = np.zeros(nsamp, dtype=np.complex128)
    sig = fwhm_us / (2.0 * np.sqrt(2.0 * np.log(2.0))) * rate_mhz   # samples
    half = int(np.ceil(5.0 * sig)) + nsub
    width = 2 * half + 2
    tp = np.asarray(list(t_pulses_us), dtype=np.float64)
    if tp.size == 0:
        return y
    ar = np.arange(width)
    for s in range(nsub):
        nu = (s + 0.5) / nsub * rate_mhz                 # MHz above f_lo
        f_s = f_lo + nu
        nu_c = nu - rate_mhz / 2.0                       # relative to centre
        centre = (tp + arrival_us(f_s)) * rate_mhz       # samples, per pulse
        t = (np.floor(centre).astype(np.int64) - half)[:, None] + ar[None, :]
        w = rng.standard_normal((tp.size, width + nsub - 1, 2))
        wn = (w[..., 0] + 1j * w[..., 1]) / np.sqrt(2.0)
        if nsub > 1:
            c = np.concatenate([np.zeros((tp.size, 1)), np.cumsum(wn, axis=1)], axis=1)
            wn = (c[:, nsub:] - c[:, :-nsub]) / np.sqrt(nsub)
        env = np.exp(-0.5 * ((t - centre[:, None]) / sig) ** 2)
        val = (amp / np.sqrt(nsub)) * env * wn[:, :width] \
            * np.exp(2j * np.pi * nu_c * t / rate_mhz)
        ok = (t >= 0) & (t < nsamp)
        np.add.at(y, t[ok], val[ok])
    return y


def pulse_times_us(beam: Beam, first_us: float | None = None):
    dur = beam.nsamp / beam.df
    if beam.period_s <= 0:
        return [dur / 2.0 if first_us is None else first_us]
    per = beam.period_s * 1e6
    t0 = per / 3.0 if first_us is None else first_us
    return list(np.arange(t0, dur, per))


def make_beam(beam: Beam, rng, arrival_us=None, nsub: int = 8,
              pulse_chans=None) -> np.ndarray:
    """Noise plus (if arrival_us is given) a dispersed pulse train.

    int8 beams: [nsamp][nchan][2] int8, Gaussian noise of sigma per
    component plus pulses of amp_sigma * sigma, rounded half to even once and
    clipped to +-127.  Complex beams: [nsamp][nchan] complex64.
    ``pulse_chans`` limits the pulse synthesis to some channels (speed).
    """
    fc_lo = beam.f_centre - beam.bw / 2.0
    T, C = beam.nsamp, beam.nchan
    if beam.int8:
        g = np.empty((T, C, 2), dtype=np.float32)
        chunk = max(1, (1 << 22) // (2 * C))
        for t0 in range(0, T, chunk):
            t1 = min(T, t0 + chunk)
            g[t0:t1] = rng.standard_normal((t1 - t0, C, 2), dtype=np.float32)
            g[t0:t1] *= np.float32(beam.sigma)
    else:
        data = np.stack([noise_cf32(rng, T, beam.sigma) for _ in range(C)], axis=1)
    if arrival_us is not None and beam.amp_sigma != 0:
        tps = pulse_times_us(beam)
        chans = range(C) if pulse_chans is None else pulse_chans
        for c in chans:
            p = pulse_channel(rng, T, beam.df, fc_lo + c * beam.df, tps, arrival_us,
                              beam.fwhm_s * 1e6, beam.amp_sigma * beam.sigma, nsub)
            nz = np.flatnonzero(p)
            if beam.int8:
                g[nz, c, 0] += p.real[nz].astype(np.float32)
                g[nz, c, 1] += p.imag[nz].astype(np.float32)
            else:
                data[nz, c] += p[nz].astype(np.complex64)
    if not beam.int8:
        return data
    out = np.empty((T, C, 2), dtype=np.int8)
    chunk = max(1, (1 << 24) // (2 * C))
    for t0 in range(0, T, chunk):
        t1 = min(T, t0 + chunk)
        out[t0:t1] = np.clip(np.rint(g[t0:t1]), -127, 127).astype(np.int8)
    return out


def single_pulse_cf32(rng, nsamp: int, rate_mhz: float, f_centre: float,
                      t0_us: float, arrival_us, fwhm_us: float, amp: float,
                      nsub: int, noise_sigma: float = 1.0) -> np.ndarray:
    """One-channel complex baseband: noise plus one dispersed pulse."""
    x = noise_cf32(rng, nsamp, noise_sigma).astype(np.complex128) \
        if noise_sigma > 0 else np.zeros(nsamp, dtype=np.complex128)
    x += pulse_channel(rng, nsamp, rate_mhz, f_centre - rate_mhz / 2.0, [t0_us],
                       arrival_us, fwhm_us, amp, nsub)
    return x
