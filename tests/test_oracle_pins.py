"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a missing 1/N, an off-by-one
window) fails at least one of them.  Nothing here uses the HIP library.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Textbook cold-plasma dispersion constant, written independently of the
# oracle: arrival delay of frequency f (MHz) is K_DM*DM/f^2 microseconds.
K_DM_US = 4.148808e9


def arrival_law(dm, f_ref):
    """Physical arrival time (us) of frequency f relative to f_ref."""
    return lambda f: K_DM_US * dm * (1.0 / (f * f) - 1.0 / (f_ref * f_ref))


def direct_idft(X):
    """x[n] = (1/N) sum_j X[j] exp(+2 pi i j n / N), by explicit loops."""
    n = len(X)
    out = np.zeros(n, dtype=np.complex128)
    for t in range(n):
        acc = 0j
        for j in range(n):
            ang = 2.0 * math.pi * ((j * t) % n) / n
            acc += X[j] * complex(math.cos(ang), math.sin(ang))
        out[t] = acc / n
    return out


# --------------------------------------------------------------------------
# Overlap-save machinery: brute-force time-domain evaluation
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,L,nfront,T", [(64, 16, 7, 203), (32, 8, 0, 70),
                                          (64, 20, 20, 64), (16, 4, 3, 1)])
def test_overlap_save_equals_brute_force_block_convolution(N, L, nfront, T):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    H = O.transfer(N, 301.0, 0.5, 3.0)
    h = direct_idft(H)                       # circular impulse response
    M = N - L
    want = np.zeros(T, dtype=np.complex128)
    for k in range(-(-T // M)):
        for m in range(M):
            t = k * M + m
            if t >= T:
                break
            acc = 0j
            for mp in range(N):
                src = k * M - nfront + mp
                if 0 <= src < T:
                    acc += x[src] * h[(nfront + m - mp) % N]
            want[t] = acc
    got = O.overlap_save(x, H, L, nfront)
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))


def test_direct_dft_matches_numpy_convention():
    """The oracle's O(N^2) DFT and numpy agree on sign and scale."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal(24) + 1j * rng.standard_normal(24)
    assert np.allclose(O.dft_direct(x), np.fft.fft(x), atol=1e-11)
    assert np.allclose(direct_idft(np.fft.fft(x)), x, atol=1e-12)


# --------------------------------------------------------------------------
# |H| = 1 (all-pass), DM = 0, round trip
# --------------------------------------------------------------------------
@pytest.mark.parametrize("fc,df,dm,n", [(325.0, 0.0625, 67.9, 8192),
                                        (610.0, 16.0, 10.0, 1 << 14),
                                        (300.02, 0.048828125, -120.0, 4096)])
def test_parseval_per_block(fc, df, dm, n):
    rng = np.random.default_rng(3)
    s = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    z = np.fft.ifft(np.fft.fft(s) * O.transfer(n, fc, df, dm))
    e0, e1 = np.sum(np.abs(s) ** 2), np.sum(np.abs(z) ** 2)
    assert abs(e1 - e0) / e0 < 1e-13
    # and it is not the identity
    assert np.max(np.abs(z - s)) > 0.1


def test_dm_zero_is_identity_and_plain_incoherent_sum():
    rng = np.random.default_rng(4)
    T, C = 1000, 5
    v = rng.integers(-127, 128, size=(T, C, 2)).astype(np.int8)
    out = O.dedisperse(v, 325.0, 1.0, 0.0, n_int=3, fft_len=256, overlap=24,
                       nfront=11, want_voltages=True)
    x = v[..., 0].astype(float) + 1j * v[..., 1].astype(float)
    assert np.max(np.abs(out["y"] - x.T)) < 1e-12
    p = np.abs(x) ** 2
    P = np.array([[p[3 * u:3 * u + 3, c].sum() for u in range(T // 3)] for c in range(C)])
    assert np.allclose(out["P"], P, rtol=0, atol=1e-9)
    assert np.all(out["d"] == 0)
    assert np.allclose(out["I"], P.sum(0)) and np.all(out["cov"] == C)


def test_round_trip_block_level():
    rng = np.random.default_rng(5)
    n = 4096
    s = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    disp = np.fft.ifft(np.fft.fft(s) * O.transfer(n, 330.0, 0.25, 40.0, sign=+1))
    back = np.fft.ifft(np.fft.fft(disp) * O.transfer(n, 330.0, 0.25, 40.0, sign=-1))
    assert np.max(np.abs(back - s)) < 1e-12
    # dedispersing at -DM is dispersing at +DM
    a = O.transfer(n, 330.0, 0.25, -40.0, sign=-1)
    b = O.transfer(n, 330.0, 0.25, 40.0, sign=+1)
    assert np.max(np.abs(a - b)) < 1e-9


# --------------------------------------------------------------------------
# Physics: a dispersed pulse collapses to its emission time
# --------------------------------------------------------------------------
def _smooth(p, w):
    k = np.ones(w) / w
    return np.convolve(p, k, mode="same")


def test_single_channel_pulse_collapses_to_emission_time():
    """Pulse synthesised from wave packets at their physical arrival times
    (centre-referenced) is brought back to t0 by the dedispersing filter,
    and smeared to twice the sweep by the opposite sign."""
    rate, fcen, dm = 4.0, 300.0, 5.0
    nsamp = 1 << 17
    t0_us = 12000.0
    rng = np.random.default_rng(6)
    x = synth.single_pulse_cf32(rng, nsamp, rate, fcen, t0_us,
                                arrival_law(dm, fcen), fwhm_us=40.0, amp=40.0,
                                nsub=128, noise_sigma=0.0)
    # the dispersed signal is spread over the sweep
    sweep = K_DM_US * dm * ((fcen - rate / 2) ** -2 - (fcen + rate / 2) ** -2) * rate
    assert sweep > 20000
    N, L, nfront = O.overlap_plan(fcen, rate, 1, [dm], n_int=1)
    y = O.overlap_save(x, O.transfer(N, fcen, rate, dm), L, nfront)
    p = _smooth(np.abs(y) ** 2, 64)
    t_peak = int(np.argmax(p))
    assert abs(t_peak - t0_us * rate) < 40
    # at least 60% of the pulse energy within +-300 samples of t0
    c = int(t0_us * rate)
    assert np.sum(np.abs(y[c - 300:c + 300]) ** 2) > 0.6 * np.sum(np.abs(y) ** 2)
    # wrong sign: no collapse
    yw = O.overlap_save(x, O.transfer(N, fcen, rate, dm, sign=+1), L, nfront)
    pw = _smooth(np.abs(yw) ** 2, 64)
    assert pw.max() < 0.1 * p.max()


def test_channelised_pulse_arrives_at_delay_and_aligns():
    """Per channel the dedispersed pulse sits at t0 + D DM (f_c^-2 - f_ref^-2);
    after the delay-aligned sum it sits at t0 for every channel."""
    b = synth.Beam(325.0, 2.0, 32, 40000, 60.0, n_int=4, sigma=0.0,
                   period_s=0.0, amp_sigma=1.0, fwhm_s=0.4e-3)
    b.sigma = 1.0
    rng = np.random.default_rng(7)
    fc, df = O.channel_centres(b.f_centre, b.bw, b.nchan)
    t0_us = 120000.0
    data = np.zeros((b.nsamp, b.nchan), dtype=np.complex128)
    for c in range(b.nchan):
        data[:, c] = synth.pulse_channel(rng, b.nsamp, df, fc[c] - df / 2, [t0_us],
                                         arrival_law(b.dm, fc[-1]), 400.0, 30.0, 8)
    out = O.dedisperse(data, b.f_centre, b.bw, b.dm, b.n_int)
    for c in range(0, b.nchan, 5):
        expect = (t0_us + K_DM_US * b.dm * (fc[c] ** -2 - fc[-1] ** -2)) * df / b.n_int
        got = np.argmax(_smooth(out["P"][c], 5))
        assert abs(got - expect) <= 3, (c, got, expect)
    u0 = t0_us * df / b.n_int
    assert abs(np.argmax(_smooth(out["I"], 5)) - u0) <= 2
    # the aligned peak is about nchan times one channel's
    assert out["I"].max() > 0.5 * b.nchan * np.mean([out["P"][c].max() for c in range(b.nchan)])


# --------------------------------------------------------------------------
# Chirp form: full-band chirp = per-channel chirp + delay + constant
# --------------------------------------------------------------------------
@pytest.mark.parametrize("f0,fc,dm", [(309.0, 311.53125, 67.9), (600.0, 615.5, 10.0)])
def test_fullband_chirp_restricted_to_channel_is_channel_chirp_plus_delay(f0, fc, dm):
    f = np.linspace(-0.03, 0.03, 41)
    full = O.chirp_turns((fc - f0) + f, f0, dm)
    chan = O.chirp_turns(f, fc, dm)
    diff = full - chan
    # affine in f: second differences vanish (relative to the phase size)
    d2 = diff[2:] - 2 * diff[1:-1] + diff[:-2]
    assert np.max(np.abs(d2)) < 1e-9 * max(1.0, np.max(np.abs(full)))
    slope = np.polyfit(f, diff, 1)[0]              # turns per MHz = us
    want = K_DM_US * dm * (1.0 / f0 ** 2 - 1.0 / fc ** 2)
    assert abs(slope - want) < 1e-6 * abs(want)


def test_chirp_group_delay_is_cold_plasma_law():
    fc, dm = 327.0, 30.0
    f = np.array([-0.5, -0.1, 0.2, 0.7])
    h = 1e-6
    dq = (O.chirp_turns(f + h, fc, dm) - O.chirp_turns(f - h, fc, dm)) / (2 * h)
    want = K_DM_US * dm * (1.0 / fc ** 2 - 1.0 / (fc + f) ** 2)
    assert np.allclose(dq, want, rtol=1e-6)
    assert np.allclose(O.group_delay_us(f, fc, dm), want, rtol=1e-12)


# --------------------------------------------------------------------------
# Impulse response extent and the overlap / length rules
# --------------------------------------------------------------------------
def test_impulse_response_confined_to_predicted_extent():
    fc, df, dm, n = 309.03125, 0.0625, 67.9, 4096
    front, back = O.wrap_extent(fc, df, dm)
    assert 30 < front < 45 and 30 < back < 45
    h = np.fft.ifft(O.transfer(n, fc, df, dm))
    lag = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)
    inside = (lag >= -math.ceil(back) - 3) & (lag <= math.ceil(front) + 3)
    e = np.abs(h) ** 2
    assert e[inside].sum() > 0.97 * e.sum()
    # both ends are reached: high frequencies delayed (positive lag) by ~front
    assert e[(lag > front - 8) & (lag <= front + 3)].sum() > 0.01 * e.sum()
    assert e[(lag < -back + 8) & (lag >= -back - 3)].sum() > 0.01 * e.sum()


def test_length_rule_reproduces_max_dm_cases():
    """Sec. 4.5's memory-bound DM limits each correspond to the same
    real-sampled transform length under the Sec. 2.3 rule (2^27 points),
    and twice the DM needs the next length."""
    g = json.load(open(os.path.join(GOLDEN, "max_dm_sec4_5.json")))
    for case in g["cases"]:
        f, bw, dm = case["f_mhz"], case["bw_mhz"], case["dm"]
        real_rate = 2.0 * bw
        disp = O.dispersion_samples(f - bw / 2, f + bw / 2, real_rate, dm)
        assert O.fft_len_rule(disp) == 1 << 27, case
        disp2 = O.dispersion_samples(f - bw / 2, f + bw / 2, real_rate, 2.2 * dm)
        assert O.fft_len_rule(disp2) == 1 << 28, case


def test_plan_rule_reproduces_config1_lengths():
    """The workload states FFT length 2^18 and overlap 2^17 for the 16 MHz
    band at 610 MHz and DM 10: the length and overlap rules give both."""
    N, L, nfront = O.overlap_plan(610.0, 16.0, 1, [10.0], n_int=16)
    assert N == 1 << 18 and L == 1 << 17
    front, back = O.wrap_extent(610.0, 16.0, 10.0)
    assert math.ceil(front) <= nfront <= L - math.ceil(back)


@pytest.mark.parametrize("fcen,bw,nchan,dms,n_int,fft", [
    (325.0, 32.0, 512, [67.9], 4, 8192), (400.0, 200.0, 4096, [120.0], 4, 8192),
    (325.0, 32.0, 512, [60.0, 76.0], 4, None), (610.0, 16.0, 512, [-10.0], 3, None),
    (610.0, 16.0, 1, [10.0], 16, None)])
def test_plan_window_lies_inside_uncorrupted_span(fcen, bw, nchan, dms, n_int, fft):
    N, L, nfront = O.overlap_plan(fcen, bw, nchan, dms, n_int, fft)
    fc, df = O.channel_centres(fcen, bw, nchan)
    assert (N - L) % n_int == 0 and N & (N - 1) == 0
    fronts = []
    for dm in dms:
        fr, bk = O.wrap_extent(fc, df, dm)
        assert nfront >= math.ceil(fr) and nfront + (N - L) <= N - math.ceil(bk)
        fronts.append(math.ceil(fr))
    # the window start is a multiple of 16 unless rounding it down would cut
    # into the impulse response's reach
    assert nfront % 16 == 0 or (nfront - nfront % 16) < max(fronts)


# --------------------------------------------------------------------------
# Detection, integration, delays and the aligned sum: brute force
# --------------------------------------------------------------------------
def test_detect_integrate_and_delay_sum_brute_force():
    rng = np.random.default_rng(8)
    C, T, n_int = 4, 23, 3
    y = rng.standard_normal((C, T)) + 1j * rng.standard_normal((C, T))
    P = O.detect_integrate(y, n_int)
    t_int = T // n_int
    assert P.shape == (C, t_int)
    for c in range(C):
        for u in range(t_int):
            s = 0.0
            for r in range(n_int):
                z = y[c, u * n_int + r]
                s += z.real * z.real + z.imag * z.imag
            assert abs(P[c, u] - s) < 1e-12
    d = np.array([5, 0, 2, 9])
    I, cov = O.delay_sum(P, d)
    for u in range(t_int):
        s, n = 0.0, 0
        for c in range(C):
            if u + d[c] < t_int:
                s += P[c, u + d[c]]
                n += 1
        assert abs(I[u] - s) < 1e-12 and cov[u] == n


def test_channel_delays_sign_and_reference():
    d = O.channel_delays(325.0, 32.0, 512, 67.9, 4)
    assert d[-1] == 0 and d[0] > 0 and np.all(np.diff(d) <= 0)
    fc, df = O.channel_centres(325.0, 32.0, 512)
    want0 = K_DM_US * 67.9 * (fc[0] ** -2 - fc[-1] ** -2) * df / 4
    assert abs(d[0] - want0) <= 0.5
    dn = O.channel_delays(325.0, 32.0, 512, -67.9, 4)
    assert dn[0] == 0 and dn[-1] > 0 and np.all(dn >= 0)


def test_channel_centres_tile_the_band():
    fc, df = O.channel_centres(325.0, 32.0, 512)
    assert df == 0.0625 and fc[0] == 309.03125 and fc[-1] == 340.96875
    assert np.allclose(np.diff(fc), df)


def test_nyquist_bin_is_lower_band_edge():
    """Channels are half-open, [f_c - df/2, f_c + df/2); the N/2 bin of a
    channel's transform therefore sits at the lower edge, -df/2."""
    off = O.bin_offsets(16, 2.0)
    assert off[8] == -1.0 and off[7] == 7 * 2.0 / 16 and off.min() == -1.0
    assert off.max() < 1.0


# ---------------------------------------------------------------------------
# Taper windows (Sec. 2.2: the window that turns the inverse transfer
# function into the chirp function)
# ---------------------------------------------------------------------------
def test_hanning_at_zero_dm_is_the_three_tap_smoother():
    """A raised-cosine window over the channel is, in time, y[t] = x[t]/2 +
    (x[t-1] + x[t+1])/4 (the window is 1/2 + (e^{+} + e^{-})/4 in frequency).
    With DM 0 and a block margin of at least one sample each side, the
    whole overlap-save output must equal that three-tap filter exactly
    (zeros before the start and after the end)."""
    rng = np.random.default_rng(11)
    T, N, L, nf = 3000, 256, 8, 4
    x = rng.standard_normal(T) + 1j * rng.standard_normal(T)
    H = O.transfer(N, 300.0, 0.5, 0.0, window="hann")
    y = O.overlap_save(x, H, L, nf)
    xp = np.concatenate(([0], x, [0]))
    ref = 0.5 * xp[1:-1] + 0.25 * (xp[:-2] + xp[2:])
    assert np.max(np.abs(y - ref)) < 1e-12


@pytest.mark.parametrize("window,gains", [("hann", (1.0, 0.5, 0.5, 0.0)),
                                          ("welch", (1.0, 0.75, 0.75, 0.0))])
def test_taper_scales_tones_by_their_place_in_the_channel(window, gains):
    """Pure tones through the DM-0 filter: at the channel centre the gain is
    1, a quarter of the channel width above or below it the window's value
    there, at the lower band edge (the N/2 bin) 0 -- measured on the output amplitude
    in the block interiors, which fixes the window's orientation and edge."""
    T, N, L, nf = 4096, 256, 64, 32
    t = np.arange(T)
    for frac, g in zip((0.0, 0.25, -0.25, -0.5), gains):
        x = np.exp(2j * np.pi * frac * t)
        y = O.overlap_save(x, O.transfer(N, 300.0, 0.5, 0.0, window=window), L, nf)
        mid = slice(N, T - N)
        assert np.allclose(y[mid], g * x[mid], atol=1e-9), (window, frac)


@pytest.mark.parametrize("window", ["hann", "welch"])
def test_tapered_block_energy_is_the_windowed_spectral_energy(window):
    """Parseval with the taper: for every block, the inverse transform's
    energy equals (1/N) sum |w_j S_j|^2 -- the chirp function's magnitude is
    exactly the window and its phase unimodular, at a large DM."""
    rng = np.random.default_rng(12)
    N, fc, df, dm = 2048, 330.0, 0.0625, 60.0
    s = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    S = np.fft.fft(s)
    z = np.fft.ifft(S * O.transfer(N, fc, df, dm, window=window))
    w = O.taper(N, window)
    assert abs(np.sum(np.abs(z) ** 2) - np.sum(np.abs(w * S) ** 2) / N) \
        <= 1e-12 * np.sum(np.abs(S) ** 2) / N


# ---------------------------------------------------------------------------
# Incoherent baseline (Sec. 1.2, the comparison of Fig. 1 on synthetic data)
# ---------------------------------------------------------------------------
def _span50(p):
    """Samples between the 25% and 75% points of the cumulative energy."""
    c = np.cumsum(p) / np.sum(p)
    return int(np.searchsorted(c, 0.75) - np.searchsorted(c, 0.25)) + 1


def test_incoherent_keeps_the_intra_channel_smear_that_coherent_removes():
    """A narrow pulse dispersed across 16 channels of 0.25 MHz at 325 MHz, DM
    60: after the aligned sum the incoherent profile spreads the pulse over
    the intra-channel sweep D DM ((f-df/2)^-2 - (f+df/2)^-2) (about 3.6 ms
    here), the coherent one keeps it within a few pulse widths, and both are
    centred on the emission time.  Without the chirp step the incoherent intensities are the
    coherent ones at DM 0."""
    nchan, df, nsamp, dm, n_int = 16, 0.25, 12_000, 60.0, 4
    fcen = 325.0
    fc, _ = O.channel_centres(fcen, nchan * df, nchan)
    rng = np.random.default_rng(21)
    t0_us = 20_000.0
    data = np.zeros((nsamp, nchan), dtype=np.complex128)
    for c in range(nchan):
        data[:, c] = synth.pulse_channel(rng, nsamp, df, fc[c] - df / 2, [t0_us],
                                         arrival_law(dm, fc[-1]), 60.0, 30.0, 16)
    coh = O.dedisperse(data, fcen, nchan * df, dm, n_int)
    inc = O.incoherent(data, fcen, nchan * df, dm, n_int)
    sweep = np.mean([K_DM_US * dm * ((f - df / 2) ** -2 - (f + df / 2) ** -2) for f in fc])
    us_per_u = n_int / df
    # the middle half of the pulse energy: spread over half the sweep when
    # incoherent (a flat smear; the pulse is a comb of 16 sub-band packets
    # per channel), a few packet widths when coherent
    w_inc = _span50(inc["I"]) * us_per_u
    w_coh = _span50(coh["I"]) * us_per_u
    assert 0.35 * sweep < w_inc < 0.65 * sweep, (w_inc, sweep)
    assert w_coh < 0.1 * sweep, (w_coh, sweep)
    u0 = t0_us / us_per_u
    mid = lambda p: np.searchsorted(np.cumsum(p) / np.sum(p), 0.5)  # noqa: E731
    assert abs(mid(coh["I"]) - u0) <= 3
    assert abs(mid(inc["I"]) - u0) <= 0.05 * sweep / us_per_u
    zero = O.dedisperse(data, fcen, nchan * df, 0.0, n_int, fft_len=256, overlap=1, nfront=0)
    assert np.allclose(inc["P"], zero["P"], rtol=1e-10, atol=1e-9)


# ---------------------------------------------------------------------------
# Folding (Sec. 4.5 compares folded profiles)
# ---------------------------------------------------------------------------
def test_fold_of_an_impulse_train_lands_in_one_bin():
    """Impulses every 37 samples starting at 5, folded with 37 bins at the
    same period and half a bin of phase (so no sample sits on a bin edge):
    every impulse in bin 5, one sample per bin per period."""
    T, P = 37 * 40, 37
    I = np.zeros(T)
    I[5::P] = 1.0
    prof, cnt = O.fold(I, float(P), 0.5 / P, P)
    assert prof[5] == 40 and np.sum(prof) == 40 and np.all(cnt == 40)


def test_fold_conserves_energy_and_counts_at_a_fractional_period():
    rng = np.random.default_rng(31)
    I = rng.random(10_000)
    prof, cnt = O.fold(I, 137.37, 0.29, 64)
    assert abs(np.sum(prof) - np.sum(I)) < 1e-9 and np.sum(cnt) == len(I)
    # a phase step of a whole turn changes nothing; half a turn rotates by nbins/2
    p2, c2 = O.fold(I, 137.37, 1.29, 64)
    assert np.array_equal(c2, cnt) and np.allclose(p2, prof)
    p3, c3 = O.fold(I, 137.37, 0.79, 64)
    assert np.array_equal(np.roll(c3, -32), cnt) or np.sum(np.abs(np.roll(c3, -32) - cnt)) <= 2


def test_coherent_folded_profile_is_sharper_than_incoherent():
    """A pulse train (period 20 ms, 60 us pulses) through 16 channels of
    0.25 MHz at DM 60, folded at its period: the coherent profile's peak bin
    holds a larger share of the energy than the incoherent one (the comparison
    of Sec. 1.2 / Fig. 1 and Sec. 4.5, on synthetic data)."""
    nchan, df, nsamp, dm, n_int = 16, 0.25, 60_000, 60.0, 4
    fcen = 325.0
    fc, _ = O.channel_centres(fcen, nchan * df, nchan)
    rng = np.random.default_rng(22)
    t0s = [20_000.0 + 20_000.0 * i for i in range(10)]
    data = np.zeros((nsamp, nchan), dtype=np.complex128)
    for c in range(nchan):
        data[:, c] = synth.pulse_channel(rng, nsamp, df, fc[c] - df / 2, t0s,
                                         arrival_law(dm, fc[-1]), 60.0, 30.0, 16)
    period_u = 20_000.0 * df / n_int        # integrated samples per period
    coh = O.dedisperse(data, fcen, nchan * df, dm, n_int)
    inc = O.incoherent(data, fcen, nchan * df, dm, n_int)
    pc, _ = O.fold(coh["I"], period_u, 0.0, 128)
    pi, _ = O.fold(inc["I"], period_u, 0.0, 128)
    share = lambda p: p.max() / p.sum()     # noqa: E731
    assert share(pc) > 4 * share(pi), (share(pc), share(pi))
    assert abs(int(np.argmax(pc)) - 0) <= 2 or abs(int(np.argmax(pc)) - 128) <= 2


# ---------------------------------------------------------------------------
# Full-band mode: recorded spectra -> real series -> one long real transform
# (Sec. 2.1 real-sampled band from its lower edge, Sec. 2.3, Sec. 3.1)
# ---------------------------------------------------------------------------
def _real_idft_direct(X, n):
    """x[m] = (1/n) (Re X_0 + Re X_{n/2} (-1)^m + 2 sum_{0<j<n/2} Re(X_j
    exp(2 pi i j m / n))) by explicit loops: the inverse DFT of a Hermitian
    spectrum given by its first n/2 + 1 bins."""
    out = np.zeros(n)
    for m in range(n):
        acc = X[0].real + (X[n // 2].real * (-1) ** m if len(X) > n // 2 else 0.0)
        for j in range(1, n // 2):
            ang = 2.0 * math.pi * ((j * m) % n) / n
            acc += 2.0 * (X[j] * complex(math.cos(ang), math.sin(ang))).real
        out[m] = acc / n
    return out


def test_gsb_inverse_is_the_explicit_real_inverse_sum():
    """Each record's bins 0..nchan-1 (Nyquist absent, DC imaginary part
    dropped) inverse transformed by the explicit real inverse DFT sum, and
    records laid end to end in time order."""
    rng = np.random.default_rng(31)
    nchan, T = 8, 3
    sp = rng.integers(-100, 100, size=(T, nchan, 2)).astype(np.int8)
    x = O.gsb_inverse(sp)
    assert x.shape == (T * 2 * nchan,)
    for t in range(T):
        X = sp[t, :, 0].astype(float) + 1j * sp[t, :, 1].astype(float)
        want = _real_idft_direct(np.append(X, 0.0), 2 * nchan)
        assert np.allclose(x[t * 2 * nchan:(t + 1) * 2 * nchan], want, atol=1e-12)


def test_gsb_inverse_returns_the_recorded_series_but_its_nyquist_term():
    """Records made by a forward real FFT of consecutive 2*nchan-sample
    segments come back as those segments, less the unrecorded Nyquist term
    X_nchan (-1)^m / (2 nchan) of each; a tone at bin c comes back as a
    cosine of c cycles per record."""
    rng = np.random.default_rng(32)
    nchan, T = 16, 5
    x = rng.standard_normal(T * 2 * nchan)
    seg = x.reshape(T, 2 * nchan)
    spec = np.fft.rfft(seg, axis=1)
    back = O.gsb_inverse(spec[:, :nchan])
    m = np.arange(2 * nchan)
    nyq = spec[:, nchan].real[:, None] * ((-1.0) ** m)[None, :] / (2 * nchan)
    assert np.allclose(back, (seg - nyq).reshape(-1), atol=1e-12)
    tone = np.zeros((1, nchan), dtype=complex)
    tone[0, 3] = nchan  # amplitude 1 after the 1/(2 nchan) and the mirror bin
    assert np.allclose(O.gsb_inverse(tone), np.cos(2 * np.pi * 3 * m / (2 * nchan)), atol=1e-12)


@pytest.mark.parametrize("N,L,nfront,T", [(64, 16, 6, 300), (32, 8, 0, 70), (16, 4, 4, 16)])
def test_fullband_overlap_save_equals_brute_force_real_convolution(N, L, nfront, T):
    """Every block of the real overlap-save equals the circular convolution
    of the block with the real impulse response (explicit real inverse DFT
    of the filter), kept from nfront for N - L samples."""
    rng = np.random.default_rng(N + T)
    x = rng.standard_normal(T)
    H = O.fullband_transfer(N, 300.0, 4.0, 0.02)
    h = _real_idft_direct(H, N)
    M = N - L
    want = np.zeros(T)
    for k in range(-(-T // M)):
        s = np.zeros(N)
        for n in range(N):
            t = k * M - nfront + n
            if 0 <= t < T:
                s[n] = x[t]
        for m in range(M):
            if k * M + m < T:
                n = nfront + m
                want[k * M + m] = sum(s[i] * h[(n - i) % N] for i in range(N))
    got = O.overlap_save_real(x, H, N, L, nfront)
    assert np.allclose(got, want, atol=1e-11)


def test_fullband_dm_zero_is_identity():
    rng = np.random.default_rng(33)
    x = rng.standard_normal(5000)
    r = O.fullband_dedisperse(x, 610.0, 16.0, 0.0, 4, fft_len=1024, overlap=64,
                              nfront=20, want_voltages=True)
    assert np.allclose(r["y"], x, atol=1e-12)
    assert np.allclose(r["P"], (x[:5000 // 4 * 4] ** 2).reshape(-1, 4).sum(1))


def test_fullband_filter_delays_each_frequency_to_the_lower_edge_arrival():
    """A real-sampled pulse built from wave packets that arrive at t0 + the
    cold-plasma delay of their frequency relative to the lower band edge
    (earlier for higher frequencies) collapses at t0 after the full-band
    filter, and smears with the opposite sign.  Baseband frequency fb of the
    real series is the sky frequency f_lo + fb (upper sideband)."""
    f_lo, bw, dm = 300.0, 4.0, 5.0
    fs = 2.0 * bw
    nsamp = 1 << 17
    t0 = 14000.0  # us: arrival at f_lo
    law = arrival_law(dm, f_lo)
    sweep_us = -law(f_lo + bw)
    assert sweep_us > 5000
    rng = np.random.default_rng(34)
    t = np.arange(nsamp) / fs
    x = np.zeros(nsamp)
    nsub, sig = 128, 40.0 / 2.3548
    for k in range(nsub):
        fb = (k + 0.5) * bw / nsub
        tau = t0 + law(f_lo + fb)
        env = np.exp(-0.5 * ((t - tau) / sig) ** 2)
        x += env * np.cos(2 * np.pi * fb * (t - tau) + rng.uniform(0, 2 * np.pi))
    N, L, nf = O.fullband_plan(f_lo, bw, dm, 2)
    assert L >= sweep_us * fs
    y = O.overlap_save_real(x, O.fullband_transfer(N, f_lo, bw, dm), N, L, nf)
    p = _smooth(y * y, 64)
    c = int(t0 * fs)
    assert abs(int(np.argmax(p)) - c) < 80
    assert np.sum(y[c - 600:c + 600] ** 2) > 0.5 * np.sum(y * y)
    yw = O.overlap_save_real(x, O.fullband_transfer(N, f_lo, bw, dm, sign=+1), N, L, nf)
    assert _smooth(yw * yw, 64).max() < 0.1 * p.max()


def test_fullband_impulse_response_reaches_forward_by_the_sweep():
    """About the lower edge the dedispersing filter is causal: a delta comes
    out spread over [0, sweep] samples after it (ripple aside), nothing
    before; the plan's front covers the sweep and nfront lies inside it."""
    f_lo, bw, dm = 600.0, 2.0, 30.0
    N, L, nf = O.fullband_plan(f_lo, bw, dm, 2)
    sweep = O.dispersion_samples(f_lo, f_lo + bw, 2 * bw, dm)
    assert math.ceil(sweep) <= nf <= L and nf % 2 == 0
    h = np.fft.irfft(O.fullband_transfer(N, f_lo, bw, dm), n=N)
    e = h * h
    fwd = e[:int(sweep) + 8].sum()
    assert fwd > 0.99 * e.sum()
    assert e[N - 64:].sum() < 1e-3 * e.sum()


def test_fullband_plan_reproduces_the_papers_lengths():
    """The Sec. 2.3 rule on the whole band: 2^19 real points (= the 2^18
    complex of the channel form) and a 2^18 overlap for 16 MHz at 610 MHz,
    DM 10; 2^27 real points for each of Sec. 4.5's memory-bound DM limits."""
    N, L, nf = O.fullband_plan(602.0, 16.0, 10.0, 16)
    assert (N, L) == (1 << 19, 1 << 18)
    g = json.load(open(os.path.join(GOLDEN, "max_dm_sec4_5.json")))
    for case in g["cases"]:
        f, bw, dm = case["f_mhz"], case["bw_mhz"], case["dm"]
        assert O.fullband_plan(f - bw / 2, bw, dm, 2)[0] == 1 << 27, case


def test_fullband_and_gsb_inverse_take_int8_records():
    """The int8 [T][nchan][2] records and the same values as complex give
    the same full-band result."""
    rng = np.random.default_rng(35)
    sp = rng.integers(-60, 60, size=(40, 32, 2)).astype(np.int8)
    cx = sp[..., 0].astype(float) + 1j * sp[..., 1]
    a = O.fullband_dedisperse(sp, 610.0, 16.0, 0.01, 4, fft_len=1024)
    b = O.fullband_dedisperse(cx, 610.0, 16.0, 0.01, 4, fft_len=1024)
    assert np.array_equal(a["P"], b["P"])


def test_fullband_hanning_at_dm_zero_is_the_band_pass_three_tap_filter():
    """Over the band [f_lo, f_lo + bw] the Hanning window is sin^2(pi f/bw)
    = 1/2 - cos(2 pi f/bw)/2; at DM 0 on a real series sampled at 2 bw that
    is y[n] = x[n]/2 - (x[n-2] + x[n+2])/4 (zero at DC and Nyquist)."""
    rng = np.random.default_rng(36)
    x = rng.standard_normal(3000)
    r = O.fullband_dedisperse(x, 610.0, 16.0, 0.0, 2, fft_len=512, overlap=8, nfront=4,
                              window="hann", want_voltages=True)
    want = 0.5 * x[2:-2] - 0.25 * (x[:-4] + x[4:])
    assert np.allclose(r["y"][2:-2], want, atol=1e-12)


@pytest.mark.parametrize("j,gain", [(0, 0.0), (64, 0.75), (128, 1.0), (192, 0.75), (256, 0.0)])
def test_fullband_welch_at_dm_zero_scales_band_tones_by_the_parabola(j, gain):
    """Welch over the band [f_lo, f_lo + bw] is 1 - (2 f/bw - 1)^2 = 4 u (1 - u)
    at u = f/bw (Sec. 2.2's taper written out over the whole band): at DM 0 a
    real tone at bin j of a 512-point transform (u = j/256; its period divides
    every block that lies inside the data, so it is one bin pair in each) comes
    out scaled by 3/4 at a quarter and three quarters of the band, by 1 at the
    centre, and removed at DC and Nyquist.  The first and last blocks see the
    zeros outside the series and are left out."""
    n = np.arange(4000)
    x = np.cos(2.0 * np.pi * j * n / 512.0 + (0.3 if 0 < j < 256 else 0.0))
    r = O.fullband_dedisperse(x, 610.0, 16.0, 0.0, 2, fft_len=512, overlap=8, nfront=4,
                              window="welch", want_voltages=True)
    assert np.allclose(r["y"][512:-512], gain * x[512:-512], atol=1e-11)
