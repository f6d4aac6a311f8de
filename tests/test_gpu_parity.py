"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (stated as relative L2 against the oracle): dedispersed voltages
<= 1e-5, intensities (per channel and the aligned sum) <= 1e-4; coverage
counts and delays exact.  Every input is seeded and synthetic.
"""
import numpy as np
import pytest

import oracle as O
import synth
from tests.util import arrival_law, flush, rel_l2, to_dev

pytestmark = pytest.mark.gpu

TOL_V, TOL_I = 1e-5, 1e-4


def _cdd():
    import paper_1509_00186_amd as cdd
    return cdd


def _run_both(v, fcen, bw, dm, n_int, fft_len=0, phase_mode=0, want_v=True, taper="none",
              **plan):
    import torch
    cdd = _cdd()
    flush("case: shape=%s dtype=%s fcen=%g bw=%g dm=%g n_int=%d N=%d phase=%d taper=%s" %
          (tuple(v.shape), v.dtype, fcen, bw, dm, n_int, fft_len, phase_mode, taper))
    g = cdd.dedisperse(to_dev(v), fcen, bw, dm, fft_len, n_int, want_chan=True,
                       want_voltages=want_v, phase_mode=phase_mode, taper=taper, **plan)
    torch.cuda.synchronize()
    info = g["info"]
    o = O.dedisperse(v, fcen, bw, dm, n_int, fft_len=info["fft_len"],
                     overlap=info["overlap"], nfront=info["nfront"], want_voltages=want_v,
                     window=taper)
    got = {k: g[k].cpu().numpy() for k in ("I", "cov", "P") + (("y",) if want_v else ())}
    return got, o, info


def _check(got, o, tol_v=TOL_V, tol_i=TOL_I):
    if "y" in got:
        assert rel_l2(got["y"], o["y"]) <= tol_v, rel_l2(got["y"], o["y"])
    assert rel_l2(got["P"], o["P"]) <= tol_i, rel_l2(got["P"], o["P"])
    assert rel_l2(got["I"], o["I"]) <= tol_i, rel_l2(got["I"], o["I"])
    assert np.array_equal(got["cov"], o["cov"])


def _beam_int8(seed, nsamp, nchan, fcen, bw, dm, pulse=True):
    b = synth.Beam(fcen, bw, nchan, nsamp, dm, period_s=0.02, fwhm_s=0.3e-3)
    rng = np.random.default_rng(seed)
    fc, _ = O.channel_centres(fcen, bw, nchan)
    return synth.make_beam(b, rng, arrival_law(dm, fc[-1]) if pulse else None)


@pytest.mark.parametrize("N", [256, 512, 1024, 2048, 4096, 8192, 16384])
def test_every_block_length_int8(N):
    # channel width chosen so the impulse response fits N/8 at this DM
    nchan, fcen, dm = 6, 330.0, 25.0
    df = {256: 0.02, 512: 0.03, 1024: 0.04, 2048: 0.05, 4096: 0.0625, 8192: 0.08,
          16384: 0.1}[N]
    M_guess = N - N // 8
    nsamp = 3 * M_guess + 777
    v = _beam_int8(10 + N, nsamp, nchan, fcen, df * nchan, dm)
    got, o, info = _run_both(v, fcen, df * nchan, dm, 4, N)
    assert info["fft_len"] == N
    _check(got, o)


def test_cf32_single_channel_no_transpose():
    rng = np.random.default_rng(21)
    x = (rng.standard_normal(20_011) + 1j * rng.standard_normal(20_011)).astype(np.complex64)
    got, o, _ = _run_both(x, 600.0, 2.0, 3.0, 2, 4096)
    _check(got, o)


def test_cf32_multichannel_ragged_channels():
    rng = np.random.default_rng(22)
    x = (rng.standard_normal((9_000, 67)) + 1j * rng.standard_normal((9_000, 67)))
    x = x.astype(np.complex64) * 7.0
    got, o, _ = _run_both(x, 325.0, 67 * 0.0625, 40.0, 3, 2048)
    _check(got, o)


def test_negative_dm_and_odd_integration():
    v = _beam_int8(23, 15_001, 16, 325.0, 1.0, -30.0, pulse=False)
    got, o, info = _run_both(v, 325.0, 1.0, -30.0, 5, 1024)
    assert (info["fft_len"] - info["overlap"]) % 5 == 0
    _check(got, o)


def test_dm_zero_returns_input():
    v = _beam_int8(24, 5000, 3, 325.0, 0.5, 0.0, pulse=False)
    got, o, _ = _run_both(v, 325.0, 0.5, 0.0, 1, 512)
    x = (v[..., 0].astype(float) + 1j * v[..., 1]).T
    assert rel_l2(got["y"], x) < 1e-6
    _check(got, o)


def test_tiny_and_edge_shapes():
    # one sample, n_int = nsamp
    v = _beam_int8(25, 1, 1, 325.0, 0.0625, 10.0, pulse=False)
    got, o, _ = _run_both(v, 325.0, 0.0625, 10.0, 1, 256)
    _check(got, o)
    # fewer samples than one block step, integration longer than a block
    v = _beam_int8(26, 700, 65, 325.0, 65 * 0.0625, 10.0, pulse=False)
    got, o, _ = _run_both(v, 325.0, 65 * 0.0625, 10.0, 700, 1024)
    _check(got, o)
    # explicit plan: off-centre window
    v = _beam_int8(27, 3000, 2, 325.0, 0.125, 10.0, pulse=False)
    q = _cdd().query(0, 3000, 2, 325.0, 0.125, 10.0, 512, 2)
    nf = q["front"] + 1
    got, o, info = _run_both(v, 325.0, 0.125, 10.0, 2, 512, overlap=q["overlap"], nfront=nf)
    assert info["nfront"] == nf
    _check(got, o)


def test_phase_fp32_variant_error_is_reported_not_hidden():
    v = _beam_int8(28, 20_000, 8, 400.0, 8 * 0.048828125, 120.0)
    got64, o, _ = _run_both(v, 400.0, 8 * 0.048828125, 120.0, 4, 8192, phase_mode=0)
    got32, _, _ = _run_both(v, 400.0, 8 * 0.048828125, 120.0, 4, 8192, phase_mode=1)
    e64, e32 = rel_l2(got64["y"], o["y"]), rel_l2(got32["y"], o["y"])
    flush("voltage rel L2: fp64-reduced %.3g  fp32 phase %.3g" % (e64, e32))
    assert e64 <= TOL_V
    assert e32 > e64          # the FP32 phase is measurably worse
    assert rel_l2(got32["I"], o["I"]) <= 1e-3


@pytest.mark.parametrize("window", ["hann", "welch"])
def test_taper_one_dm_against_oracle(window):
    """Tapered chirp function (Sec. 2.2) through the one-DM path (table
    built per call): voltages, per-channel and aligned intensities."""
    v = _beam_int8(130, 30_000, 24, 325.0, 24 * 0.0625, 67.9)
    import torch
    cdd = _cdd()
    g = cdd.dedisperse(to_dev(v), 325.0, 24 * 0.0625, 67.9, 2048, 4, want_chan=True,
                       want_voltages=True, taper=window)
    torch.cuda.synchronize()
    info = g["info"]
    o = O.dedisperse(v, 325.0, 24 * 0.0625, 67.9, 4, fft_len=2048, overlap=info["overlap"],
                     nfront=info["nfront"], want_voltages=True, window=window)
    got = {k: g[k].cpu().numpy() for k in ("I", "cov", "P", "y")}
    _check(got, o)
    # the taper changes the result (it is not silently ignored)
    plain = O.dedisperse(v, 325.0, 24 * 0.0625, 67.9, 4, fft_len=2048,
                         overlap=info["overlap"], nfront=info["nfront"])
    assert rel_l2(got["I"], plain["I"]) > 1e-3


@pytest.mark.parametrize("dms", [[10.0, 11.5, 8.0], [8.0, 9.5, 11.0, 12.5]],
                         ids=["uneven", "evenly_spaced"])
@pytest.mark.parametrize("window", ["hann", "welch"])
def test_taper_batched_dm_trials_against_oracle(window, dms):
    """The taper in the chirp generated inside the persistent batched kernel,
    with the per-trial phase (uneven DMs) and the rotation step (evenly
    spaced DMs)."""
    import torch
    cdd = _cdd()
    v = _beam_int8(131, 12_000, 16, 610.0, 16 * 0.03125, 10.0)
    plan = cdd.Plan([dict(voltages=to_dev(v), f_centre=610.0, bw=0.5, dms=dms, n_int=2,
                          fft_len=1024)], taper=window)
    plan.execute()
    torch.cuda.synchronize()
    info = plan.info(0)
    for i, dm in enumerate(dms):
        o = O.dedisperse(v, 610.0, 0.5, dm, 2, fft_len=1024, overlap=info["overlap"],
                         nfront=info["nfront"], window=window)
        assert rel_l2(plan.I[0][i].cpu().numpy(), o["I"]) <= TOL_I, (window, dm)
    plan.close()


def test_taper_long_transform_against_oracle():
    """Hanning taper on the four-step path (N = 2^15)."""
    N = 1 << 15
    rng = np.random.default_rng(132)
    nsamp = 2 * N + 777
    x = (rng.standard_normal(nsamp) + 1j * rng.standard_normal(nsamp)).astype(np.complex64)
    got, o, info = _run_both(x, 300.0, 4.0, 1.5, 8, N, taper="hann")
    assert info["fft_len"] == N
    _check(got, o)


def test_incoherent_against_oracle():
    """Incoherent dedispersion (no coherent step): per-channel intensities
    exactly (int8 squares sum exactly in FP32), the aligned sum and coverage."""
    import torch
    cdd = _cdd()
    v = _beam_int8(150, 21_001, 40, 325.0, 40 * 0.0625, 67.9)
    g = cdd.incoherent(to_dev(v), 325.0, 40 * 0.0625, 67.9, 4, want_chan=True)
    torch.cuda.synchronize()
    o = O.incoherent(v, 325.0, 40 * 0.0625, 67.9, 4)
    assert np.array_equal(g["P"].cpu().numpy().astype(np.float64), o["P"])
    assert rel_l2(g["I"].cpu().numpy(), o["I"]) <= 1e-6
    assert np.array_equal(g["cov"].cpu().numpy(), o["cov"])
    # complex-float, one channel: the input is read in place
    rng = np.random.default_rng(151)
    x = (rng.standard_normal(5003) + 1j * rng.standard_normal(5003)).astype(np.complex64)
    g = cdd.incoherent(to_dev(x), 610.0, 16.0, 10.0, 7)
    torch.cuda.synchronize()
    o = O.incoherent(x, 610.0, 16.0, 10.0, 7)
    assert rel_l2(g["I"].cpu().numpy(), o["I"]) <= 1e-6


def test_fold_against_oracle():
    """Folding on the GPU: counts exact, per-bin sums (ascending u, FP64
    accumulation) against the FP64 oracle, at integer and fractional periods
    and with a single bin holding the whole series."""
    import torch
    cdd = _cdd()
    rng = np.random.default_rng(170)
    I = rng.random(62_500).astype(np.float32) * 1000
    for period, phase0, nbins in ((1390.625, 0.3, 128), (37.0, -2.25, 37), (5000.5, 0.0, 1)):
        prof, cnt = cdd.fold(to_dev(I), period, phase0, nbins)
        torch.cuda.synchronize()
        op, oc = O.fold(I.astype(np.float64), period, phase0, nbins)
        assert np.array_equal(cnt.cpu().numpy(), oc), (period, nbins)
        assert rel_l2(prof.cpu().numpy(), op) <= 1e-6, (period, nbins)


def test_two_polarisations_sum_their_intensities():
    """npol = 2: two records back to back; per-channel and aligned
    intensities equal the oracle's sums over the two polarisations."""
    import torch
    cdd = _cdd()
    fcen, nchan, df, nsamp, dm, N = 325.0, 32, 0.0625, 30_000, 67.9, 2048
    p0 = _beam_int8(180, nsamp, nchan, fcen, nchan * df, dm)
    p1 = _beam_int8(181, nsamp, nchan, fcen, nchan * df, dm)
    both = np.ascontiguousarray(np.stack([p0, p1]))
    g = cdd.dedisperse(to_dev(both), fcen, nchan * df, dm, N, 4, want_chan=True, npol=2)
    torch.cuda.synchronize()
    info = g["info"]
    o0 = O.dedisperse(p0, fcen, nchan * df, dm, 4, fft_len=N, overlap=info["overlap"],
                      nfront=info["nfront"])
    o1 = O.dedisperse(p1, fcen, nchan * df, dm, 4, fft_len=N, overlap=info["overlap"],
                      nfront=info["nfront"])
    assert rel_l2(g["P"].cpu().numpy(), o0["P"] + o1["P"]) <= TOL_I
    assert rel_l2(g["I"].cpu().numpy(), o0["I"] + o1["I"]) <= TOL_I
    assert np.array_equal(g["cov"].cpu().numpy(), o0["cov"])
    with pytest.raises(cdd.CddError):
        cdd.dedisperse(to_dev(both), fcen, nchan * df, dm, N, 4, npol=2, time_chunks=2)


@pytest.mark.parametrize("chunks", [1, 3, 8, 12])
def test_time_chunks_do_not_change_results(chunks):
    """The record split that overlaps the layout change and the aligned sums
    with the block kernel (uneven splits included) gives bit-identical
    outputs, which match the oracle."""
    import torch
    cdd = _cdd()
    fcen, nchan, df, nsamp, dm, N = 325.0, 96, 0.0625, 70_001, 67.9, 2048
    v = _beam_int8(120, nsamp, nchan, fcen, nchan * df, dm)
    vd = to_dev(v)
    ref = cdd.dedisperse(vd, fcen, nchan * df, dm, N, 4, want_chan=True, time_chunks=2)
    g = cdd.dedisperse(vd, fcen, nchan * df, dm, N, 4, want_chan=True, time_chunks=chunks)
    torch.cuda.synchronize()
    for k in ("I", "cov", "P"):
        assert torch.equal(g[k], ref[k]), k
    info = g["info"]
    o = O.dedisperse(v, fcen, nchan * df, dm, 4, fft_len=N, overlap=info["overlap"],
                     nfront=info["nfront"], channels=[0, 50, 95])
    assert rel_l2(g["P"].cpu().numpy()[[0, 50, 95]], o["P"]) <= TOL_I
    d = O.channel_delays(fcen, nchan * df, nchan, dm, 4)
    I, cov = O.delay_sum(g["P"].cpu().numpy().astype(np.float64), d)
    assert rel_l2(g["I"].cpu().numpy(), I) <= 1e-5
    assert np.array_equal(g["cov"].cpu().numpy(), cov)


def test_batched_dm_trials_equal_single_calls_and_oracle():
    import torch
    cdd = _cdd()
    fcen, bw, nchan, nsamp, n_int = 325.0, 16 * 0.0625, 16, 30_000, 4
    dms = [60.0 + 0.254 * i * 8 for i in range(8)]
    v = _beam_int8(30, nsamp, nchan, fcen, bw, 67.9)
    vd = to_dev(v)
    plan = cdd.Plan([dict(voltages=vd, f_centre=fcen, bw=bw, dms=dms, n_int=n_int,
                          fft_len=4096)])
    info = plan.info(0)
    plan.execute()
    torch.cuda.synchronize()
    for i, dm in enumerate(dms):
        one = cdd.dedisperse(vd, fcen, bw, dm, 4096, n_int, overlap=info["overlap"],
                             nfront=info["nfront"])
        torch.cuda.synchronize()
        a, b1 = plan.I[0][i].cpu().numpy(), one["I"].cpu().numpy()
        assert rel_l2(a, b1) <= 1e-6
        o = O.dedisperse(v, fcen, bw, dm, n_int, fft_len=4096, overlap=info["overlap"],
                         nfront=info["nfront"])
        assert rel_l2(a, o["I"]) <= TOL_I
        assert np.array_equal(plan.cov[0][i].cpu().numpy(), o["cov"])
    plan.close()


def test_multi_beam_plan_uneven_beams():
    import torch
    cdd = _cdd()
    beams, raw = [], []
    for k, (fcen, nchan, df, nsamp, dm) in enumerate([(610.0, 8, 0.03125, 12_000, 10.0),
                                                      (325.0, 24, 0.0625, 9_000, 67.9)]):
        v = _beam_int8(40 + k, nsamp, nchan, fcen, nchan * df, dm)
        raw.append((v, fcen, nchan * df, [dm, dm + 1.5, dm - 2.0]))
        beams.append(dict(voltages=to_dev(v), f_centre=fcen, bw=nchan * df,
                          dms=[dm, dm + 1.5, dm - 2.0], n_int=2))
    plan = cdd.Plan(beams)
    plan.execute()
    torch.cuda.synchronize()
    for bi, (v, fcen, bw, dms) in enumerate(raw):
        info = plan.info(bi)
        for i, dm in enumerate(dms):
            o = O.dedisperse(v, fcen, bw, dm, 2, fft_len=info["fft_len"],
                             overlap=info["overlap"], nfront=info["nfront"])
            assert rel_l2(plan.I[bi][i].cpu().numpy(), o["I"]) <= TOL_I
            assert np.array_equal(plan.cov[bi][i].cpu().numpy(), o["cov"])
    plan.close()


# ---------------------------------------------------------------------------
# Long transforms (four-step kernels, N >= 2^15)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lgN", [15, 16, 17, 19, 20, 21, 22, 23, 24])
def test_long_transform_lengths_cf32(lgN):
    N = 1 << lgN
    fcen, bw = 300.0, 4.0
    dm = 1.5 * N / (1 << 15)          # impulse response about N/4 samples
    nsamp = 2 * N + N // 2 + 1234
    rng = np.random.default_rng(50 + lgN)
    x = (rng.standard_normal(nsamp) + 1j * rng.standard_normal(nsamp)).astype(np.complex64)
    got, o, info = _run_both(x, fcen, bw, dm, 8, N)
    assert info["fft_len"] == N
    _check(got, o)


@pytest.mark.parametrize("n_int,odd_start", [(16, True), (16, False), (3, False)])
def test_three_level_transform_2_26_cf32(n_int, odd_start):
    """2^26-point transforms (rows of 2^11, columns split 2^8 x 2^7): two
    blocks, the second ragged; integration fused into the last column pass,
    with an odd window start (groups split between its runs) or the rule's
    (a multiple of 16: none split), or the separate integration (n_int 3)."""
    N = 1 << 26
    fcen, bw, dm = 300.0, 4.0, 3072.0
    q = _cdd().query(1, 1000, 1, fcen, bw, dm, N, n_int)
    nsamp = q["step"] + 12_345
    rng = np.random.default_rng(77 + n_int + odd_start)
    x = (rng.standard_normal(nsamp) + 1j * rng.standard_normal(nsamp)).astype(np.complex64)
    plan = dict(overlap=q["overlap"], nfront=q["nfront"] | 1) if odd_start else {}
    got, o, info = _run_both(x, fcen, bw, dm, n_int, N, **plan)
    assert (info["fft_len"], info["nblocks"]) == (N, 2)
    assert (info["nfront"] % 16 != 0) == odd_start
    _check(got, o)


def test_short_record_on_a_long_transform_stays_inside_its_workspace():
    """A record far shorter than its transform (1000 samples, N = 2^15) with
    integration groups split across the fused pass's runs: every partial sum
    lands inside the workspace (a canary after it is untouched) and the
    results match the oracle."""
    import torch
    cdd = _cdd()
    N, n_int = 1 << 15, 4
    rng = np.random.default_rng(79)
    x = (rng.standard_normal(1000) + 1j * rng.standard_normal(1000)).astype(np.complex64)
    q = cdd.query(1, 1000, 1, 300.0, 4.0, 0.5, N, n_int, want_voltages=True)
    L, nfront = q["overlap"], q["nfront"] | 1
    q = cdd.query(1, 1000, 1, 300.0, 4.0, 0.5, N, n_int, want_voltages=True,
                  overlap=L, nfront=nfront)
    ws = torch.full((q["ws_bytes"] + (1 << 20),), 0x5A, dtype=torch.uint8, device="cuda")
    flush("case: short record N=2^15 nfront=%d ws=%d" % (nfront, q["ws_bytes"]))
    g = cdd.dedisperse(to_dev(x), 300.0, 4.0, 0.5, N, n_int, want_chan=True,
                       want_voltages=True, overlap=L, nfront=nfront, out={"ws": ws})
    torch.cuda.synchronize()
    assert bool((ws[q["ws_bytes"]:] == 0x5A).all())
    o = O.dedisperse(x, 300.0, 4.0, 0.5, n_int, fft_len=N, overlap=L, nfront=nfront,
                     want_voltages=True)
    _check({k: g[k].cpu().numpy() for k in ("I", "cov", "P", "y")}, o)


def test_long_transform_multichannel_int8():
    v = _beam_int8(60, 70_000, 3, 300.0, 3 * 1.0, 3.0, pulse=False)
    got, o, info = _run_both(v, 300.0, 3.0, 3.0, 4, 1 << 15)
    _check(got, o)


def test_config1_full_size_and_pulse():
    """2^23 complex samples of a 16 MHz band at 610 MHz, one pulse dispersed
    at DM 10; N = 2^18, L = 2^17: voltages and intensities against the
    oracle, and the dedispersed pulse back at its emission time."""
    import torch
    cdd = _cdd()
    b = synth.config(1)
    t0_us = (1 << 22) / b.bw
    rng = synth.rng_for(1)
    x = synth.single_pulse_cf32(rng, b.nsamp, b.bw, b.f_centre, t0_us,
                                arrival_law(b.dm, b.f_centre), fwhm_us=20.0,
                                amp=b.amp_sigma, nsub=256).astype(np.complex64)
    flush("config 1 full size")
    g = cdd.dedisperse(to_dev(x), b.f_centre, b.bw, b.dm, 0, b.n_int, want_voltages=True,
                       want_chan=True)
    torch.cuda.synchronize()
    info = g["info"]
    assert (info["fft_len"], info["overlap"], info["nfront"]) == (1 << 18, 1 << 17, 64608)
    y = g["y"].cpu().numpy()[0]
    o = O.dedisperse(x, b.f_centre, b.bw, b.dm, b.n_int, fft_len=1 << 18, overlap=1 << 17,
                     nfront=64608, want_voltages=True)
    ev, ei = rel_l2(y, o["y"][0]), rel_l2(g["I"].cpu().numpy(), o["I"])
    flush("config 1 voltage rel L2 %.3g intensity rel L2 %.3g" % (ev, ei))
    assert ev <= TOL_V and ei <= TOL_I
    p = np.convolve(np.abs(y) ** 2, np.ones(320) / 320, mode="same")
    assert abs(int(np.argmax(p)) - (1 << 22)) < 200


def test_long_transform_batched_plan():
    import torch
    cdd = _cdd()
    rng = np.random.default_rng(61)
    nsamp = 90_000
    x = (rng.standard_normal(nsamp) + 1j * rng.standard_normal(nsamp)).astype(np.complex64)
    dms = [1.0, 1.4]
    plan = cdd.Plan([dict(voltages=to_dev(x), f_centre=300.0, bw=4.0, dms=dms, n_int=2,
                          fft_len=1 << 15)])
    plan.execute()
    torch.cuda.synchronize()
    info = plan.info(0)
    for i, dm in enumerate(dms):
        o = O.dedisperse(x, 300.0, 4.0, dm, 2, fft_len=1 << 15, overlap=info["overlap"],
                         nfront=info["nfront"])
        assert rel_l2(plan.I[0][i].cpu().numpy(), o["I"]) <= TOL_I
    plan.close()


def test_persistent_launch_several_beams_same_length():
    """Three beams of different width and channel count, one transform
    length: one persistent launch; each beam's DM trials against the oracle."""
    import torch
    cdd = _cdd()
    specs = [(610.0, 8, 0.03125, 11_000, [10.0, 12.0]),
             (325.0, 20, 0.0625, 9_500, [67.9, 60.0, 70.0]),
             (400.0, 33, 0.048828125, 7_000, [120.0])]
    beams, raw = [], []
    for k, (fcen, nchan, df, nsamp, dms) in enumerate(specs):
        v = _beam_int8(70 + k, nsamp, nchan, fcen, nchan * df, dms[0])
        raw.append((v, fcen, nchan * df, dms))
        beams.append(dict(voltages=to_dev(v), f_centre=fcen, bw=nchan * df, dms=dms,
                          n_int=4, fft_len=2048))
    plan = cdd.Plan(beams)
    for rep in range(2):          # the plan runs again with the same buffers
        plan.execute()
        torch.cuda.synchronize()
        for bi, (v, fcen, bw, dms) in enumerate(raw):
            info = plan.info(bi)
            assert info["fft_len"] == 2048
            for i, dm in enumerate(dms):
                o = O.dedisperse(v, fcen, bw, dm, 4, fft_len=2048, overlap=info["overlap"],
                                 nfront=info["nfront"])
                assert rel_l2(plan.I[bi][i].cpu().numpy(), o["I"]) <= TOL_I
                assert np.array_equal(plan.cov[bi][i].cpu().numpy(), o["cov"])
    plan.close()


def test_persistent_launch_mixed_sample_types():
    """An int8 beam and a complex-float beam of the same transform length in
    one persistent launch, each against the oracle."""
    import torch
    cdd = _cdd()
    v0 = _beam_int8(75, 9_000, 16, 325.0, 1.0, 67.9)
    v1 = _beam_int8(76, 8_000, 4, 325.0, 0.25, 30.0)
    x1 = (v1[..., 0].astype(np.float32) + 1j * v1[..., 1]).astype(np.complex64)
    raw = [(v0, 325.0, 1.0, [67.9]), (x1, 325.0, 0.25, [30.0, 31.0])]
    plan = cdd.Plan([dict(voltages=to_dev(v), f_centre=f, bw=bw, dms=dms, n_int=4, fft_len=2048)
                     for (v, f, bw, dms) in raw])
    plan.execute()
    torch.cuda.synchronize()
    for bi, (v, fcen, bw, dms) in enumerate(raw):
        info = plan.info(bi)
        for i, dm in enumerate(dms):
            o = O.dedisperse(v, fcen, bw, dm, 4, fft_len=2048, overlap=info["overlap"],
                             nfront=info["nfront"])
            assert rel_l2(plan.I[bi][i].cpu().numpy(), o["I"]) <= TOL_I, (bi, i)
    plan.close()


def test_plan_of_one_dm_beams_uses_tables_and_matches_oracle():
    """One-DM beams of one transform length (int8 and complex float, uneven
    channel counts) in one launch over their chirp tables; a one-DM beam of
    another length and a multi-DM beam in the same plan."""
    import torch
    cdd = _cdd()
    v0 = _beam_int8(160, 9_000, 24, 325.0, 1.5, 67.9)
    v1 = _beam_int8(161, 7_000, 8, 610.0, 0.25, 10.0)
    x1 = (v1[..., 0].astype(np.float32) + 1j * v1[..., 1]).astype(np.complex64)
    v2 = _beam_int8(162, 6_000, 16, 400.0, 0.78125, 30.0)
    v3 = _beam_int8(163, 8_000, 12, 325.0, 0.75, 40.0)
    raw = [(v0, 325.0, 1.5, [67.9], 2048), (x1, 610.0, 0.25, [10.0], 2048),
           (v2, 400.0, 0.78125, [30.0], 1024), (v3, 325.0, 0.75, [40.0, 41.0], 2048)]
    plan = cdd.Plan([dict(voltages=to_dev(v), f_centre=f, bw=bw, dms=dms, n_int=4, fft_len=N)
                     for (v, f, bw, dms, N) in raw])
    for rep in range(2):
        plan.execute()
        torch.cuda.synchronize()
        for bi, (v, fcen, bw, dms, N) in enumerate(raw):
            info = plan.info(bi)
            for i, dm in enumerate(dms):
                o = O.dedisperse(v, fcen, bw, dm, 4, fft_len=N, overlap=info["overlap"],
                                 nfront=info["nfront"])
                assert rel_l2(plan.I[bi][i].cpu().numpy(), o["I"]) <= TOL_I, (bi, i)
                assert np.array_equal(plan.cov[bi][i].cpu().numpy(), o["cov"])
    plan.close()


def test_mixed_lengths_one_persistent_launch():
    """Beams of transform lengths 512 to 8192 -- one-DM beams reading their
    chirp tables, a beam with three DM trials, uneven channel counts and
    durations -- in one persistent launch per execute with single_launch
    (checked with the stage timer: one block-kernel launch), every beam and
    DM against the oracle; the same with every chirp formed in the kernel,
    and the default pipelined plan (one launch per beam), match the oracle
    too."""
    import torch
    cdd = _cdd()
    spec = [(610.0, 16, 0.03125, 9_000, [10.0], 512),
            (400.0, 8, 0.048828125, 7_001, [30.0], 1024),
            (325.0, 24, 0.0625, 11_000, [67.9, 69.0, 66.5], 2048),
            (325.0, 6, 0.0625, 13_000, [50.0], 4096),
            (325.0, 4, 0.0625, 20_000, [67.9], 8192)]
    raw = []
    for k, (fcen, nchan, df, nsamp, dms, N) in enumerate(spec):
        raw.append((_beam_int8(170 + k, nsamp, nchan, fcen, nchan * df, dms[0]), fcen,
                    nchan * df, dms, N))
    devs = [to_dev(r[0]) for r in raw]
    for single, in_kernel in ((True, False), (True, True), (False, False)):
        flush("case: mixed lengths, single_launch=%s chirp_in_kernel=%s" % (single, in_kernel))
        plan = cdd.Plan([dict(voltages=vd, f_centre=f, bw=bw, dms=dms, n_int=4, fft_len=N)
                         for vd, (v, f, bw, dms, N) in zip(devs, raw)],
                        chirp_in_kernel=in_kernel, single_launch=single)
        plan.execute()
        torch.cuda.synchronize()
        cdd.profile_read()
        cdd.profile_enable(True, stages=["block"])
        plan.execute()
        torch.cuda.synchronize()
        cdd.profile_enable(False)
        st = cdd.profile_read()
        assert st["block"][1] == (1 if single else len(raw)), st
        for bi, (v, fcen, bw, dms, N) in enumerate(raw):
            info = plan.info(bi)
            assert info["fft_len"] == N
            for i, dm in enumerate(dms):
                o = O.dedisperse(v, fcen, bw, dm, 4, fft_len=N, overlap=info["overlap"],
                                 nfront=info["nfront"])
                assert rel_l2(plan.I[bi][i].cpu().numpy(), o["I"]) <= TOL_I, (bi, i)
                assert np.array_equal(plan.cov[bi][i].cpu().numpy(), o["cov"])
        plan.close()


def test_one_length_beams_in_one_launch_of_that_length():
    """One-DM beams that all share one transform length (1024): with
    single_launch they go through one launch of that length's own kernel
    (not the mixed one), every beam against the oracle."""
    import torch
    cdd = _cdd()
    spec = [(610.0, 16, 0.03125, 9_000, 10.0), (325.0, 24, 0.0625, 11_000, 67.9),
            (400.0, 8, 0.048828125, 7_001, 30.0)]
    raw = [(_beam_int8(190 + k, nsamp, nchan, fcen, nchan * df, dm), fcen, nchan * df, dm)
           for k, (fcen, nchan, df, nsamp, dm) in enumerate(spec)]
    flush("case: three one-DM beams at N 1024, single_launch")
    plan = cdd.Plan([dict(voltages=to_dev(v), f_centre=f, bw=bw, dms=[dm], n_int=4,
                          fft_len=1024) for v, f, bw, dm in raw], single_launch=True)
    plan.execute()
    torch.cuda.synchronize()
    cdd.profile_read()
    cdd.profile_enable(True, stages=["block"])
    plan.execute()
    torch.cuda.synchronize()
    cdd.profile_enable(False)
    st = cdd.profile_read()
    assert st["block"][1] == 1, st
    for bi, (v, fcen, bw, dm) in enumerate(raw):
        info = plan.info(bi)
        o = O.dedisperse(v, fcen, bw, dm, 4, fft_len=1024, overlap=info["overlap"],
                         nfront=info["nfront"])
        assert rel_l2(plan.I[bi][0].cpu().numpy(), o["I"]) <= TOL_I, bi
        assert np.array_equal(plan.cov[bi][0].cpu().numpy(), o["cov"])
    plan.close()


def test_evenly_spaced_dm_tile_recurrence():
    """64 evenly spaced DM trials (one tile), ascending and descending, on a
    band whose chirp phases reach about 115 turns at the channel edges (1.7
    turns between neighbouring trials): the tile advances the
    chirped spectrum by a fixed per-bin rotation per trial; every trial
    against the one-DM call (chirp table from the FP64 phase) and the first,
    middle and last against the oracle."""
    import torch
    cdd = _cdd()
    fcen, nchan, df, nsamp, n_int, N = 150.0, 8, 0.25, 12_000, 4, 2048
    v = _beam_int8(90, nsamp, nchan, fcen, nchan * df, 3.0)
    vd = to_dev(v)
    step = 5.5 / 63
    for dms in ([0.5 + step * i for i in range(64)], [6.0 - step * i for i in range(64)]):
        flush("case: evenly spaced tile from DM %.2f step %.4f" % (dms[0], dms[1] - dms[0]))
        plan = cdd.Plan([dict(voltages=vd, f_centre=fcen, bw=nchan * df, dms=dms,
                              n_int=n_int, fft_len=N)])
        plan.execute()
        torch.cuda.synchronize()
        info = plan.info(0)
        for i, dm in enumerate(dms):
            one = cdd.dedisperse(vd, fcen, nchan * df, dm, N, n_int, overlap=info["overlap"],
                                 nfront=info["nfront"])
            torch.cuda.synchronize()
            assert rel_l2(plan.I[0][i].cpu().numpy(), one["I"].cpu().numpy()) <= 1e-5, (i, dm)
        for i in (0, 31, 63):
            o = O.dedisperse(v, fcen, nchan * df, dms[i], n_int, fft_len=N,
                             overlap=info["overlap"], nfront=info["nfront"])
            assert rel_l2(plan.I[0][i].cpu().numpy(), o["I"]) <= TOL_I, i
            assert np.array_equal(plan.cov[0][i].cpu().numpy(), o["cov"])
        plan.close()


def test_dm_tiles_beyond_one_launch():
    """More DM trials than one launch holds (70 > 64): two rounds."""
    import torch
    cdd = _cdd()
    v = _beam_int8(80, 6_000, 4, 325.0, 0.25, 30.0, pulse=False)
    dms = [20.0 + 0.3 * i for i in range(70)]
    plan = cdd.Plan([dict(voltages=to_dev(v), f_centre=325.0, bw=0.25, dms=dms, n_int=2,
                          fft_len=1024)])
    plan.execute()
    torch.cuda.synchronize()
    info = plan.info(0)
    for i in (0, 33, 63, 64, 69):
        o = O.dedisperse(v, 325.0, 0.25, dms[i], 2, fft_len=1024, overlap=info["overlap"],
                         nfront=info["nfront"])
        assert rel_l2(plan.I[0][i].cpu().numpy(), o["I"]) <= TOL_I
    plan.close()


def test_autotuner_picks_a_valid_plan_and_plan_uses_it():
    import torch
    cdd = _cdd()
    fcen, nchan, df, dms = 325.0, 32, 0.0625, [60.0, 64.0, 68.0]
    r = cdd.autotune(nchan, fcen, nchan * df, dms, 4)
    flush("autotune: %s" % r)
    assert r["fft_len"] in (2048, 4096, 8192, 16384) and r["msamples_per_s"] > 0
    assert 0 <= r["kernel_variant"] < cdd.lib.cdd_kernel_variants(r["fft_len"])
    # a schedule the persistent batched kernel runs, and a tile of the beam's trials
    assert r["kernel_variant"] == 0 or (r["fft_len"], r["kernel_variant"]) in (
        (4096, 3), (8192, 1), (8192, 2), (16384, 2))
    assert r["dm_tile"] == len(dms)
    assert cdd.autotune(nchan, fcen, nchan * df, dms, 4) == r      # cached
    one = cdd.autotune(nchan, fcen, nchan * df, [64.0], 4)
    assert one["dm_tile"] == 1 and one["kernel_variant"] == 0
    v = _beam_int8(120, 20_000, nchan, fcen, nchan * df, 64.0)
    plan = cdd.Plan([dict(voltages=to_dev(v), f_centre=fcen, bw=nchan * df, dms=dms, n_int=4)],
                    autotune=True)
    info = plan.info(0)
    assert info["fft_len"] == r["fft_len"]
    plan.execute()
    torch.cuda.synchronize()
    for i, dm in enumerate(dms):
        o = O.dedisperse(v, fcen, nchan * df, dm, 4, fft_len=info["fft_len"],
                         overlap=info["overlap"], nfront=info["nfront"])
        assert rel_l2(plan.I[0][i].cpu().numpy(), o["I"]) <= TOL_I
    plan.close()


def test_long_transforms_in_several_chunks():
    """2^22-point channel transforms keep at most 16 (channel, block) items
    of spectra in the workspace: 4 channels of 5 blocks run in two chunks."""
    import torch
    cdd = _cdd()
    nchan, fcen, bw, dm, n_int = 4, 300.0, 4.0, 0.001, 4
    N = 1 << 22
    q = cdd.query(0, 1 << 20, nchan, fcen, bw, dm, N, n_int)
    M = q["step"]
    nsamp = 5 * M - 1000
    rng = np.random.default_rng(41)
    v = synth.noise_int8(rng, nsamp, nchan, 20.0)
    flush("case: long transforms, %d channels x %d samples, N 2^22" % (nchan, nsamp))
    g = cdd.dedisperse(to_dev(v), fcen, bw, dm, N, n_int, want_chan=True)
    torch.cuda.synchronize()
    info = g["info"]
    assert info["nblocks"] == 5
    o = O.dedisperse(v, fcen, bw, dm, n_int, fft_len=N, overlap=info["overlap"],
                     nfront=info["nfront"])
    assert rel_l2(g["P"].cpu().numpy(), o["P"]) <= TOL_I
    assert rel_l2(g["I"].cpu().numpy(), o["I"]) <= TOL_I
