"""Parity of the full-band mode with the FP64 oracle, through the C ABI.

The recorded beam is a sequence of real-FFT spectra; the HIP path inverse
transforms them into one real series and dedisperses it as a single band
(real transforms of up to 2^27 points, chirp about the lower band edge).
Tolerances as for the channel path: the dedispersed series <= 1e-5 and the
integrated intensities <= 1e-4 relative L2.  Records are seeded int8 noise
(the spectra of white noise are themselves independent complex Gaussians).
"""
import numpy as np
import pytest

import oracle as O
import synth
from tests.util import flush, rel_l2, to_dev

pytestmark = pytest.mark.gpu

TOL_V, TOL_I = 1e-5, 1e-4


def _cdd():
    import paper_1509_00186_amd as cdd
    return cdd


def _records(seed, nspec, nchan):
    return synth.noise_int8(np.random.default_rng(seed), nspec, nchan, 20.0)


@pytest.mark.parametrize("nchan,nspec", [(128, 1), (256, 37), (512, 301), (1024, 64),
                                         (2048, 5)])
def test_gsb_inverse_against_oracle(nchan, nspec):
    import torch
    flush("case: gsb_inverse nchan=%d nspec=%d" % (nchan, nspec))
    sp = _records(nchan + nspec, nspec, nchan)
    got = _cdd().gsb_inverse(to_dev(sp))
    torch.cuda.synchronize()
    want = O.gsb_inverse(sp)
    assert rel_l2(got.cpu().numpy(), want) <= TOL_V


def _fb_both(sp, fcen, bw, dm, n_int, taper="none", **kw):
    import torch
    flush("case: fullband records=%s fcen=%g bw=%g dm=%g n_int=%d taper=%s %s" %
          (tuple(sp.shape), fcen, bw, dm, n_int, taper, kw))
    g = _cdd().fullband(to_dev(sp), fcen, bw, dm, n_int, want_voltages=True, taper=taper, **kw)
    torch.cuda.synchronize()
    info = g["info"]
    o = O.fullband_dedisperse(sp, fcen, bw, dm, n_int, fft_len=info["fft_len"],
                              overlap=info["overlap"], nfront=info["nfront"], window=taper,
                              want_voltages=True)
    return g["y"].cpu().numpy(), g["I"].cpu().numpy(), o, info


@pytest.mark.parametrize("nchan,nspec,fcen,bw,dm,n_int,taper", [
    (512, 300, 610.0, 16.0, 0.3, 2, "none"),     # 2^16 points, six blocks, ragged tail
    (512, 300, 610.0, 16.0, 0.3, 4, "hann"),
    (512, 300, 610.0, 16.0, 0.3, 6, "welch"),    # overlap raised to 8194 for n_int 6
    (256, 700, 325.0, 16.0, -0.5, 2, "none"),    # negative DM: the reach is backward
    (1024, 200, 325.0, 32.0, 0.2, 8, "none"),    # 2^18 points
    (512, 2048, 610.0, 16.0, 10.0, 16, "none"),  # the 16 MHz, DM 10 geometry: 2^19 points
    (128, 1, 610.0, 16.0, 0.0, 2, "none"),       # one record, DM 0
])
def test_fullband_against_oracle(nchan, nspec, fcen, bw, dm, n_int, taper):
    sp = _records(7 * nchan + nspec, nspec, nchan)
    y, I, o, info = _fb_both(sp, fcen, bw, dm, n_int, taper)
    assert info["nsamp"] == nspec * 2 * nchan and I.shape == (info["t_int"],)
    assert rel_l2(y, o["y"]) <= TOL_V, rel_l2(y, o["y"])
    assert rel_l2(I, o["P"]) <= TOL_I, rel_l2(I, o["P"])
    if dm == 0.0:
        assert rel_l2(y, o["x"]) <= TOL_V


@pytest.mark.parametrize("lg", [20, 21, 22])
def test_fullband_two_level_lengths(lg):
    """Real transforms of 2^20 .. 2^22 points (2048-point row pairs, columns
    of 256 .. 1024): 16 MHz at 610 MHz with the DM scaled so the impulse
    response spans about an eighth of the transform, two blocks, the second
    ragged."""
    N = 1 << lg
    dm = 10.0 * N / (1 << 21)
    nspec = (8 * N // 5) // 1024 + 3
    sp = _records(40 + lg, nspec, 512)
    y, I, o, info = _fb_both(sp, 610.0, 16.0, dm, 16, fft_len=N)
    assert info["fft_len"] == N and info["nblocks"] == 2
    assert rel_l2(y, o["y"]) <= TOL_V, rel_l2(y, o["y"])
    assert rel_l2(I, o["P"]) <= TOL_I, rel_l2(I, o["P"])


def test_fullband_explicit_plan():
    sp = _records(11, 400, 512)
    y, I, o, info = _fb_both(sp, 610.0, 16.0, 0.5, 4, fft_len=1 << 17, overlap=1 << 15,
                             nfront=12000)
    assert (info["fft_len"], info["overlap"], info["nfront"]) == (1 << 17, 1 << 15, 12000)
    assert rel_l2(y, o["y"]) <= TOL_V
    assert rel_l2(I, o["P"]) <= TOL_I


def test_fullband_full_size_16mhz_dm10():
    """The benchmark record: 16384 records of 512 bins (2^24 real samples,
    0.52 s at 32 Msamples/s), 610 MHz, DM 10, 2^19-point transforms."""
    sp = _records(12, 16384, 512)
    y, I, o, info = _fb_both(sp, 610.0, 16.0, 10.0, 16)
    assert info["fft_len"] == 1 << 19 and info["nblocks"] == 64
    assert rel_l2(y, o["y"]) <= TOL_V
    assert rel_l2(I, o["P"]) <= TOL_I


def test_fullband_repeated_calls_reuse_buffers():
    import torch
    cdd = _cdd()
    sp = to_dev(_records(13, 300, 512))
    a = cdd.fullband(sp, 610.0, 16.0, 0.3, 2)
    first = a["I"].clone()
    b = cdd.fullband(sp, 610.0, 16.0, 0.3, 2, out=a)
    torch.cuda.synchronize()
    assert torch.equal(first, b["I"])


def test_fullband_several_chunks_of_spectra():
    """2^23-point transforms keep at most 16 blocks of spectra in the
    workspace: a record of 17 blocks runs in two chunks."""
    nchan = 512
    M = (1 << 23) - 1024
    nspec = -(-16 * M // (2 * nchan)) + 5
    sp = _records(14, nspec, nchan)
    y, I, o, info = _fb_both(sp, 610.0, 16.0, 0.05, 2, fft_len=1 << 23)
    assert info["nblocks"] == 17 and info["overlap"] == 1024
    assert rel_l2(y, o["y"]) <= TOL_V
    assert rel_l2(I, o["P"]) <= TOL_I


@pytest.mark.parametrize("lg,dm,n_int,odd_pairs", [(24, 0.5, 16, True), (24, 0.5, 16, False),
                                                   (25, 1.0, 6, False)])
def test_fullband_three_level_transforms(lg, dm, n_int, odd_pairs):
    """Real transforms of 2^24 and 2^25 points (packed complex 2^23 and
    2^24, columns split in two passes each): two blocks, the second ragged;
    fused integration with an odd pair start (split groups) or the rule's
    (a multiple of 32 samples), and the separate integration (n_int 6)."""
    nchan = 512
    q = _cdd().fullband_query(1, nchan, 610.0, 16.0, dm, n_int, fft_len=1 << lg)
    M = q["step"]
    nspec = -(-(M + M // 3 + 5000) // (2 * nchan))
    sp = _records(20 + lg + odd_pairs, nspec, nchan)
    plan = dict(overlap=q["overlap"], nfront=q["nfront"] + 2) if odd_pairs else {}
    y, I, o, info = _fb_both(sp, 610.0, 16.0, dm, n_int, fft_len=1 << lg, **plan)
    assert (info["fft_len"], info["nblocks"]) == (1 << lg, 2)
    assert ((info["nfront"] // 2) % 2 == 1) == odd_pairs
    assert rel_l2(y, o["y"]) <= TOL_V, rel_l2(y, o["y"])
    assert rel_l2(I, o["P"]) <= TOL_I, rel_l2(I, o["P"])


def test_fullband_at_the_section_4_5_dm_limit():
    """The first of Sec. 4.5's memory-bound limits, DM 3000 at 610 MHz over
    16 MHz, planned by the length rule at 2^27 real points (L = 2^26): one
    block over 2^25 real samples (1 s), against the oracle."""
    sp = _records(31, 1 << 15, 512)
    y, I, o, info = _fb_both(sp, 610.0, 16.0, 3000.0, 16)
    assert (info["fft_len"], info["overlap"], info["nblocks"]) == (1 << 27, 1 << 26, 1)
    assert rel_l2(y, o["y"]) <= TOL_V, rel_l2(y, o["y"])
    assert rel_l2(I, o["P"]) <= TOL_I, rel_l2(I, o["P"])


def test_fullband_short_record_stays_inside_its_workspace():
    """One record of 128 bins (256 real samples) on a 2^16-point transform:
    the fused integration's partial sums stay inside the workspace (a canary
    after it is untouched) and the result matches the oracle."""
    import torch
    cdd = _cdd()
    sp = _records(32, 1, 128)
    q = cdd.fullband_query(1, 128, 610.0, 16.0, 0.05, 2, fft_len=1 << 16)
    ws = torch.full((q["ws_bytes"] + (1 << 20),), 0x5A, dtype=torch.uint8, device="cuda")
    flush("case: fullband short record ws=%d" % q["ws_bytes"])
    g = cdd.fullband(to_dev(sp), 610.0, 16.0, 0.05, 2, fft_len=1 << 16, want_voltages=True,
                     out={"ws": ws})
    torch.cuda.synchronize()
    assert bool((ws[q["ws_bytes"]:] == 0x5A).all())
    o = O.fullband_dedisperse(sp, 610.0, 16.0, 0.05, 2, fft_len=1 << 16, overlap=q["overlap"],
                              nfront=q["nfront"], want_voltages=True)
    assert rel_l2(g["y"].cpu().numpy(), o["y"]) <= TOL_V
    assert rel_l2(g["I"].cpu().numpy(), o["P"]) <= TOL_I
