"""The entry point that allocates nothing (cdd_dedisperse_noalloc) against
cdd_dedisperse: the same results, through the C ABI, on calls in a row whose
second input is smaller than the first (the static scratch keeps the first
call's contents), for the fused block kernel and the long transforms, and
both against the FP64 oracle.  Oversized requests are refused before any
launch."""
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


def _pair(v, fcen, bw, dm, fft_len, n_int):
    """Both entry points on the same resident input; voltages and channel
    intensities too."""
    import torch
    cdd = _cdd()
    vd = to_dev(v)
    kw = dict(want_chan=True, want_voltages=True)
    a = cdd.dedisperse_noalloc(vd, fcen, bw, dm, fft_len, n_int, **kw)
    torch.cuda.synchronize()
    b = cdd.dedisperse(vd, fcen, bw, dm, fft_len, n_int, time_chunks=1, **kw)
    torch.cuda.synchronize()
    return ({k: a[k].cpu().numpy() for k in ("I", "cov", "P", "y")},
            {k: b[k].cpu().numpy() for k in ("I", "cov", "P", "y")}, a["info"])


def _compare(a, b, o):
    for k in ("I", "P"):
        assert rel_l2(a[k], b[k]) <= TOL_I, k
        assert np.array_equal(a[k], b[k]), k     # same kernels, same launch shape
    assert rel_l2(a["y"], b["y"]) <= TOL_V
    assert np.array_equal(a["cov"], b["cov"])
    assert rel_l2(a["y"], o["y"]) <= TOL_V
    assert rel_l2(a["P"], o["P"]) <= TOL_I
    assert rel_l2(a["I"], o["I"]) <= TOL_I
    assert np.array_equal(a["cov"], o["cov"])


def _beam(seed, nsamp, nchan, fcen, bw, dm):
    b = synth.Beam(fcen, bw, nchan, nsamp, dm, period_s=0.02, fwhm_s=0.3e-3)
    fc, _ = O.channel_centres(fcen, bw, nchan)
    return synth.make_beam(b, np.random.default_rng(seed), arrival_law(dm, fc[-1]))


@pytest.mark.parametrize("case", [
    # (nsamp, nchan, fcen, bw, dm, N, n_int): larger first, then smaller
    [(60_001, 96, 325.0, 96 * 0.0625, 67.9, 2048, 4), (20_000, 17, 325.0, 17 * 0.0625, 30.0,
                                                        1024, 3)],
])
def test_noalloc_block_kernel_two_calls(case):
    for i, (nsamp, nchan, fcen, bw, dm, N, n_int) in enumerate(case):
        flush("case: noalloc call %d: nsamp=%d nchan=%d N=%d dm=%g n_int=%d" %
              (i, nsamp, nchan, N, dm, n_int))
        v = _beam(700 + i, nsamp, nchan, fcen, bw, dm)
        a, b, info = _pair(v, fcen, bw, dm, N, n_int)
        o = O.dedisperse(v, fcen, bw, dm, n_int, fft_len=info["fft_len"],
                         overlap=info["overlap"], nfront=info["nfront"], want_voltages=True)
        _compare(a, b, o)


def test_noalloc_long_transforms_two_calls():
    rng = np.random.default_rng(710)
    for i, (nsamp, N) in enumerate([(200_003, 1 << 16), (70_000, 1 << 15)]):
        flush("case: noalloc long call %d: nsamp=%d N=%d" % (i, nsamp, N))
        x = ((rng.standard_normal(nsamp) + 1j * rng.standard_normal(nsamp)) * 3.0)
        x = x.astype(np.complex64)
        a, b, info = _pair(x, 610.0, 4.0, 5.0 + i, N, 4)
        o = O.dedisperse(x, 610.0, 4.0, 5.0 + i, 4, fft_len=info["fft_len"],
                         overlap=info["overlap"], nfront=info["nfront"], want_voltages=True)
        _compare(a, b, o)


def test_noalloc_refuses_oversized_and_unsupported():
    cdd = _cdd()
    import torch
    # 4096 channels x 2 s needs about 1.6 GB of workspace
    v = torch.zeros((97_656, 4096, 2), dtype=torch.int8, device="cuda:0")
    with pytest.raises(cdd.CddError) as ei:
        cdd.dedisperse_noalloc(v, 400.0, 200.0, 120.0, 8192, 4)
    assert ei.value.status == -1 and "scratch" in str(ei.value)
    del v
    torch.cuda.empty_cache()
