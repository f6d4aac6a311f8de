"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/cdd.h declares, validates arguments, and its planner
agrees with the oracle's rules."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cdd.h")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _lib():
    import paper_1509_00186_amd as cdd
    return cdd


def test_library_exports_every_declared_function():
    cdd = _lib()
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(cdd_[a-z_0-9]+)\s*\(", src))
    assert {"cdd_dedisperse", "cdd_query", "cdd_plan_create", "cdd_plan_execute",
            "cdd_plan_destroy", "cdd_last_error"} <= names
    raw = ctypes.CDLL(cdd.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(raw, n)]
    assert not missing, missing
    assert cdd.lib.cdd_abi_version() == 1


def test_status_strings():
    cdd = _lib()
    for code, name in cdd._binding.STATUS.items():
        assert cdd.lib.cdd_status_str(code).decode() == name


CASES = [
    (0, 250_000, 512, 325.0, 32.0, 67.9, 8192, 4),
    (0, 97_656, 4096, 400.0, 200.0, 120.0, 8192, 4),
    (1, 1 << 23, 1, 610.0, 16.0, 10.0, 0, 16),
    (0, 31_250, 512, 610.0, 16.0, 10.0, 0, 4),
    (0, 125_000, 512, 325.0, 32.0, 67.9, 0, 4),
    (0, 93_750, 1024, 325.0, 32.0, 67.9, 0, 4),
    (0, 195_312, 4096, 400.0, 200.0, 120.0, 0, 4),
    (0, 10_000, 64, 325.0, 32.0 / 8, -40.0, 0, 3),
    (1, 5000, 3, 150.0, 1.0, 0.0, 0, 1),
    (0, 100_000, 256, 235.0, 16.0, 67.99, 0, 5),
    (1, 1000, 1, 300.0, 4.0, 1.0, 1 << 15, 4),
    (1, 3 << 24, 1, 300.0, 4.0, 3072.0, 1 << 26, 8),
]


@pytest.mark.parametrize("case", CASES)
def test_planner_matches_oracle_rules(case):
    cdd = _lib()
    dt, nsamp, nchan, fcen, bw, dm, fft, n_int = case
    q = cdd.query(dt, nsamp, nchan, fcen, bw, dm, fft, n_int)
    N, L, nfront = O.overlap_plan(fcen, bw, nchan, [dm], n_int, fft or None)
    assert (q["fft_len"], q["overlap"], q["nfront"]) == (N, L, nfront)
    assert q["step"] == N - L and q["nblocks"] == -(-nsamp // (N - L))
    assert q["t_int"] == nsamp // n_int
    d = O.channel_delays(fcen, bw, nchan, dm, n_int)
    assert q["d_max"] == int(d.max())
    fc, df = O.channel_centres(fcen, bw, nchan)
    fr, bk = O.wrap_extent(fc, df, dm)
    assert (q["front"], q["back"]) == (math.ceil(fr), math.ceil(bk))


@pytest.mark.parametrize("args,frag", [
    (dict(dtype=2), "dtype"),
    (dict(nsamp=0), "nsamp"),
    (dict(nchan=0), "nchan"),
    (dict(n_int=0), "n_int"),
    (dict(n_int=10_001), "n_int"),
    (dict(bw=-1.0), "bw"),
    (dict(f_centre=10.0, bw=32.0), "above 0"),
    (dict(dm=float("nan")), "DM"),
    (dict(fft_len=1000), "power of two"),
    (dict(fft_len=128), "power of two"),
    (dict(fft_len=1 << 27), "power of two"),
    (dict(dm=3000.0, fft_len=256), "DM too large"),
    (dict(f_centre=float("inf")), "finite"),
])
def test_invalid_arguments_are_rejected(args, frag):
    cdd = _lib()
    a = dict(dtype=0, nsamp=10_000, nchan=64, f_centre=325.0, bw=4.0, dm=30.0,
             fft_len=0, n_int=4)
    a.update(args)
    with pytest.raises(cdd.CddError) as ei:
        cdd.query(a["dtype"], a["nsamp"], a["nchan"], a["f_centre"], a["bw"], a["dm"],
                  a["fft_len"], a["n_int"])
    assert ei.value.status == -1 and frag in str(ei.value), str(ei.value)


def test_incoherent_validation_without_device():
    cdd = _lib()
    assert cdd.lib.cdd_incoherent_ws_bytes(0, 10_000, 64, 4) >= 64 * 10_000 * 2
    assert cdd.lib.cdd_incoherent_ws_bytes(0, 10_000, 64, 0) == 0
    assert cdd.lib.cdd_incoherent_ws_bytes(5, 10_000, 64, 4) == 0
    o = cdd._binding.make_opts()
    ws = cdd.lib.cdd_incoherent_ws_bytes(0, 10_000, 64, 4)
    st = cdd.lib.cdd_incoherent(ctypes.c_void_p(0x1000), 0, 10_000, 64, 325.0, 4.0, 3000.0, 4,
                                ctypes.c_void_p(0x2000), None, None, ctypes.byref(o), None, 0,
                                None)
    assert st == -1 and b"workspace" in cdd.lib.cdd_last_error()
    st = cdd.lib.cdd_incoherent(ctypes.c_void_p(0x1000), 0, 10_000, 64, 10.0, 32.0, 30.0, 4,
                                ctypes.c_void_p(0x2000), None, None, ctypes.byref(o),
                                ctypes.c_void_p(0x3000), ws, None)
    assert st == -1 and b"above 0" in cdd.lib.cdd_last_error()


def test_fold_validation_without_device():
    cdd = _lib()
    st = cdd.lib.cdd_fold(None, 100, 10.0, 0.0, 8, ctypes.c_void_p(0x100), None, None)
    assert st == -1 and b"NULL" in cdd.lib.cdd_last_error()
    st = cdd.lib.cdd_fold(ctypes.c_void_p(0x100), 100, 0.5, 0.0, 8, ctypes.c_void_p(0x200),
                          None, None)
    assert st == -1 and b"period" in cdd.lib.cdd_last_error()
    st = cdd.lib.cdd_fold(ctypes.c_void_p(0x100), 100, 10.0, 0.0, 0, ctypes.c_void_p(0x200),
                          None, None)
    assert st == -1 and b"nbins" in cdd.lib.cdd_last_error()


def test_explicit_plan_validation():
    cdd = _lib()
    ok = cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4, overlap=128, nfront=64)
    assert (ok["fft_len"], ok["overlap"], ok["nfront"]) == (1024, 128, 64)
    with pytest.raises(cdd.CddError, match="multiple of n_int"):
        cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4, overlap=127, nfront=64)
    with pytest.raises(cdd.CddError, match="nfront"):
        cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4, overlap=128, nfront=0)
    with pytest.raises(cdd.CddError, match="shorter than the impulse"):
        cdd.query(0, 10_000, 64, 325.0, 4.0, 300.0, 1024, 4, overlap=8, nfront=4)
    with pytest.raises(cdd.CddError, match="dm_const"):
        cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4, dm_const=-1.0)
    with pytest.raises(cdd.CddError, match="phase_mode"):
        cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4, phase_mode=7)
    with pytest.raises(cdd.CddError, match="taper"):
        cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4, taper=3)
    # the taper leaves the plan unchanged
    assert cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4, taper="hann") == \
        cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4)


def test_dedisperse_rejects_bad_workspace_without_touching_device():
    cdd = _lib()
    o = cdd._binding.make_opts()
    st = cdd.lib.cdd_dedisperse(ctypes.c_void_p(0x1000), 0, 10_000, 64, 325.0, 4.0, 30.0,
                                1024, 4, ctypes.c_void_p(0x2000), None, None, None,
                                ctypes.byref(o), None, 0, None)
    assert st == -1 and b"workspace" in cdd.lib.cdd_last_error()
    st = cdd.lib.cdd_dedisperse(None, 0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4,
                                ctypes.c_void_p(0x2000), None, None, None, ctypes.byref(o),
                                None, 0, None)
    assert st == -1 and b"voltages" in cdd.lib.cdd_last_error()
    q = cdd.query(0, 10_000, 64, 325.0, 4.0, 30.0, 1024, 4)
    st = cdd.lib.cdd_dedisperse(ctypes.c_void_p(0x1000), 0, 10_000, 64, 325.0, 4.0, 30.0,
                                1024, 4, ctypes.c_void_p(0x2000), None, None, None,
                                ctypes.byref(o), ctypes.c_void_p(0x3001), q["ws_bytes"], None)
    assert st == -1 and b"aligned" in cdd.lib.cdd_last_error()
    o.time_chunks = -2
    st = cdd.lib.cdd_dedisperse(ctypes.c_void_p(0x1000), 0, 10_000, 64, 325.0, 4.0, 30.0,
                                1024, 4, ctypes.c_void_p(0x2000), None, None, None,
                                ctypes.byref(o), ctypes.c_void_p(0x3000), q["ws_bytes"], None)
    assert st == -1 and b"time_chunks" in cdd.lib.cdd_last_error()


def test_last_error_is_thread_local():
    import threading
    cdd = _lib()
    with pytest.raises(cdd.CddError):
        cdd.query(0, 0, 64, 325.0, 4.0, 30.0, 0, 4)
    seen = {}

    def worker():
        seen["msg"] = cdd.lib.cdd_last_error()
    th = threading.Thread(target=worker)
    th.start()
    th.join()
    assert seen["msg"] == b""
    assert b"nsamp" in cdd.lib.cdd_last_error()


def test_plan_create_validates_beams():
    cdd = _lib()
    B = cdd._binding.BeamDesc
    descs = (B * 1)()
    h = ctypes.c_void_p()
    o = cdd._binding.make_opts()
    assert cdd.lib.cdd_plan_create(descs, 1, ctypes.byref(o), ctypes.byref(h)) == -1
    assert b"NULL" in cdd.lib.cdd_last_error()
    dms = (ctypes.c_double * 2)(10.0, float("inf"))
    d = descs[0]
    d.voltages, d.intensity = 0x1000, 0x2000
    d.dtype, d.nchan, d.nsamp, d.f_centre_mhz, d.bw_mhz = 0, 8, 5000, 325.0, 1.0
    d.host_dms, d.ndm, d.n_int = dms, 2, 4
    assert cdd.lib.cdd_plan_create(descs, 1, ctypes.byref(o), ctypes.byref(h)) == -1
    assert b"beam 0" in cdd.lib.cdd_last_error()
    dms[1] = 12.0
    assert cdd.lib.cdd_plan_create(descs, 1, ctypes.byref(o), ctypes.byref(h)) == 0
    info = cdd._binding.PlanInfo()
    assert cdd.lib.cdd_plan_info_get(h, 0, ctypes.byref(info)) == 0
    N, L, nfront = O.overlap_plan(325.0, 1.0, 8, [10.0, 12.0], 4)
    assert (info.fft_len, info.overlap, info.nfront) == (N, L, nfront)
    assert cdd.lib.cdd_plan_info_get(h, 1, ctypes.byref(info)) == -1
    cdd.lib.cdd_plan_destroy(h)


@pytest.mark.parametrize("args", [
    (300, 512, 610.0, 16.0, 0.3, 2), (16384, 512, 610.0, 16.0, 10.0, 16),
    (1000, 1024, 325.0, 32.0, -2.0, 8), (500, 256, 610.0, 16.0, 0.0, 2),
    (300, 512, 610.0, 16.0, 0.3, 6), (4000, 2048, 325.0, 32.0, 3.0, 4),
])
def test_fullband_planner_matches_oracle_rules(args):
    nspec, nchan, fcen, bw, dm, n_int = args
    q = _lib().fullband_query(nspec, nchan, fcen, bw, dm, n_int)
    N, L, nf = O.fullband_plan(fcen - bw / 2, bw, dm, n_int)
    assert (q["fft_len"], q["overlap"], q["nfront"]) == (N, L, nf)
    assert q["nsamp"] == nspec * 2 * nchan and q["step"] == N - L
    assert q["nblocks"] == -(-q["nsamp"] // (N - L)) and q["t_int"] == q["nsamp"] // n_int


@pytest.mark.parametrize("args,kw,frag", [
    ((300, 500, 610.0, 16.0, 0.3, 2), {}, "nchan"),
    ((300, 512, 610.0, 16.0, 0.3, 3), {}, "n_int"),
    ((0, 512, 610.0, 16.0, 0.3, 2), {}, "nspec"),
    ((300, 512, 610.0, 16.0, 0.3, 2), {"fft_len": 1 << 15}, "fft_len"),
    ((300, 512, 610.0, 16.0, 6600.0, 2), {}, "DM too large"),
    ((300, 512, 610.0, 16.0, 0.3, 2), {"phase_mode": 1}, "FP64"),
    ((300, 512, 10.0, 30.0, 0.3, 2), {}, "band"),
])
def test_fullband_invalid_arguments_are_rejected(args, kw, frag):
    cdd = _lib()
    with pytest.raises(cdd.CddError) as e:
        cdd.fullband_query(*args, **kw)
    assert frag in str(e.value)


def test_fullband_plans_the_section_4_5_dm_limits_at_2_27_points():
    """Each of Sec. 4.5's memory-bound DM limits needs 2^27-point real
    transforms under the length rule; the library plans them (and refuses a
    DM that would need 2^28)."""
    g = json.load(open(os.path.join(GOLDEN, "max_dm_sec4_5.json")))
    for case in g["cases"]:
        f, bw, dm = case["f_mhz"], case["bw_mhz"], case["dm"]
        q = _lib().fullband_query(1 << 15, 512, f, bw, dm, 2)
        N, L, nf = O.fullband_plan(f - bw / 2, bw, dm, 2)
        assert q["fft_len"] == N == 1 << 27, case
        assert (q["overlap"], q["nfront"]) == (L, nf), case
        with pytest.raises(_lib().CddError) as e:
            _lib().fullband_query(1 << 15, 512, f, bw, 2.2 * dm, 2)
        assert "DM too large" in str(e.value), case


@pytest.mark.parametrize("nsamp,N,n_int", [(1000, 1 << 15, 4), (5000, 1 << 17, 16),
                                           (2, 1 << 16, 2)])
def test_workspace_holds_the_partial_integration_sums(nsamp, N, n_int):
    """With integration fused into the long transforms, two partial sums per
    run of 8-16 samples of every transformed block are kept in the |y|^2
    buffer; a record much shorter than its transform still gets room for
    them (one block: S and the chirp table take 16 N bytes, the partial sums
    up to N bytes more)."""
    q = _lib().query(1, nsamp, 1, 300.0, 4.0, 0.5, N, n_int)
    assert q["nblocks"] == 1
    assert q["ws_bytes"] >= 16 * N + N
    f = _lib().fullband_query(1, 128, 610.0, 16.0, 0.05, 2, fft_len=1 << 16)
    assert f["ws_bytes"] >= 256 * 4 + (1 << 15) * 8 + (1 << 15) + ((1 << 15) + 1) * 8


def test_profile_select_validation():
    cdd = _lib()
    assert cdd.lib.cdd_profile_select(0) == -1
    assert cdd.lib.cdd_profile_select(1 << 4) == -1
    assert cdd.lib.cdd_profile_select(0b0100) == 0
    assert cdd.lib.cdd_profile_select(0b1111) == 0


def test_fullband_entry_points_validate_without_device():
    """Argument errors of the full-band calls are reported before any launch."""
    import ctypes
    cdd = _lib()
    L = cdd.lib
    buf = ctypes.create_string_buffer(1 << 16)
    base = ctypes.addressof(buf)
    aligned = (base + 255) & ~255
    # inverse transform: NULL, misaligned, bad shapes
    assert L.cdd_gsb_inverse(None, 4, 512, ctypes.c_void_p(aligned), None) == -1
    assert L.cdd_gsb_inverse(ctypes.c_void_p(aligned + 2), 4, 512, ctypes.c_void_p(aligned), None) == -1
    assert L.cdd_gsb_inverse(ctypes.c_void_p(aligned), 4, 500, ctypes.c_void_p(aligned), None) == -1
    assert L.cdd_gsb_inverse(ctypes.c_void_p(aligned), 0, 512, ctypes.c_void_p(aligned), None) == -1
    # whole path: short workspace, misaligned workspace, odd n_int
    from paper_1509_00186_amd._binding import make_opts
    o = make_opts()
    args = (ctypes.c_void_p(aligned), 300, 512, 610.0, 16.0, 0.3, 0, 2,
            ctypes.c_void_p(aligned), None, ctypes.byref(o))
    assert L.cdd_fullband_dedisperse(*args, ctypes.c_void_p(aligned), 256, None) == -1
    assert "workspace" in L.cdd_last_error().decode()
    assert L.cdd_fullband_dedisperse(*args, ctypes.c_void_p(aligned + 8), 1 << 40, None) == -1
    assert "aligned" in L.cdd_last_error().decode()
    bad = (ctypes.c_void_p(aligned), 300, 512, 610.0, 16.0, 0.3, 0, 3,
           ctypes.c_void_p(aligned), None, ctypes.byref(o))
    assert L.cdd_fullband_dedisperse(*bad, ctypes.c_void_p(aligned), 1 << 40, None) == -1
    assert "n_int" in L.cdd_last_error().decode()


def test_noalloc_refuses_a_workspace_beyond_its_scratch_before_any_launch():
    """cdd_dedisperse_noalloc checks the call's workspace against its static
    scratch (CDD_NOALLOC_SCRATCH_BYTES) before touching the device, so the
    refusal needs no GPU; pointers are never dereferenced on that path."""
    cdd = _lib()
    src = open(HEADER).read()
    m = re.search(r"#define CDD_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", src)
    cap = int(m.group(1)) << int(m.group(2))
    # 4096 channels x 97,656 int8 samples: the channel-major copy alone is 800 MB
    q = cdd.query(0, 97_656, 4096, 400.0, 200.0, 120.0, 8192, 4)
    assert q["ws_bytes"] > cap
    fake = ctypes.c_void_p(1 << 20)
    st = cdd.lib.cdd_dedisperse_noalloc(fake, 0, 97_656, 4096, 400.0, 200.0, 120.0, 8192, 4,
                                        fake, None, None, None, None, None)
    assert st == -1
    assert b"scratch" in cdd.lib.cdd_last_error()
    # npol 2 is not taken
    o = cdd._binding.make_opts(8192)
    o.npol = 2
    st = cdd.lib.cdd_dedisperse_noalloc(fake, 0, 1000, 4, 325.0, 0.25, 1.0, 8192, 4, fake, None,
                                        None, None, ctypes.byref(o), None)
    assert st == -7
