"""ctypes binding of libcdd.so: argument marshalling only.

Every step of the computation runs in the HIP library; PyTorch supplies
device memory (outputs and workspace) and the stream.  If the library has not
been built, importing this module raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libcdd.so")

CDD_CI8, CDD_CF32 = 0, 1
PHASE_FP64_REDUCED, PHASE_FP32 = 0, 1

STATUS = {0: "CDD_OK", -1: "CDD_EINVAL", -2: "CDD_ENOMEM", -3: "CDD_EDEVICE",
          -4: "CDD_EBUSY", -5: "CDD_EAGAIN", -6: "CDD_EINTERNAL", -7: "CDD_ENOTSUP"}


class CddError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status
        self.name = STATUS.get(status, str(status))


class Opts(ctypes.Structure):
    _fields_ = [("explicit_plan", ctypes.c_int32), ("fft_len", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("nfront", ctypes.c_int32),
                ("dm_const", ctypes.c_double), ("phase_mode", ctypes.c_int32),
                ("kernel_variant", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("time_chunks", ctypes.c_int32), ("taper", ctypes.c_int32),
                ("npol", ctypes.c_int32), ("chirp_in_kernel", ctypes.c_int32),
                ("single_launch", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("fft_len", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("nfront", ctypes.c_int32), ("step", ctypes.c_int32),
                ("nblocks", ctypes.c_int64), ("t_int", ctypes.c_int64),
                ("front", ctypes.c_int32), ("back", ctypes.c_int32),
                ("d_max", ctypes.c_int64), ("ws_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FullbandInfo(ctypes.Structure):
    _fields_ = [("fft_len", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("nfront", ctypes.c_int32), ("step", ctypes.c_int32),
                ("nsamp", ctypes.c_int64), ("nblocks", ctypes.c_int64),
                ("t_int", ctypes.c_int64), ("front", ctypes.c_int32),
                ("back", ctypes.c_int32), ("ws_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BeamDesc(ctypes.Structure):
    _fields_ = [("voltages", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("nchan", ctypes.c_int32), ("nsamp", ctypes.c_int64),
                ("f_centre_mhz", ctypes.c_double), ("bw_mhz", ctypes.c_double),
                ("host_dms", ctypes.POINTER(ctypes.c_double)), ("ndm", ctypes.c_int32),
                ("n_int", ctypes.c_int32), ("fft_len", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("intensity", ctypes.c_void_p),
                ("coverage", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 4), ("count", ctypes.c_int64 * 4)]


STAGES = ("transpose", "delays", "block", "dsum")


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_streams", ctypes.c_int32),
                ("queue_depth", ctypes.c_int32), ("reserved", ctypes.c_int32 * 6)]


class StreamDesc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("nchan", ctypes.c_int32),
                ("f_centre_mhz", ctypes.c_double), ("bw_mhz", ctypes.c_double),
                ("dm", ctypes.c_double), ("fft_len", ctypes.c_int32), ("n_int", ctypes.c_int32),
                ("max_block", ctypes.c_int64), ("phase_mode", ctypes.c_int32),
                ("taper", ctypes.c_int32), ("block_len", ctypes.c_int64),
                ("reserved", ctypes.c_int32 * 2)]


class ServerStats(ctypes.Structure):
    _fields_ = [("blocks_in", ctypes.c_int64), ("blocks_done", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("gaps", ctypes.c_int64),
                ("admitted", ctypes.c_int64), ("refused", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("lat_p50_ms", ctypes.c_double),
                ("lat_p99_ms", ctypes.c_double), ("lat_max_ms", ctypes.c_double),
                ("data_s", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("hbm_used", ctypes.c_size_t), ("hbm_budget", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("fft_len", ctypes.c_int32), ("kernel_variant", ctypes.c_int32),
                ("ms", ctypes.c_double), ("msamples_per_s", ctypes.c_double),
                ("dm_tile", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libcdd.so is not built (%s); run __graft_entry__.build()" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, f64, vp, sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_void_p, ctypes.c_size_t)
    lib.cdd_query.argtypes = [i32, i64, i32, f64, f64, f64, i32, i32, i32,
                              ctypes.POINTER(Opts), ctypes.POINTER(PlanInfo)]
    lib.cdd_dedisperse.argtypes = [vp, i32, i64, i32, f64, f64, f64, i32, i32, vp, vp, vp,
                                   vp, ctypes.POINTER(Opts), vp, sz, vp]
    lib.cdd_dedisperse_noalloc.argtypes = [vp, i32, i64, i32, f64, f64, f64, i32, i32, vp, vp,
                                           vp, vp, ctypes.POINTER(Opts), vp]
    lib.cdd_dedisperse_noalloc.restype = ctypes.c_int
    lib.cdd_plan_create.argtypes = [ctypes.POINTER(BeamDesc), i32, ctypes.POINTER(Opts),
                                    ctypes.POINTER(vp)]
    lib.cdd_plan_info_get.argtypes = [vp, i32, ctypes.POINTER(PlanInfo)]
    lib.cdd_plan_execute.argtypes = [vp, vp, sz, vp]
    lib.cdd_plan_destroy.argtypes = [vp]
    lib.cdd_plan_destroy.restype = None
    for f in ("cdd_query", "cdd_dedisperse", "cdd_plan_create", "cdd_plan_info_get",
              "cdd_plan_execute"):
        getattr(lib, f).restype = ctypes.c_int
    lib.cdd_profile_enable.argtypes = [i32]
    lib.cdd_profile_enable.restype = ctypes.c_int
    lib.cdd_profile_select.argtypes = [ctypes.c_uint32]
    lib.cdd_profile_select.restype = ctypes.c_int
    lib.cdd_profile_read.argtypes = [ctypes.POINTER(Profile)]
    lib.cdd_profile_read.restype = ctypes.c_int
    lib.cdd_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.cdd_server_destroy.argtypes = [vp]
    lib.cdd_server_destroy.restype = None
    lib.cdd_stream_open.argtypes = [vp, ctypes.POINTER(StreamDesc), ctypes.POINTER(i32)]
    lib.cdd_stream_push.argtypes = [vp, i32, vp, i64, ctypes.c_uint64]
    lib.cdd_stream_poll.argtypes = [vp, i32, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.cdd_stream_close.argtypes = [vp, i32]
    lib.cdd_stream_invalid.argtypes = [vp, i32, vp, i64, ctypes.POINTER(i64)]
    lib.cdd_server_sync.argtypes = [vp]
    lib.cdd_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    for f in ("cdd_server_create", "cdd_stream_open", "cdd_stream_push", "cdd_stream_poll",
              "cdd_stream_close", "cdd_stream_invalid", "cdd_server_sync",
              "cdd_server_stats_get"):
        getattr(lib, f).restype = ctypes.c_int
    lib.cdd_autotune.argtypes = [i32, i32, f64, f64, ctypes.POINTER(f64), i32, i32, i32, i32,
                                 ctypes.POINTER(TuneResult)]
    lib.cdd_autotune.restype = ctypes.c_int
    lib.cdd_last_error.restype = ctypes.c_char_p
    lib.cdd_last_error.argtypes = []
    lib.cdd_status_str.restype = ctypes.c_char_p
    lib.cdd_status_str.argtypes = [ctypes.c_int]
    lib.cdd_abi_version.restype = ctypes.c_int32
    lib.cdd_kernel_variants.argtypes = [i32]
    lib.cdd_kernel_variants.restype = ctypes.c_int32
    lib.cdd_incoherent_ws_bytes.argtypes = [i32, i64, i32, i32]
    lib.cdd_incoherent_ws_bytes.restype = sz
    lib.cdd_incoherent.argtypes = [vp, i32, i64, i32, f64, f64, f64, i32, vp, vp, vp,
                                   ctypes.POINTER(Opts), vp, sz, vp]
    lib.cdd_incoherent.restype = ctypes.c_int
    lib.cdd_fold.argtypes = [vp, i64, f64, f64, i32, vp, vp, vp]
    lib.cdd_fold.restype = ctypes.c_int
    lib.cdd_gsb_inverse.argtypes = [vp, i64, i32, vp, vp]
    lib.cdd_gsb_inverse.restype = ctypes.c_int
    lib.cdd_fullband_query.argtypes = [i64, i32, f64, f64, f64, i32, i32, ctypes.POINTER(Opts),
                                       ctypes.POINTER(FullbandInfo)]
    lib.cdd_fullband_query.restype = ctypes.c_int
    lib.cdd_fullband_dedisperse.argtypes = [vp, i64, i32, f64, f64, f64, i32, i32, vp, vp,
                                            ctypes.POINTER(Opts), vp, sz, vp]
    lib.cdd_fullband_dedisperse.restype = ctypes.c_int
    return lib


lib = _load()
LIB_PATH = _LIB_PATH


def _check(status: int):
    if status != 0:
        raise CddError(status, lib.cdd_last_error().decode())


def profile_enable(on: bool = True, stages=None):
    """Switch stage timing on or off; ``stages`` (names from STAGES) limits
    it to those stages, None times every stage."""
    mask = (1 << len(STAGES)) - 1 if stages is None else sum(1 << STAGES.index(s) for s in stages)
    _check(lib.cdd_profile_select(ctypes.c_uint32(mask)))
    _check(lib.cdd_profile_enable(int(bool(on))))


def profile_read():
    """{stage: (total_ms, count)} accumulated since the last read."""
    p = Profile()
    _check(lib.cdd_profile_read(ctypes.byref(p)))
    return {name: (p.ms[i], p.count[i]) for i, name in enumerate(STAGES)}


def autotune(nchan, f_centre, bw, dms, n_int, n_min=0, n_max=0, dtype=CDD_CI8):
    """cdd_autotune: best (fft_len, kernel_variant) for a beam shape."""
    arr = (ctypes.c_double * len(dms))(*[float(x) for x in dms])
    r = TuneResult()
    _check(lib.cdd_autotune(int(dtype), int(nchan), float(f_centre), float(bw), arr, len(dms),
                            int(n_int), int(n_min), int(n_max), ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in r._fields_}


TAPERS = {"none": 0, "hann": 1, "welch": 2}


def make_opts(fft_len=0, overlap=None, nfront=None, dm_const=0.0, phase_mode=0, variant=0,
              autotune=0, time_chunks=0, taper="none"):
    o = Opts()
    o.taper = TAPERS[taper] if isinstance(taper, str) else int(taper)
    o.kernel_variant = int(variant)
    o.autotune = int(autotune)
    o.time_chunks = int(time_chunks)
    if overlap is not None or nfront is not None:
        o.explicit_plan = 1
        o.fft_len = int(fft_len)
        o.overlap = int(overlap)
        o.nfront = int(nfront)
    o.dm_const = float(dm_const)
    o.phase_mode = int(phase_mode)
    return o


def query(dtype, nsamp, nchan, f_centre, bw, dm, fft_len=0, n_int=1, want_voltages=False,
          **opt):
    """Plan figures of cdd_query as a dict (host only)."""
    info = PlanInfo()
    o = make_opts(fft_len, **opt)
    _check(lib.cdd_query(int(dtype), int(nsamp), int(nchan), float(f_centre), float(bw),
                         float(dm), int(fft_len), int(n_int), int(bool(want_voltages)),
                         ctypes.byref(o), ctypes.byref(info)))
    return info.as_dict()


def _layout(v):
    """(dtype code, nsamp, nchan) of a time-major voltage tensor."""
    import torch
    if v.dtype == torch.int8:
        if v.dim() != 3 or v.shape[2] != 2:
            raise ValueError("int8 voltages must be [nsamp][nchan][2]")
        return CDD_CI8, v.shape[0], v.shape[1]
    if v.dtype == torch.complex64:
        if v.dim() == 1:
            return CDD_CF32, v.shape[0], 1
        if v.dim() == 2:
            return CDD_CF32, v.shape[0], v.shape[1]
    raise ValueError("voltages must be int8 [T][C][2] or complex64 [T][C]")


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def dedisperse(voltages, f_centre, bw, dm, fft_len=0, n_int=1, *, want_chan=False,
               want_voltages=False, overlap=None, nfront=None, dm_const=0.0, phase_mode=0,
               variant=0, time_chunks=0, taper="none", npol=1, stream=None, out=None):
    """Run cdd_dedisperse on a resident device tensor.

    With npol=2 the tensor holds two polarisation records, [2][nsamp][...],
    whose detected intensities are summed.

    Returns a dict: I [t_int] float32, cov [t_int] int32, P [nchan][t_int]
    (if want_chan), y [nchan][nsamp] complex64 (if want_voltages), info.
    ``out`` may pass preallocated tensors (keys I, cov, P, y, ws).
    """
    import torch
    if not voltages.is_cuda or not voltages.is_contiguous():
        raise ValueError("voltages must be a contiguous device tensor")
    if npol == 2:
        if voltages.shape[0] != 2:
            raise ValueError("npol=2 needs voltages shaped [2][nsamp][...]")
        dt, nsamp, nchan = _layout(voltages[0])
    else:
        dt, nsamp, nchan = _layout(voltages)
    o = make_opts(fft_len, overlap, nfront, dm_const, phase_mode, variant,
                  time_chunks=time_chunks, taper=taper)
    o.npol = int(npol)
    info = PlanInfo()
    _check(lib.cdd_query(dt, nsamp, nchan, float(f_centre), float(bw), float(dm), int(fft_len),
                         int(n_int), int(want_voltages), ctypes.byref(o), ctypes.byref(info)))
    dev = voltages.device
    out = dict(out or {})
    t_int = info.t_int
    if "I" not in out:
        out["I"] = torch.empty(t_int, dtype=torch.float32, device=dev)
    if "cov" not in out:
        out["cov"] = torch.empty(t_int, dtype=torch.int32, device=dev)
    if want_chan and "P" not in out:
        out["P"] = torch.empty((nchan, t_int), dtype=torch.float32, device=dev)
    if want_voltages and "y" not in out:
        out["y"] = torch.empty((nchan, nsamp), dtype=torch.complex64, device=dev)
    if "ws" not in out or out["ws"].numel() < info.ws_bytes:
        out["ws"] = torch.empty(max(info.ws_bytes, 256), dtype=torch.uint8, device=dev)
    ptr = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None  # noqa: E731
    _check(lib.cdd_dedisperse(ctypes.c_void_p(voltages.data_ptr()), dt, nsamp, nchan,
                              float(f_centre), float(bw), float(dm), int(fft_len), int(n_int),
                              ptr("I"), ptr("cov"), ptr("P") if want_chan else None,
                              ptr("y") if want_voltages else None, ctypes.byref(o),
                              ptr("ws"), out["ws"].numel(), _stream_handle(stream)))
    out["info"] = info.as_dict()
    return out


def dedisperse_noalloc(voltages, f_centre, bw, dm, fft_len=0, n_int=1, *, want_chan=False,
                       want_voltages=False, overlap=None, nfront=None, dm_const=0.0,
                       phase_mode=0, taper="none", stream=None, out=None):
    """Run cdd_dedisperse_noalloc (the library's static scratch instead of a
    workspace).  Outputs as dedisperse; ``out`` may pass preallocated tensors
    (keys I, cov, P, y), and with all of them given this call allocates
    nothing on the device."""
    import torch
    if not voltages.is_cuda or not voltages.is_contiguous():
        raise ValueError("voltages must be a contiguous device tensor")
    dt, nsamp, nchan = _layout(voltages)
    o = make_opts(fft_len, overlap, nfront, dm_const, phase_mode, 0, taper=taper)
    info = PlanInfo()
    _check(lib.cdd_query(dt, nsamp, nchan, float(f_centre), float(bw), float(dm), int(fft_len),
                         int(n_int), int(want_voltages), ctypes.byref(o), ctypes.byref(info)))
    dev = voltages.device
    out = dict(out or {})
    t_int = info.t_int
    if "I" not in out:
        out["I"] = torch.empty(t_int, dtype=torch.float32, device=dev)
    if "cov" not in out:
        out["cov"] = torch.empty(t_int, dtype=torch.int32, device=dev)
    if want_chan and "P" not in out:
        out["P"] = torch.empty((nchan, t_int), dtype=torch.float32, device=dev)
    if want_voltages and "y" not in out:
        out["y"] = torch.empty((nchan, nsamp), dtype=torch.complex64, device=dev)
    ptr = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None  # noqa: E731
    _check(lib.cdd_dedisperse_noalloc(ctypes.c_void_p(voltages.data_ptr()), dt, nsamp, nchan,
                                      float(f_centre), float(bw), float(dm), int(fft_len),
                                      int(n_int), ptr("I"), ptr("cov"),
                                      ptr("P") if want_chan else None,
                                      ptr("y") if want_voltages else None, ctypes.byref(o),
                                      _stream_handle(stream)))
    out["info"] = info.as_dict()
    return out


def incoherent(voltages, f_centre, bw, dm, n_int=1, *, want_chan=False, dm_const=0.0,
               stream=None, out=None):
    """Run cdd_incoherent (detection, integration and the delay-aligned sum
    without the coherent step) on a resident device tensor.  Returns a dict
    with I, cov and, if want_chan, P."""
    import torch
    if not voltages.is_cuda or not voltages.is_contiguous():
        raise ValueError("voltages must be a contiguous device tensor")
    dt, nsamp, nchan = _layout(voltages)
    o = make_opts(dm_const=dm_const)
    ws = lib.cdd_incoherent_ws_bytes(dt, nsamp, nchan, int(n_int))
    if ws == 0:
        raise CddError(-1, "cdd_incoherent_ws_bytes: invalid shape")
    dev = voltages.device
    out = dict(out or {})
    t_int = nsamp // int(n_int)
    if "I" not in out:
        out["I"] = torch.empty(t_int, dtype=torch.float32, device=dev)
    if "cov" not in out:
        out["cov"] = torch.empty(t_int, dtype=torch.int32, device=dev)
    if want_chan and "P" not in out:
        out["P"] = torch.empty((nchan, t_int), dtype=torch.float32, device=dev)
    if "ws" not in out or out["ws"].numel() < ws:
        out["ws"] = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    ptr = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None  # noqa: E731
    _check(lib.cdd_incoherent(ctypes.c_void_p(voltages.data_ptr()), dt, nsamp, nchan,
                              float(f_centre), float(bw), float(dm), int(n_int), ptr("I"),
                              ptr("cov"), ptr("P") if want_chan else None, ctypes.byref(o),
                              ptr("ws"), out["ws"].numel(), _stream_handle(stream)))
    return out


def fold(intensity, period, phase0=0.0, nbins=128, stream=None):
    """cdd_fold of a device float series: (profile [nbins] float32, counts
    [nbins] int32) device tensors."""
    import torch
    if not intensity.is_cuda or intensity.dtype != torch.float32 or intensity.dim() != 1:
        raise ValueError("intensity must be a 1-D float32 device tensor")
    x = intensity.contiguous()
    prof = torch.empty(int(nbins), dtype=torch.float32, device=x.device)
    cnt = torch.empty(int(nbins), dtype=torch.int32, device=x.device)
    _check(lib.cdd_fold(ctypes.c_void_p(x.data_ptr()), x.numel(), float(period), float(phase0),
                        int(nbins), ctypes.c_void_p(prof.data_ptr()),
                        ctypes.c_void_p(cnt.data_ptr()), _stream_handle(stream)))
    return prof, cnt


def _records(spectra):
    """(nspec, nchan) of a device int8 [nspec][nchan][2] record tensor."""
    import torch
    if (not spectra.is_cuda or spectra.dtype != torch.int8 or spectra.dim() != 3
            or spectra.shape[2] != 2 or not spectra.is_contiguous()):
        raise ValueError("spectra must be a contiguous int8 device tensor [nspec][nchan][2]")
    return spectra.shape[0], spectra.shape[1]


def gsb_inverse(spectra, stream=None, out=None):
    """cdd_gsb_inverse: recorded real-FFT spectra [nspec][nchan][2] int8 ->
    the real series [nspec * 2 nchan] float32 (device tensors)."""
    import torch
    nspec, nchan = _records(spectra)
    if out is None:
        out = torch.empty(nspec * 2 * nchan, dtype=torch.float32, device=spectra.device)
    _check(lib.cdd_gsb_inverse(ctypes.c_void_p(spectra.data_ptr()), nspec, nchan,
                               ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def fullband_query(nspec, nchan, f_centre, bw, dm, n_int=2, fft_len=0, **opt):
    """Plan figures of cdd_fullband_query (host only)."""
    info = FullbandInfo()
    o = make_opts(fft_len, **opt)
    _check(lib.cdd_fullband_query(int(nspec), int(nchan), float(f_centre), float(bw), float(dm),
                                  int(fft_len), int(n_int), ctypes.byref(o), ctypes.byref(info)))
    return info.as_dict()


def fullband(spectra, f_centre, bw, dm, n_int=2, fft_len=0, *, overlap=None, nfront=None,
             dm_const=0.0, taper="none", want_voltages=False, stream=None, out=None):
    """cdd_fullband_dedisperse on resident records: returns a dict with I
    [t_int] float32, y [nsamp] float32 (the dedispersed real series, if
    want_voltages) and info.  ``out`` may pass preallocated I, y, ws."""
    import torch
    nspec, nchan = _records(spectra)
    o = make_opts(fft_len, overlap, nfront, dm_const, taper=taper)
    info = FullbandInfo()
    _check(lib.cdd_fullband_query(nspec, nchan, float(f_centre), float(bw), float(dm),
                                  int(fft_len), int(n_int), ctypes.byref(o), ctypes.byref(info)))
    dev = spectra.device
    out = dict(out or {})
    if "I" not in out:
        out["I"] = torch.empty(info.t_int, dtype=torch.float32, device=dev)
    if want_voltages and "y" not in out:
        out["y"] = torch.empty(info.nsamp, dtype=torch.float32, device=dev)
    if "ws" not in out or out["ws"].numel() < info.ws_bytes:
        out["ws"] = torch.empty(max(info.ws_bytes, 256), dtype=torch.uint8, device=dev)
    _check(lib.cdd_fullband_dedisperse(
        ctypes.c_void_p(spectra.data_ptr()), nspec, nchan, float(f_centre), float(bw), float(dm),
        int(fft_len), int(n_int), ctypes.c_void_p(out["I"].data_ptr()),
        ctypes.c_void_p(out["y"].data_ptr()) if want_voltages else None, ctypes.byref(o),
        ctypes.c_void_p(out["ws"].data_ptr()), out["ws"].numel(), _stream_handle(stream)))
    out["info"] = info.as_dict()
    return out


class Plan:
    """Batched DM trials over one or more beams (cdd_plan_*).

    beams: list of dicts with keys voltages (device tensor), f_centre, bw,
    dms (list of float), n_int, and optionally fft_len.  Output tensors are
    allocated here: ``self.I[b]`` [ndm][t_int], ``self.cov[b]``.
    """

    def __init__(self, beams, dm_const=0.0, phase_mode=0, fft_len=0, overlap=None,
                 nfront=None, autotune=False, variant=0, taper="none", chirp_in_kernel=False,
                 single_launch=False):
        import torch
        self._descs = (BeamDesc * len(beams))()
        self._keep = []
        self.I, self.cov = [], []
        for i, b in enumerate(beams):
            v = b["voltages"]
            dt, nsamp, nchan = _layout(v)
            dms = (ctypes.c_double * len(b["dms"]))(*[float(x) for x in b["dms"]])
            n_int = int(b.get("n_int", 1))
            t_int = nsamp // n_int
            I = torch.empty((len(b["dms"]), t_int), dtype=torch.float32, device=v.device)
            cov = torch.empty((len(b["dms"]), t_int), dtype=torch.int32, device=v.device)
            self.I.append(I)
            self.cov.append(cov)
            self._keep += [v, dms]
            d = self._descs[i]
            d.voltages, d.dtype, d.nchan, d.nsamp = v.data_ptr(), dt, nchan, nsamp
            d.f_centre_mhz, d.bw_mhz = float(b["f_centre"]), float(b["bw"])
            d.host_dms, d.ndm, d.n_int = dms, len(b["dms"]), n_int
            d.fft_len = int(b.get("fft_len", fft_len))
            d.intensity, d.coverage = I.data_ptr(), cov.data_ptr()
        o = make_opts(fft_len, overlap, nfront, dm_const, phase_mode, variant=variant,
                      autotune=autotune, taper=taper)
        o.chirp_in_kernel = int(bool(chirp_in_kernel))
        o.single_launch = int(bool(single_launch))
        h = ctypes.c_void_p()
        _check(lib.cdd_plan_create(self._descs, len(beams), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        info = self.info(0)
        self.ws = torch.empty(max(info["ws_bytes"], 256), dtype=torch.uint8,
                              device=beams[0]["voltages"].device)

    def info(self, beam):
        inf = PlanInfo()
        _check(lib.cdd_plan_info_get(self._h, int(beam), ctypes.byref(inf)))
        return inf.as_dict()

    def execute(self, stream=None):
        _check(lib.cdd_plan_execute(self._h, ctypes.c_void_p(self.ws.data_ptr()),
                                    self.ws.numel(), _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib.cdd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Real-time serving (cdd_server_* / cdd_stream_*): host numpy blocks in,
    aligned intensities out."""

    def __init__(self, hbm_budget=0, max_streams=0, queue_depth=0):
        o = ServerOpts()
        o.hbm_budget, o.max_streams, o.queue_depth = int(hbm_budget), int(max_streams), \
            int(queue_depth)
        h = ctypes.c_void_p()
        _check(lib.cdd_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def open(self, dtype, nchan, f_centre, bw, dm, n_int, max_block, fft_len=0, phase_mode=0,
             taper="none", block_len=0):
        d = StreamDesc()
        d.block_len = int(block_len)
        d.dtype, d.nchan, d.f_centre_mhz, d.bw_mhz, d.dm = int(dtype), int(nchan), \
            float(f_centre), float(bw), float(dm)
        d.fft_len, d.n_int, d.max_block, d.phase_mode = int(fft_len), int(n_int), \
            int(max_block), int(phase_mode)
        d.taper = TAPERS[taper] if isinstance(taper, str) else int(taper)
        sid = ctypes.c_int32()
        _check(lib.cdd_stream_open(self._h, ctypes.byref(d), ctypes.byref(sid)))
        return sid.value

    def push(self, sid, block, seq):
        """block: numpy [nsamp][nchan][2] int8 or [nsamp][nchan] complex64
        (C-contiguous).  Returns the status (0, or -5 when the queue is full)."""
        import numpy as np
        b = np.ascontiguousarray(block)
        st = lib.cdd_stream_push(self._h, int(sid), ctypes.c_void_p(b.ctypes.data),
                                 int(b.shape[0]), ctypes.c_uint64(int(seq)))
        if st not in (0, -5):
            _check(st)
        return st

    def poll(self, sid, cap=1 << 20):
        import numpy as np
        out = np.empty(cap, dtype=np.float32)
        n, u0 = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.cdd_stream_poll(self._h, int(sid), ctypes.c_void_p(out.ctypes.data), cap,
                                   ctypes.byref(n), ctypes.byref(u0)))
        return u0.value, out[:n.value].copy()

    def invalid(self, sid, cap=1024):
        """[(begin, end)] output spans that include lost input."""
        buf = (ctypes.c_int64 * (2 * cap))()
        n = ctypes.c_int64()
        _check(lib.cdd_stream_invalid(self._h, int(sid), buf, cap, ctypes.byref(n)))
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(min(n.value, cap))]

    def close_stream(self, sid):
        _check(lib.cdd_stream_close(self._h, int(sid)))

    def sync(self):
        _check(lib.cdd_server_sync(self._h))

    def stats(self):
        s = ServerStats()
        _check(lib.cdd_server_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib.cdd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
