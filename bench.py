#!/usr/bin/env python3
"""Throughput of the coherent-dedispersion hot path on one MI355X.

Workload (default): the 32 MHz GMRT-like filterbank beam -- 512 channels of
62.5 kHz centred at 325 MHz, 4 s of int8 complex voltages (Gaussian sigma 20,
clipped to +-127) with a dispersed 89 ms pulse train at DM 67.9; per-channel
FFT length 8192, integration x4, delay-aligned sum to FP32 intensity.  Inputs
are seeded, synthetic and resident in device memory before timing starts.

One step = one call of the whole path (layout change, delays, fused
FFT/chirp/IFFT/detect/integrate kernel, delay-aligned sum).  Prints one JSON
line with Msamples/s (complex samples summed over channels per second), the
real-time factor, the dominant kernel's roofline figures (from HIP events
recorded on the launch stream during the timed steps) and the FP64 oracle
timed on the host on a bounded sample of the same workload.  The line also
carries every other workload as a sub-object, each measured in the same run:
64 DM trials batched against the loop, the single-channel long transforms
(2^23 and 2^26 samples), the 4096-channel beam with the errors of both phase
modes, four uneven beams in one plan against the loop, the serving loop
(paced and unpaced) and the full-band mode.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published)
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E (published)
K_DM_US = 4.148808e9       # cold-plasma constant, only to synthesise the pulses

WORKLOADS = {
    1: "single_channel_16MHz_610MHz_cf32_2^23_N2^18_nint16_dm10_voltages_out",
    2: "filterbank_32MHz_512ch_4s_int8_N8192_nint4_dm67.9",
    3: "filterbank_200MHz_4096ch_2s_int8_N8192_nint4_dm120",
    4: "multibeam_16-32-32-200MHz_512-512-1024-4096ch_1-4s_int8_nint4_autotuned",
    5: "serving_8streams_16-32-200MHz_int8_dm5-300",
    6: "fullband_16MHz_610MHz_512bin_records_2^24_real_N2^19_nint16_dm10",
}

# Serving mix: (bandwidth MHz, channels, centre MHz) per stream.
SERVING_MIX = [(16.0, 512, 610.0), (32.0, 512, 325.0), (200.0, 4096, 400.0), (16.0, 512, 610.0),
               (32.0, 512, 325.0), (200.0, 4096, 400.0), (32.0, 512, 325.0), (16.0, 512, 610.0)]


def flops_per_output_sample(N: int, M: int) -> float:
    """Algorithmic flops per output sample of the overlap-save path: two
    complex FFTs at 5 N log2 N each (the paper's Eq. 5 convention) and the
    chirp multiply (6 flops per bin), over the M samples a block keeps, plus
    detection and integration (4 flops per output sample)."""
    return (10.0 * math.log2(N) + 6.0) * N / M + 4.0


def source_digest(files=("cdd_block.hip", "cdd_fft.h", "cdd_internal.h")) -> str:
    """Digest of the sources a kernel is compiled from."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1509_00186_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None if it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        data = json.load(open(path))
        rec = data[kernel][workload]
    except Exception:
        return None
    files = rec.get("sources", ["cdd_block.hip", "cdd_fft.h", "cdd_internal.h"])
    if rec.get("source_digest") != source_digest(files):
        return None
    return rec.get("bytes_per_launch")


def make_input(cfg: int):
    import synth
    b = synth.config(cfg)
    df = b.bw / b.nchan
    fref = b.f_centre + b.bw / 2.0 - df / 2.0
    law = lambda f: K_DM_US * b.dm * (1.0 / (f * f) - 1.0 / (fref * fref))  # noqa: E731
    return b, synth.make_beam(b, synth.rng_for(cfg), law)


def _channel_task(v, b, c):
    """Channel c of the beam as a one-channel beam centred on that channel
    (the oracle then computes exactly that channel's transform and chirp)."""
    df = b.bw / b.nchan
    fc = (b.f_centre - b.bw / 2.0) + (c + 0.5) * df
    return (np.ascontiguousarray(v[:, c:c + 1]), fc, df, b.dm, b.n_int, b.fft_len)


def cpu_baseline(v, b, seconds: float):
    """The FP64 oracle on whole channels of the same beam, one core, until
    about ``seconds`` of work is done (channels taken in order, starting over
    after the last one)."""
    done, t0 = 0, time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds and n < max(8 * b.nchan, 64):
        done += _oracle_channel(_channel_task(v, b, n % b.nchan))
        n += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt / 1e6, "unit": "Msamples/s", "cores": 1, "kind": "oracle",
            "sample": "%d channel passes over the %d channels, full %d-sample duration, "
                      "FP64 numpy, %.1f s" % (n, b.nchan, b.nsamp, dt)}


def _oracle_channel(args):
    """One channel of the beam through the FP64 oracle (a worker process)."""
    import oracle as O
    col, fc, df, dm, n_int, N = args
    O.dedisperse(col, fc, df, dm, n_int, fft_len=N, overlap=128, nfront=64)
    return col.shape[0]


def cpu_baseline_all_cores(v, b, seconds: float, per_core_rate: float):
    """The same oracle on whole channels spread over the host's cores (one
    channel per task, spawned worker processes that load only numpy and the
    oracle), for about ``seconds`` of wall time."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    per_chan_s = b.nsamp / (per_core_rate * 1e6)
    n = min(8 * b.nchan, max(cores, int(cores * seconds / per_chan_s)))
    base = [_channel_task(v, b, c) for c in range(min(n, b.nchan))]
    tasks = [base[c % len(base)] for c in range(n)]
    ctx = mp.get_context("spawn")
    pool = ctx.Pool(cores)
    try:
        # start-up outside the timing; a pool that cannot start is abandoned
        pool.map_async(_oracle_channel, tasks[:cores]).get(timeout=120)
        t0 = time.perf_counter()
        done = sum(pool.map_async(_oracle_channel, tasks, chunksize=1).get(
            timeout=max(120.0, 20 * seconds)))
        dt = time.perf_counter() - t0
    except mp.TimeoutError:
        return None
    finally:
        pool.terminate()
        pool.join()
    return {"value": done / dt / 1e6, "unit": "Msamples/s", "cores": cores, "kind": "oracle",
            "sample": "%d channel passes over the %d channels, one per task over %d "
                      "processes, %.1f s" % (n, b.nchan, cores, dt)}


def fullband(cdd, torch, steps: int, warmup: int, sweep: bool = True):
    """The unchannelised mode on a 16 MHz band at 610 MHz (GSB-style records
    of 512 bins from 1024-point real FFTs, 16384 records = 2^24 real samples,
    0.52 s at 32 Msamples/s), DM 10: inverse transform of the records, then
    2^19-point real overlap-save transforms over the band, y^2 and 16-sample
    integration.  Seeded int8 noise records, resident in HBM."""
    import synth
    nspec, nchan, fcen, bw, dm, n_int = 16384, 512, 610.0, 16.0, 10.0, 16
    sp = torch.from_numpy(synth.noise_int8(synth.rng_for(6), nspec, nchan, 20.0)).cuda()
    out = cdd.fullband(sp, fcen, bw, dm, n_int)
    info = out["info"]
    for _ in range(warmup):
        cdd.fullband(sp, fcen, bw, dm, n_int, out=out)
    torch.cuda.synchronize()
    cdd.profile_read()
    cdd.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        cdd.fullband(sp, fcen, bw, dm, n_int, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    cdd.profile_enable(False)
    st = cdd.profile_read()
    T = info["nsamp"]
    r = info["fft_len"] / info["step"]
    design = fullband_design_bytes(r, n_int)
    inv_ms = st["transpose"][0] / max(st["transpose"][1], 1)
    long_ms = st["block"][0] / max(st["block"][1], 1)
    # longer transforms than the rule's minimum re-transform less overlap
    by_len = {}
    for lg in (range(20, 24) if sweep else ()):
        o2 = cdd.fullband(sp, fcen, bw, dm, n_int, fft_len=1 << lg)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            cdd.fullband(sp, fcen, bw, dm, n_int, fft_len=1 << lg, out=o2)
        torch.cuda.synchronize()
        by_len[str(1 << lg)] = round((time.perf_counter() - t1) / steps * 1e3, 4)
        del o2
    del out
    limit = fullband_dm_limit(cdd, torch, max(2, steps // 4))
    return {"workload": WORKLOADS[6], "plan": {k: info[k] for k in ("fft_len", "overlap",
                                                                   "nfront", "nblocks")},
            "ms_per_call": round(dt * 1e3, 4),
            "msamples_per_s": round(T / dt / 1e6, 1),
            "x_realtime": round(T / (2 * bw) / 1e6 / dt, 1),
            "stages_ms": {"inverse_transform": round(inv_ms, 4),
                          "long_transforms": round(long_ms, 4)},
            "design_bytes_per_sample": round(design, 2),
            "design_hbm_frac": round(design * T / dt / 1e9 / PEAK_HBM_GBS, 4),
            "inverse_transform_gbs": round(5.0 * T / (inv_ms * 1e-3) / 1e9, 1),
            "ms_per_call_by_fft_len": by_len,
            "dm_limit_sec4_5": limit}


def fullband_design_bytes(r, n_int, fft_len=0, group=16):
    """Bytes the full-band passes must move per real output sample: records in
    (1) and series out (4); column, row and column passes each read and write
    the 8-byte packed spectra of 2 samples, times the N/M re-transform of the
    overlap (above 2^23 real points the column transforms take two passes
    each way: 16 more); I written.  With integration fused into the last
    column pass (n_int/2 dividing its group of 16 pairs) two partial sums per
    group are written and read back; otherwise the power of each pair (4
    bytes per pair) is written and read back."""
    passes = 20.0 + (16.0 if fft_len > (1 << 23) else 0.0)
    base = 5.0 + passes * r + 4.0 / n_int
    if group % (n_int // 2) == 0:
        return base + 16.0 * r / (2 * group)
    return base + 4.0


def fullband_dm_limit(cdd, torch, steps):
    """The first of Sec. 4.5's memory-bound real-time limits: DM 3000 over 16 MHz
    at 610 MHz, planned by the length rule at 2^27 real points (L = 2^26),
    on 2^27 real samples (131072 records of 512 bins, 4.19 s): two blocks."""
    import synth
    nspec, nchan, fcen, bw, dm, n_int = 1 << 17, 512, 610.0, 16.0, 3000.0, 16
    sp = torch.from_numpy(synth.noise_int8(synth.rng_for(7), nspec, nchan, 20.0)).cuda()
    out = cdd.fullband(sp, fcen, bw, dm, n_int)
    info = out["info"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cdd.fullband(sp, fcen, bw, dm, n_int, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    T = info["nsamp"]
    r = info["fft_len"] / info["step"]
    design = fullband_design_bytes(r, n_int, info["fft_len"])
    del out, sp
    return {"what": "DM 3000, 16 MHz at 610 MHz, 2^27 real samples (4.19 s), n_int 16",
            "plan": {k: info[k] for k in ("fft_len", "overlap", "nfront", "nblocks")},
            "ms_per_call": round(dt * 1e3, 4),
            "x_realtime": round(T / (2 * bw) / 1e6 / dt, 1),
            "design_bytes_per_sample": round(design, 2),
            "design_hbm_frac": round(design * T / dt / 1e9 / PEAK_HBM_GBS, 4),
            "steps": steps}


def _time(fn, torch, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _time_interleaved(fns, torch, reps, rounds=3, warmup=2):
    """Seconds per call of each function, timed in alternating rounds of
    ``reps`` calls after ``warmup`` untimed calls of each (the best round of
    each counts), so that the GPU's clock ramp favours none of them."""
    for fn in fns:
        for _ in range(warmup):
            fn()
    torch.cuda.synchronize()
    best = [float("inf")] * len(fns)
    for _ in range(rounds):
        for i, fn in enumerate(fns):
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            best[i] = min(best[i], (time.perf_counter() - t0) / reps)
    return best


def multibeam(cdd, torch, reps: int = 5, vd2=None, b2=None):
    """Four beams of uneven bandwidth and length (16/32/32/200 MHz, 512/512/
    1024/4096 channels, 1-4 s, DM 10/67.9/67.9/120), seeded int8 noise: one
    plan (autotuned transform length per beam; each beam in turn, and as
    variants every beam in one launch, or every chirp formed in the kernel)
    against a loop of one-shot calls at the same plans, with the
    one-DM chirps from per-execute tables and formed in the kernel (all timed
    in alternating rounds, best round each).  With the
    resident 512-channel beam ``vd2`` it also runs the workload as specified:
    64 DM trials on that beam plus the four beams in one plan, against the
    loop of 68 one-shot calls."""
    import synth
    beams = synth.extra_beams()
    vs = [torch.from_numpy(synth.noise_int8(synth.rng_for(4, salt=i + 1), b.nsamp, b.nchan,
                                            b.sigma)).cuda() for i, b in enumerate(beams)]
    t0 = time.perf_counter()
    spec = [dict(voltages=v, f_centre=b.f_centre, bw=b.bw, dms=[b.dm], n_int=b.n_int)
            for v, b in zip(vs, beams)]
    plan = cdd.Plan(spec, autotune=True)
    t_tune = time.perf_counter() - t0
    infos = [plan.info(i) for i in range(len(beams))]
    spec_n = [dict(s, fft_len=q["fft_len"]) for s, q in zip(spec, infos)]
    plan_k = cdd.Plan(spec_n, chirp_in_kernel=True)
    plan_1 = cdd.Plan(spec_n, single_launch=True)
    outs = [cdd.dedisperse(v, b.f_centre, b.bw, b.dm, q["fft_len"], b.n_int,
                           overlap=q["overlap"], nfront=q["nfront"])
            for v, b, q in zip(vs, beams, infos)]

    def loop():
        for v, b, q, o in zip(vs, beams, infos, outs):
            cdd.dedisperse(v, b.f_centre, b.bw, b.dm, q["fft_len"], b.n_int,
                           overlap=q["overlap"], nfront=q["nfront"], out=o)
    t_plan, t_plan_k, t_plan_1, t_loop = _time_interleaved(
        [plan.execute, plan_k.execute, plan_1.execute, loop], torch, reps)
    plan_1.close()
    diff = max(float(torch.linalg.norm(plan.I[i][0] - outs[i]["I"]) /
                     torch.linalg.norm(outs[i]["I"])) for i in range(len(beams)))
    diff_k = max(float(torch.linalg.norm(plan_k.I[i][0] - outs[i]["I"]) /
                       torch.linalg.norm(outs[i]["I"])) for i in range(len(beams)))
    plan.close()
    plan_k.close()
    samples = sum(b.nchan * b.nsamp for b in beams)
    duration = max(b.nsamp / (b.bw / b.nchan * 1e6) for b in beams)
    res = {"beams": [{"bw_mhz": b.bw, "nchan": b.nchan, "nsamp": b.nsamp, "dm": b.dm,
                      "fft_len": q["fft_len"]} for b, q in zip(beams, infos)],
           "plan_ms": round(t_plan * 1e3, 3), "loop_ms": round(t_loop * 1e3, 3),
           "plan_chirp_in_kernel_ms": round(t_plan_k * 1e3, 3),
           "plan_single_launch_ms": round(t_plan_1 * 1e3, 3),
           "plan_msamples_per_s": round(samples / t_plan / 1e6, 1),
           "loop_msamples_per_s": round(samples / t_loop / 1e6, 1),
           "speedup": round(t_loop / t_plan, 3),
           "speedup_chirp_in_kernel": round(t_loop / t_plan_k, 3),
           "x_realtime": round(duration / t_plan, 1),
           "autotune_s": round(t_tune, 2), "rel_l2_plan_vs_loop": diff,
           "rel_l2_plan_chirp_in_kernel_vs_loop": diff_k}
    if vd2 is not None:
        dms = synth.config(4).dms
        allspec = [dict(voltages=vd2, f_centre=b2.f_centre, bw=b2.bw, dms=dms,
                        n_int=b2.n_int, fft_len=b2.fft_len)] + spec_n
        planc = cdd.Plan(allspec)
        ic = planc.info(0)
        o2 = [cdd.dedisperse(vd2, b2.f_centre, b2.bw, dm, b2.fft_len, b2.n_int,
                             overlap=ic["overlap"], nfront=ic["nfront"]) for dm in dms]

        def loop_all():
            for dm, o in zip(dms, o2):
                cdd.dedisperse(vd2, b2.f_centre, b2.bw, dm, b2.fft_len, b2.n_int,
                               overlap=ic["overlap"], nfront=ic["nfront"], out=o)
            loop()
        t_c, t_cl = _time_interleaved([planc.execute, loop_all], torch, 2, warmup=1)
        dc = float(torch.linalg.norm(planc.I[0] - torch.stack([o["I"] for o in o2])) /
                   torch.linalg.norm(torch.stack([o["I"] for o in o2])))
        planc.close()
        sdm = b2.nchan * b2.nsamp * len(dms) + samples
        res["as_specified"] = {
            "what": "64 DM trials on the 512-channel 32 MHz beam plus the four beams, one plan",
            "plan_ms": round(t_c * 1e3, 3), "loop_ms": round(t_cl * 1e3, 3),
            "speedup": round(t_cl / t_c, 3),
            "plan_msamples_dm_per_s": round(sdm / t_c / 1e6, 1),
            "loop_msamples_dm_per_s": round(sdm / t_cl / 1e6, 1),
            "rel_l2_plan_vs_loop_dm_trials": dc}
        # the same with the autotuner choosing every beam's transform length
        # (the loop of one-shot calls runs at the lengths it chose)
        t0 = time.perf_counter()
        plana = cdd.Plan([dict(allspec[0], fft_len=0)] + spec, autotune=True)
        t_tune_a = time.perf_counter() - t0
        ia = [plana.info(i) for i in range(1 + len(beams))]
        oa = [cdd.dedisperse(vd2, b2.f_centre, b2.bw, dm, ia[0]["fft_len"], b2.n_int,
                             overlap=ia[0]["overlap"], nfront=ia[0]["nfront"]) for dm in dms]
        oa4 = [cdd.dedisperse(v, b.f_centre, b.bw, b.dm, q["fft_len"], b.n_int,
                              overlap=q["overlap"], nfront=q["nfront"])
               for v, b, q in zip(vs, beams, ia[1:])]

        def loop_all_a():
            for dm, o in zip(dms, oa):
                cdd.dedisperse(vd2, b2.f_centre, b2.bw, dm, ia[0]["fft_len"], b2.n_int,
                               overlap=ia[0]["overlap"], nfront=ia[0]["nfront"], out=o)
            for v, b, q, o in zip(vs, beams, ia[1:], oa4):
                cdd.dedisperse(v, b.f_centre, b.bw, b.dm, q["fft_len"], b.n_int,
                               overlap=q["overlap"], nfront=q["nfront"], out=o)
        t_a, t_al = _time_interleaved([plana.execute, loop_all_a], torch, 2, warmup=1)
        da = float(torch.linalg.norm(plana.I[0] - torch.stack([o["I"] for o in oa])) /
                   torch.linalg.norm(torch.stack([o["I"] for o in oa])))
        plana.close()
        res["as_specified_autotuned"] = {
            "what": "the same plan with every beam's transform length from the autotuner",
            "fft_len": [q["fft_len"] for q in ia], "autotune_s": round(t_tune_a, 2),
            "plan_ms": round(t_a * 1e3, 3), "loop_ms": round(t_al * 1e3, 3),
            "speedup": round(t_al / t_a, 3),
            "plan_msamples_dm_per_s": round(sdm / t_a / 1e6, 1),
            "loop_msamples_dm_per_s": round(sdm / t_al / 1e6, 1),
            "rel_l2_plan_vs_loop_dm_trials": da}
    return res


def polarisations_and_fold(cdd, torch, vd, b, steps: int, ms_one: float):
    """Two polarisation records of the workload (the second a seeded
    permutation of the first in time) dedispersed in one call with their
    intensities summed, then the aligned sum folded at the pulse period into
    256 bins."""
    g = torch.Generator(device="cpu").manual_seed(1509)
    perm = torch.randperm(b.nsamp, generator=g).to(vd.device)
    two = torch.stack([vd, vd[perm]]).contiguous()
    o = cdd.dedisperse(two, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, npol=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cdd.dedisperse(two, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, npol=2, out=o)
    torch.cuda.synchronize()
    ms2 = (time.perf_counter() - t0) / steps * 1e3
    period = b.period_s * 1e6 / (b.n_int / (b.bw / b.nchan))  # integrated samples
    cdd.fold(o["I"], period, 0.0, 256)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prof, cnt = cdd.fold(o["I"], period, 0.0, 256)
    torch.cuda.synchronize()
    msf = (time.perf_counter() - t0) / steps * 1e3
    del two
    return {"npol2_ms_per_step": round(ms2, 4),
            "npol2_msamples_per_s": round(2 * b.nchan * b.nsamp / (ms2 * 1e-3) / 1e6, 1),
            "npol2_cost_vs_one": round(ms2 / ms_one, 3),
            "fold_ms": round(msf, 4), "fold_bins": 256,
            "fold_period_samples": round(period, 3),
            "fold_counts_total": int(cnt.sum().item())}


def dm_trials(cdd, torch, vd, b, info, reps: int = 5, taper: str = "none",
              autotune: bool = False):
    """64 DM trials (60.0 + 0.254 i) on the same resident beam: the batched
    plan (forward transform shared, one persistent launch per 64 trials)
    against a plain loop of single-DM calls at the same (N, L, nfront), timed
    in alternating rounds (best round each).  With
    ``autotune`` the plan's transform length and schedule come from the
    autotuner (2^11 .. 2^14) instead of the beam's N."""
    import synth
    dms = synth.config(4).dms
    plan = cdd.Plan([dict(voltages=vd, f_centre=b.f_centre, bw=b.bw, dms=dms, n_int=b.n_int,
                          fft_len=0 if autotune else b.fft_len)], taper=taper,
                    autotune=autotune)
    pi = plan.info(0)
    outs = [cdd.dedisperse(vd, b.f_centre, b.bw, dm, pi["fft_len"], b.n_int,
                           overlap=pi["overlap"], nfront=pi["nfront"], taper=taper)
            for dm in dms]

    def loop():
        for dm, o in zip(dms, outs):
            cdd.dedisperse(vd, b.f_centre, b.bw, dm, pi["fft_len"], b.n_int,
                           overlap=pi["overlap"], nfront=pi["nfront"], taper=taper, out=o)
    t_batch, t_loop = _time_interleaved([plan.execute, loop], torch, reps, rounds=2, warmup=1)
    tuned = (cdd.autotune(b.nchan, b.f_centre, b.bw, dms, b.n_int) if autotune else None)
    I_loop = torch.stack([o["I"] for o in outs])
    diff = float(torch.linalg.norm(plan.I[0] - I_loop) / torch.linalg.norm(I_loop))
    plan.close()
    sdm = b.nchan * b.nsamp * len(dms)
    return {"ndm": len(dms), "dm_range": [dms[0], dms[-1]],
            "plan": {"fft_len": pi["fft_len"], "overlap": pi["overlap"], "nfront": pi["nfront"]},
            "autotuner_choice": tuned,
            "batched_ms": round(t_batch * 1e3, 3), "loop_ms": round(t_loop * 1e3, 3),
            "batched_msamples_dm_per_s": round(sdm / t_batch / 1e6, 1),
            "loop_msamples_dm_per_s": round(sdm / t_loop / 1e6, 1),
            "speedup": round(t_loop / t_batch, 3), "rel_l2_batched_vs_loop": diff}


def serving(cdd, seconds: float, paced: bool):
    """Eight streams (16/32/200 MHz, DM log-uniform in [5, 300]) pushed in
    blocks of 2^20..2^24 samples (all channels) -- at their true sample rates
    when paced, as fast as the server accepts them otherwise.  Each stream
    cycles through 0.5 s of seeded int8 data."""
    import threading
    import synth
    rng = np.random.default_rng(synth.SEED_BASE + 5)
    sv = cdd.Server(hbm_budget=64 << 30)
    streams = []
    for k, (bw, nchan, fc) in enumerate(SERVING_MIX):
        dm = float(np.exp(rng.uniform(np.log(5.0), np.log(300.0))))
        per_chan = [(1 << int(e)) // nchan for e in rng.integers(20, 25, size=64)]
        rate = bw / nchan * 1e6                          # samples/s per channel
        nbuf = int(0.5 * rate)
        beam = synth.Beam(fc, bw, nchan, nbuf, dm)
        data = synth.noise_int8(np.random.default_rng(synth.SEED_BASE + 50 + k), nbuf, nchan,
                                beam.sigma)
        sid = sv.open(0, nchan, fc, bw, dm, 4, max(per_chan))
        streams.append(dict(sid=sid, data=data, sizes=per_chan, rate=rate, dm=dm, pos=0, seq=0,
                            next_t=0.0, pushed=0))
    t0 = time.perf_counter()
    deadline = t0 + seconds
    polled = [0] * len(streams)
    while True:
        now = time.perf_counter()
        if now >= deadline:
            break
        did = False
        for i, st in enumerate(streams):
            if paced and now - t0 < st["next_t"]:
                continue
            n = st["sizes"][st["seq"] % len(st["sizes"])]
            buf = st["data"]
            if st["pos"] + n > len(buf):
                st["pos"] = 0
            blk = buf[st["pos"]:st["pos"] + n]
            if sv.push(st["sid"], blk, st["seq"]) == 0:
                st["pos"] += n
                st["seq"] += 1
                st["pushed"] += n
                st["next_t"] += n / st["rate"]
                did = True
        for i, st in enumerate(streams):
            polled[i] += len(sv.poll(st["sid"])[1])
        if not did:
            time.sleep(0.0002)
    sv.sync()
    wall = time.perf_counter() - t0
    stats = sv.stats()
    for st in streams:
        sv.close_stream(st["sid"])
    sv.sync()
    sv.close()
    agg_rate = sum(st["rate"] * SERVING_MIX[i][1] for i, st in enumerate(streams))
    done = sum(st["pushed"] * SERVING_MIX[i][1] for i, st in enumerate(streams))
    return {"paced": paced, "seconds": round(wall, 2), "streams": len(streams),
            "dms": [round(st["dm"], 2) for st in streams],
            "blocks": stats["blocks_done"], "batches": stats["batches"],
            "lat_p50_ms": round(stats["lat_p50_ms"], 3), "lat_p99_ms": round(stats["lat_p99_ms"], 3),
            "lat_max_ms": round(stats["lat_max_ms"], 3),
            "msamples_per_s": round(done / wall / 1e6, 1),
            "realtime_msamples_per_s": round(agg_rate / 1e6, 1),
            "x_realtime": round(done / wall / agg_rate, 2),
            "hbm_used_gb": round(stats["hbm_used"] / 2**30, 2)}


def time_beam(cdd, torch, b, v, steps: int, warmup: int, taper: str = "none",
              want_voltages: bool = False, workload: str = "", every: int = 5, out=None):
    """One beam through the one-shot call: W untimed steps, K timed steps
    (HIP events around the transform kernel on every ``every``-th step, on
    the launch stream), then a separate profiled run of every stage.  Returns
    the figures of a bench line (value, ms per step, roofline)."""
    dev = torch.device("cuda:0")
    vd = v if torch.is_tensor(v) else torch.from_numpy(v).to(dev)
    tk = dict(taper=taper, want_voltages=want_voltages)
    if out is None:   # allocate the outputs and workspace (the first call)
        out = cdd.dedisperse(vd, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, **tk)
    info = out["info"]
    torch.cuda.synchronize()
    for _ in range(warmup):
        cdd.dedisperse(vd, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, out=out, **tk)
    torch.cuda.synchronize()
    cdd.profile_read()
    cdd.profile_enable(False, stages=["block"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if i % every == 0:
            cdd.lib.cdd_profile_enable(1)
        cdd.dedisperse(vd, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, out=out, **tk)
        if i % every == 0:
            cdd.lib.cdd_profile_enable(0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timed_steps = (steps + every - 1) // every
    stages = cdd.profile_read()
    nst = min(steps, 20)
    cdd.profile_enable(True)
    for _ in range(nst):
        cdd.dedisperse(vd, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, out=out, **tk)
    torch.cuda.synchronize()
    cdd.profile_enable(False)
    all_stages = cdd.profile_read()

    ms = dt / steps * 1e3
    samples = b.nchan * b.nsamp
    duration_s = b.nsamp / (b.bw / b.nchan * 1e6)
    blk_ms, blk_n = stages["block"]
    blk_avg = blk_ms / max(blk_n, 1)
    # the one-shot call may split the blocks over several launches: per-launch
    # figures are the step's totals divided by the launches per step
    per_step = max(1, round(blk_n / timed_steps))
    N, M = info["fft_len"], info["step"]
    fps = flops_per_output_sample(N, M)
    flops = fps * samples / per_step
    achieved = flops / (blk_avg * 1e-3) / 1e12
    in_bytes = 2 if b.int8 else 8
    out_bytes = 8 if want_voltages else 0
    alg_bytes = (samples * (in_bytes + out_bytes) + b.nchan * info["t_int"] * 4) / per_step
    res = {
        "value": round(samples / (ms * 1e-3) / 1e6, 1),
        "ms_per_step": round(ms, 4),
        "steps": steps, "warmup": warmup,
        "config": {"workload": workload, "nchan": b.nchan, "nsamp": b.nsamp,
                   "fft_len": N, "overlap": info["overlap"], "nfront": info["nfront"],
                   "n_int": b.n_int, "dm": b.dm,
                   "input": ("int8" if b.int8 else "complex64") + " time-major, resident in HBM",
                   "voltages_out": bool(want_voltages), "taper": taper},
        "x_realtime": round(duration_s / (ms * 1e-3), 1),
        "stages_ms_per_step": {k: round(t / nst, 4) for k, (t, n) in all_stages.items()},
        "stages_note": "from a separate run of %d profiled steps after the timed ones" % nst,
    }
    if N <= 16384:
        traffic = measured_traffic("block_kernel", workload)
        res["roofline"] = {
            "kernel": "block_kernel (FFT+chirp+IFFT+detect+integrate)",
            "bound": "alu", "achieved": round(achieved, 2),
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "peak_without_packed_fp32": PEAK_FP32_TFLOPS / 2,
            "frac_without_packed_fp32": round(achieved / (PEAK_FP32_TFLOPS / 2), 4),
            "traffic": traffic,
            "avg_ms": round(blk_avg, 4),
            "launches_per_step": per_step,
            "timed_launches": blk_n, "events_on_every_nth_step": every,
            "alg_flops_per_output_sample": round(fps, 3),
            "output_samples_per_launch": samples / per_step,
            "alg_flops_per_launch": round(flops),
            "alg_hbm_bytes_per_launch": round(alg_bytes),
            "alg_hbm_frac": round(alg_bytes / (blk_avg * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        res["gflops_paper_eq5"] = round(flops / (blk_avg * 1e-3) / 1e9, 1)
    else:
        # long transforms: three passes over HBM (columns, rows, inverse
        # columns with voltages out and the integration fused in).
        # Algorithmic bytes per sample: input, voltages (if asked) and the
        # integrated output; design bytes at R = N/M: input R + 8R spectra, 8R
        # + 8R, 8R + voltages + 4/n_int, plus the partial sums of the groups
        # split across column runs (two floats per run of G samples, written
        # and read: 16R/G) -- or, where n_int does not divide G, |y|^2 written
        # and read back by a separate integration (8)
        R = N / M
        lg = int(round(math.log2(N)))
        # columns per workgroup of the last column pass (length 2^(lg/2), or
        # 128 when the column transforms are split in two above 2^22)
        G = 16 if (lg > 22 or (1 << (lg // 2)) <= 512) else 8
        fused = G % b.n_int == 0
        alg = in_bytes + out_bytes + 4.0 / b.n_int
        design = ((in_bytes + 32.0 + (32.0 if lg > 22 else 0.0)) * R + 4.0 / b.n_int +
                  out_bytes + (16.0 * R / G if fused else 8.0))
        gbs = alg * samples / (blk_avg * 1e-3) / 1e9
        dgbs = design * samples / (blk_avg * 1e-3) / 1e9
        res["roofline"] = {"kernel": "four-step passes (cols_fwd, rows, cols_inv with "
                                     "integration, split-group fix-up)",
                           "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                           "traffic": measured_traffic("fourstep_passes", workload),
                           "avg_ms": round(blk_avg, 4), "launches_per_step": per_step,
                           "alg_bytes_per_sample": round(alg, 3),
                           "design_bytes_per_sample": round(design, 2),
                           "design_gbs": round(dgbs, 1),
                           "design_frac": round(dgbs / PEAK_HBM_GBS, 4),
                           "alg_flops_per_launch": round(flops)}
    return res, out, vd


def config1_leg(cdd, torch, steps: int, warmup: int, nsamp: int | None = None):
    """Single-channel 16 MHz complex baseband at 610 MHz, DM 10, N 2^18,
    L 2^17, voltages out.  At its own length (2^23 samples, with the dispersed
    pulse) or, with ``nsamp``, a longer noise-only record whose working set
    does not fit the 256 MB last-level cache."""
    import synth
    if nsamp is None:
        b, v = make_input(1)
        wl = WORKLOADS[1]
    else:
        b = synth.scaled(synth.config(1), nsamp=nsamp)
        v = synth.noise_cf32(synth.rng_for(1, salt=7), nsamp)[:, None]
        wl = WORKLOADS[1].replace("2^23", "2^%d" % int(round(math.log2(nsamp))))
        wl = wl.replace("_dm10", "_dm10_noise")
    res, out, vd = time_beam(cdd, torch, b, v, steps, warmup, want_voltages=True, workload=wl)
    del out, vd
    torch.cuda.empty_cache()
    return res


def config3_leg(cdd, torch, steps: int, warmup: int, nerr_chan: int = 48):
    """200 MHz at 400 MHz, 4096 channels, 2 s, DM 120: throughput with the
    FP64-reduced phase, and the error of both phase modes against the FP64
    oracle on sampled channels (the lowest, largest-phase ones included),
    each channel computed by the oracle as a one-channel beam at its centre."""
    import oracle as O
    import synth
    b = synth.config(3)
    v = synth.make_beam(b, synth.rng_for(3))
    res, out, vd = time_beam(cdd, torch, b, v, steps, warmup, workload=WORKLOADS[3])
    del out
    chans = sorted(set(list(range(16)) + list(np.linspace(16, b.nchan - 1, nerr_chan - 16)
                                              .astype(int))))
    df = b.bw / b.nchan
    errs = {}
    t0 = time.perf_counter()
    orc = {}
    for c in chans:
        col, fc, dfc, dm, n_int, N = _channel_task(v, b, c)
        orc[c] = O.dedisperse(col, fc, dfc, dm, n_int, fft_len=N, overlap=128, nfront=64,
                              want_voltages=True)
    t_or = time.perf_counter() - t0
    for mode, name in ((0, "fp64_reduced"), (1, "fp32")):
        g = cdd.dedisperse(vd, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, want_chan=True,
                           want_voltages=True, phase_mode=mode)
        torch.cuda.synchronize()
        idx = torch.tensor(chans, device=vd.device)
        y = g["y"].index_select(0, idx).cpu().numpy()
        P = g["P"].index_select(0, idx).cpu().numpy()
        del g
        torch.cuda.empty_cache()
        num_v = den_v = num_p = den_p = 0.0
        num_lo = den_lo = 0.0
        for i, c in enumerate(chans):
            oy, oP = orc[c]["y"][0], orc[c]["P"][0]
            dv = float(np.sum(np.abs(y[i] - oy) ** 2))
            nv = float(np.sum(np.abs(oy) ** 2))
            num_v += dv
            den_v += nv
            num_p += float(np.sum((P[i] - oP) ** 2))
            den_p += float(np.sum(oP ** 2))
            if c < 16:
                num_lo += dv
                den_lo += nv
        errs[name] = {"voltages_rel_l2": (num_v / den_v) ** 0.5,
                      "voltages_rel_l2_lowest_16_channels": (num_lo / den_lo) ** 0.5,
                      "chan_intensity_rel_l2": (num_p / den_p) ** 0.5}
    res["precision"] = dict(errs, channels=len(chans),
                            sample="%d channels (0-15 at the 300 MHz end, the rest spread "
                                   "over the band), whole 2 s each; oracle %.1f s" %
                                   (len(chans), t_or),
                            note="the full-size comparison over every channel is a GPU test")
    del vd
    torch.cuda.empty_cache()
    return res


def other_legs(cdd, torch, vd, b, args, only=""):
    """Every other workload of the benchmark, each a sub-object of the line:
    DM trials (batched against the loop, fixed and autotuned N), the full
    band, the single-channel long transforms (at 2^23 samples and at 2^26,
    beyond the last-level cache), the 4096-channel beam with both phase
    modes' errors, the four uneven beams in one plan against the loop, and
    the serving loop paced at real time and unpaced."""
    legs = []
    if not args.no_fullband:
        legs += [("fullband", lambda: fullband(cdd, torch, args.steps, args.warmup))]
    legs += [("config5_serving_paced", lambda: serving(cdd, 4.0, paced=True)),
             ("config5_serving_unpaced", lambda: serving(cdd, 2.0, paced=False)),
             ("config1_single_channel", lambda: config1_leg(cdd, torch, args.steps, args.warmup)),
             ("config1_single_channel_2^26",
              lambda: config1_leg(cdd, torch, max(5, args.steps // 4), max(2, args.warmup // 4),
                                  nsamp=1 << 26)),
             ("config3_4096ch", lambda: config3_leg(cdd, torch, args.steps, args.warmup)),
             ("config4_multibeam", lambda: multibeam(cdd, torch, vd2=vd, b2=b))]
    # the DM-trial legs last: they keep the GPU busy right up to the headline
    if not args.no_dm_trials:
        legs += [("dm_trials_autotuned",
                  lambda: dm_trials(cdd, torch, vd, b, None, taper=args.taper, autotune=True)),
                 ("dm_trials", lambda: dm_trials(cdd, torch, vd, b, None, taper=args.taper))]
    if only == "fullband_dm_limit":  # for profiling the three-level passes alone
        legs = [("fullband_dm_limit", lambda: fullband_dm_limit(cdd, torch, max(2, args.steps)))]
    if only:
        legs = [lg for lg in legs if lg[0] == only]
        if not legs:
            raise SystemExit("no leg named %r" % only)
    out = {}
    for name, fn in legs:
        try:
            out[name] = fn()
        except Exception as e:  # a failing leg is reported, not fatal to the line
            out[name] = {"error": "%s: %s" % (type(e).__name__, e)}
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print("leg done: %s" % name, file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dm-trials", action="store_true")
    ap.add_argument("--no-fullband", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps of the chosen workload")
    ap.add_argument("--no-fullband-sweep", action="store_true",
                    help="full band at the rule's transform length only")
    ap.add_argument("--taper", default="none", choices=["none", "hann", "welch"],
                    help="taper of the chirp function over each channel")
    ap.add_argument("--seconds", type=float, default=10.0, help="serving run length (config 5)")
    ap.add_argument("--nsamp", type=int, default=0,
                    help="config 1 only: a noise record of this many samples instead")
    ap.add_argument("--leg", default="",
                    help="only this sub-object of the default line (e.g. dm_trials, "
                         "dm_trials_autotuned, config4_multibeam), or fullband_dm_limit "
                         "(the 2^27-point full-band record alone), for profiling")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (on several GPUs the path would shard by "
              "channel, beam or DM trial and reduce the aligned sums); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    # The host-side oracle on all cores runs first, in spawned worker
    # processes, before this process touches the GPU.
    pre, all_cores = None, None
    if args.config in (1, 2, 3) and not args.nsamp and not args.no_cpu_baseline \
            and not args.calibrate_copy_mb:
        pre = make_input(args.config)
        b0, v0 = pre
        if b0.nchan >= 16:
            one = cpu_baseline(v0, b0, 2.0)
            all_cores = cpu_baseline_all_cores(v0, b0, min(args.cpu_seconds, 8.0), one["value"])

    import torch
    if args.calibrate_copy_mb:
        n = args.calibrate_copy_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read_per_launch": n,
                          "bytes_written_per_launch": n, "launches": args.steps}))
        return
    import paper_1509_00186_amd as cdd

    common = {"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f32"}
    if args.config == 4:
        mb = multibeam(cdd, torch)
        res = {"metric": "Msamples/s dedispersed (four uneven beams, one plan)",
               "value": mb["plan_msamples_per_s"], "unit": "Msamples/s", "steps": 3,
               "warmup": 1, "ms_per_step": mb["plan_ms"], **common,
               "data": "synthetic (seeded int8 noise)", "config": {"workload": WORKLOADS[4]},
               "x_realtime": mb["x_realtime"], "multibeam": mb}
        print(json.dumps(res), flush=True)
        return
    if args.config == 6:
        fb = fullband(cdd, torch, args.steps, args.warmup, sweep=not args.no_fullband_sweep)
        res = {"metric": "Msamples/s dedispersed (full band, real samples)",
               "value": fb["msamples_per_s"], "unit": "Msamples/s", "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": fb["ms_per_call"], **common,
               "data": "synthetic (seeded int8 noise records)",
               "config": {"workload": WORKLOADS[6]}, "x_realtime": fb["x_realtime"],
               "fullband": fb}
        print(json.dumps(res), flush=True)
        return
    if args.config == 5:
        paced = serving(cdd, args.seconds, paced=True)
        burst = serving(cdd, max(2.0, args.seconds / 5), paced=False)
        res = {"metric": "Msamples/s dedispersed (serving)", "value": burst["msamples_per_s"],
               "unit": "Msamples/s", "steps": 0, "warmup": 0, **common, "data": "synthetic",
               "config": {"workload": WORKLOADS[5]}, "paced": paced, "unpaced": burst}
        print(json.dumps(res), flush=True)
        return
    if args.config == 1 and args.nsamp:
        r = config1_leg(cdd, torch, args.steps, args.warmup, nsamp=args.nsamp)
        res = {"metric": "Msamples/s dedispersed", "unit": "Msamples/s", **common,
               "data": "synthetic", **r}
        print(json.dumps(res), flush=True)
        return

    b, v = pre if pre is not None else make_input(args.config)
    vd = torch.from_numpy(v).to(torch.device("cuda:0"))
    if args.leg:
        r = other_legs(cdd, torch, vd, b, args, only=args.leg)
        print(json.dumps({"leg": args.leg, **r}), flush=True)
        return
    samples = b.nchan * b.nsamp
    extras = {}
    # the headline's outputs and workspace are allocated first, so that no
    # allocation sits between the other legs and its warm-up steps
    out0 = cdd.dedisperse(vd, b.f_centre, b.bw, b.dm, b.fft_len, b.n_int, taper=args.taper,
                          want_voltages=args.config == 1)
    torch.cuda.synchronize()
    if args.config == 2 and not args.no_extras:
        # the other workloads first (each timed the same way, W warm-up + K
        # steps), so that the headline below runs at steady GPU clocks, as a
        # continuously fed pipeline does
        extras = other_legs(cdd, torch, vd, b, args)
    r, out, vd = time_beam(cdd, torch, b, vd, args.steps, args.warmup, taper=args.taper,
                           want_voltages=args.config == 1, workload=WORKLOADS[args.config],
                           out=out0)
    ms = r["ms_per_step"]
    res = {"metric": "Msamples/s dedispersed", "value": r["value"], "unit": "Msamples/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": r["config"], "x_realtime": r["x_realtime"],
           "stages_ms_per_step": r["stages_ms_per_step"], "stages_note": r["stages_note"],
           "roofline": r["roofline"]}
    if "gflops_paper_eq5" in r:
        res["gflops_paper_eq5"] = r["gflops_paper_eq5"]
    if not args.no_extras:
        # the incoherent baseline (no coherent step) on the same resident beam
        oi = cdd.incoherent(vd, b.f_centre, b.bw, b.dm, b.n_int)
        for _ in range(args.warmup):
            cdd.incoherent(vd, b.f_centre, b.bw, b.dm, b.n_int, out=oi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            cdd.incoherent(vd, b.f_centre, b.bw, b.dm, b.n_int, out=oi)
        torch.cuda.synchronize()
        mi = (time.perf_counter() - t0) / args.steps * 1e3
        res["incoherent_baseline"] = {"ms_per_step": round(mi, 4),
                                      "msamples_per_s": round(samples / (mi * 1e-3) / 1e6, 1),
                                      "coherent_cost_ratio": round(ms / mi, 2)}
    if args.config == 2 and not args.no_extras:
        res["polarisations_and_fold"] = polarisations_and_fold(cdd, torch, vd, b, args.steps, ms)
        res.update(extras)
        res["order_note"] = ("legs other than the headline ran before it; the headline's "
                             "warm-up and timed steps follow them")
    if not args.no_cpu_baseline and pre is not None:
        res["cpu_baseline"] = cpu_baseline(v, b, args.cpu_seconds)
        res["cpu_baseline_all_cores"] = all_cores
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
