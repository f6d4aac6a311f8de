"""Serving loop: streams pushed in blocks of arbitrary size equal the
whole-record result (and the oracle), are the same alone and in a mix, and
admission, sequence and queue rules hold."""
import numpy as np
import pytest

import oracle as O
from tests.util import flush, rel_l2, to_dev
from tests.test_gpu_parity import _beam_int8

pytestmark = pytest.mark.gpu


def _cdd():
    import paper_1509_00186_amd as cdd
    return cdd


def _stream_all(sv, sid, data, sizes, seq0=0):
    """Push data in blocks of the given sizes (retrying while the queue is
    full), close, wait, and return (u_first, I)."""
    import time
    pos, seq = 0, seq0
    for n in sizes:
        blk = data[pos:pos + n]
        if len(blk) == 0:
            break
        while sv.push(sid, blk, seq) == -5:
            time.sleep(0.0005)
        pos += len(blk)
        seq += 1
    assert pos == len(data)
    sv.close_stream(sid)
    sv.sync()
    u0, I = sv.poll(sid)
    return u0, I


def _push_retry(sv, sid, blk, seq):
    """Push, waiting while the stream's queue is full."""
    import time
    while sv.push(sid, blk, seq) == -5:
        time.sleep(0.0005)


def _sizes(rng, total, lo, hi):
    out, s = [], 0
    while s < total:
        n = int(rng.integers(lo, hi + 1))
        out.append(n)
        s += n
    return out


def test_stream_equals_whole_record_and_oracle():
    import torch
    cdd = _cdd()
    fcen, nchan, df, nsamp, dm, n_int, N = 325.0, 16, 0.0625, 40_000, 67.9, 4, 2048
    v = _beam_int8(90, nsamp, nchan, fcen, nchan * df, dm)
    flush("stream vs whole record")
    sv = cdd.Server()
    sid = sv.open(0, nchan, fcen, nchan * df, dm, n_int, max_block=5000, fft_len=N)
    u0, I = _stream_all(sv, sid, v, _sizes(np.random.default_rng(1), nsamp, 300, 5000))
    st = sv.stats()
    sv.close()
    assert u0 == 0 and len(I) == nsamp // n_int
    g = cdd.dedisperse(to_dev(v), fcen, nchan * df, dm, N, n_int)
    torch.cuda.synchronize()
    ref = g["I"].cpu().numpy()
    assert rel_l2(I, ref) <= 1e-6, rel_l2(I, ref)
    info = g["info"]
    o = O.dedisperse(v, fcen, nchan * df, dm, n_int, fft_len=N, overlap=info["overlap"],
                     nfront=info["nfront"])
    assert rel_l2(I, o["I"]) <= 1e-4
    assert st["blocks_done"] == st["blocks_in"] and st["rejected"] == 0 and st["gaps"] == 0
    assert st["lat_p99_ms"] > 0


@pytest.mark.parametrize("cf", [0, 1])
def test_narrow_stream_alone_matches_oracle(cf):
    """Four narrow channels, int8 or complex float, pushed in ragged blocks."""
    cdd = _cdd()
    fcen, nchan, df, nsamp, dm, N = 325.0, 4, 0.0625, 20_000, 30.0, 2048
    v = _beam_int8(103, nsamp, nchan, fcen, nchan * df, dm)
    if cf:
        v = (v[..., 0].astype(np.float32) + 1j * v[..., 1]).astype(np.complex64)
    flush(f"narrow stream cf={cf}")
    sv = cdd.Server()
    sid = sv.open(cf, nchan, fcen, nchan * df, dm, 4, 3000, N)
    u0, I = _stream_all(sv, sid, v, _sizes(np.random.default_rng(7), nsamp, 200, 3000))
    sv.close()
    q = cdd.query(cf, nsamp, nchan, fcen, nchan * df, dm, N, 4)
    o = O.dedisperse(v, fcen, nchan * df, dm, 4, fft_len=N, overlap=q["overlap"],
                     nfront=q["nfront"])
    assert u0 == 0 and len(I) == len(o["I"])
    assert rel_l2(I, o["I"]) <= 1e-4, rel_l2(I, o["I"])


def test_tapered_stream_matches_whole_record():
    """A Welch-tapered stream equals the tapered whole-record call and the
    oracle."""
    import torch
    cdd = _cdd()
    fcen, nchan, df, nsamp, dm, N = 325.0, 8, 0.0625, 20_000, 40.0, 2048
    v = _beam_int8(140, nsamp, nchan, fcen, nchan * df, dm)
    sv = cdd.Server()
    sid = sv.open(0, nchan, fcen, nchan * df, dm, 4, 3000, N, taper="welch")
    u0, I = _stream_all(sv, sid, v, _sizes(np.random.default_rng(8), nsamp, 500, 3000))
    sv.close()
    g = cdd.dedisperse(to_dev(v), fcen, nchan * df, dm, N, 4, taper="welch")
    torch.cuda.synchronize()
    assert u0 == 0 and rel_l2(I, g["I"].cpu().numpy()) <= 1e-6
    q = g["info"]
    o = O.dedisperse(v, fcen, nchan * df, dm, 4, fft_len=N, overlap=q["overlap"],
                     nfront=q["nfront"], window="welch")
    assert rel_l2(I, o["I"]) <= 1e-4


def test_stream_same_alone_and_in_a_mix():
    cdd = _cdd()
    specs = [(325.0, 16, 0.0625, 30_000, 67.9, 2048, 0),
             (610.0, 8, 0.03125, 25_000, 10.0, 1024, 0),
             (400.0, 32, 0.048828125, 12_000, 120.0, 4096, 0),
             (325.0, 4, 0.0625, 20_000, 30.0, 2048, 1)]
    data = []
    for k, (fcen, nchan, df, nsamp, dm, N, cf) in enumerate(specs):
        v = _beam_int8(100 + k, nsamp, nchan, fcen, nchan * df, dm)
        if cf:
            v = (v[..., 0].astype(np.float32) + 1j * v[..., 1]).astype(np.complex64)
        data.append(v)
    rng = np.random.default_rng(5)
    sizes = [_sizes(rng, len(d), 200, 3000) for d in data]
    # stream 0 alone
    sv = cdd.Server()
    fcen, nchan, df, nsamp, dm, N, cf = specs[0]
    sid = sv.open(0, nchan, fcen, nchan * df, dm, 4, 3000, N)
    _, alone = _stream_all(sv, sid, data[0], sizes[0])
    sv.close()
    # all four, pushes interleaved
    import time
    sv = cdd.Server()
    sids = [sv.open(cf, nchan, fcen, nchan * df, dm, 4, 3000, N)
            for (fcen, nchan, df, nsamp, dm, N, cf) in specs]
    pos, seq = [0] * 4, [0] * 4
    left = True
    while left:
        left = False
        for k in range(4):
            if seq[k] < len(sizes[k]):
                left = True
                blk = data[k][pos[k]:pos[k] + sizes[k][seq[k]]]
                while sv.push(sids[k], blk, seq[k]) == -5:
                    time.sleep(0.0005)
                pos[k] += len(blk)
                seq[k] += 1
    for s in sids:
        sv.close_stream(s)
    sv.sync()
    outs = [sv.poll(s)[1] for s in sids]
    st = sv.stats()
    sv.close()
    assert np.array_equal(outs[0], alone)          # bitwise, whatever the mix
    for k, (fcen, nchan, df, nsamp, dm, N, cf) in enumerate(specs):
        q = _cdd().query(cf, nsamp, nchan, fcen, nchan * df, dm, N, 4)
        o = O.dedisperse(data[k], fcen, nchan * df, dm, 4, fft_len=N, overlap=q["overlap"],
                         nfront=q["nfront"])
        assert rel_l2(outs[k], o["I"]) <= 1e-4, (k, rel_l2(outs[k], o["I"]))
    assert st["batches"] >= 1 and st["blocks_done"] == sum(len(s) for s in sizes)


def test_admission_by_budget():
    cdd = _cdd()
    sv = cdd.Server(hbm_budget=1)                    # nothing fits
    with pytest.raises(cdd.CddError) as ei:
        sv.open(0, 16, 325.0, 1.0, 67.9, 4, 4096, 2048)
    assert ei.value.status == -5
    sv.close()
    probe = cdd.Server()
    probe.open(0, 16, 325.0, 1.0, 67.9, 4, 4096, 2048)
    one = probe.stats()["hbm_used"]
    probe.close()
    assert one > 0
    # room for one such stream: the second is refused, and admitted once the
    # first has finished and its output has been drained
    v = _beam_int8(110, 6000, 16, 325.0, 1.0, 67.9, pulse=False)
    sv = cdd.Server(hbm_budget=one + one // 2)
    s1 = sv.open(0, 16, 325.0, 1.0, 67.9, 4, 4096, 2048)
    with pytest.raises(cdd.CddError) as ei:
        sv.open(0, 16, 325.0, 1.0, 67.9, 4, 4096, 2048)
    assert ei.value.status == -5
    _stream_all(sv, s1, v, [3000, 3000])
    assert sv.stats()["hbm_used"] == 0
    s2 = sv.open(0, 16, 325.0, 1.0, 67.9, 4, 4096, 2048)
    assert s2 != s1
    st = sv.stats()
    assert st["refused"] == 1 and st["admitted"] == 2
    sv.close()


def test_sequence_rules():
    cdd = _cdd()
    v = _beam_int8(111, 9000, 8, 325.0, 0.5, 30.0, pulse=False)
    sv = cdd.Server()
    sid = sv.open(0, 8, 325.0, 0.5, 30.0, 4, 3000, 1024)
    assert sv.push(sid, v[:3000], 0) == 0
    with pytest.raises(cdd.CddError) as ei:
        sv.push(sid, v[3000:6000], 0)                # duplicate
    assert ei.value.status == -1
    assert sv.push(sid, v[3000:6000], 2) == 0        # seq 1 lost
    with pytest.raises(cdd.CddError):
        sv.push(sid, v[:5000], 3)                    # larger than max_block
    sv.close_stream(sid)
    with pytest.raises(cdd.CddError):
        sv.push(sid, v[6000:], 3)                    # closed
    sv.sync()
    u0, I = sv.poll(sid)
    st = sv.stats()
    sv.close()
    assert st["rejected"] == 1 and st["gaps"] == 1 and st["blocks_done"] == 2
    assert u0 == 0 and len(I) == 6000 // 4 and np.all(np.isfinite(I))


def test_lost_blocks_with_declared_length_become_zeros_in_place():
    """A stream with a declared block length loses two blocks: they come back
    as zeros at their true position, so every output keeps its absolute
    index and equals the whole record with those samples zero (and the
    oracle on it: the values after the gap see a zero history); the outputs
    the lost samples reach are reported."""
    import torch
    cdd = _cdd()
    fcen, nchan, df, B, dm, n_int, N = 325.0, 16, 0.0625, 3000, 67.9, 4, 2048
    v = _beam_int8(150, 8 * B, nchan, fcen, nchan * df, dm)
    flush("stream with lost blocks 3 and 4 of 8, block_len %d" % B)
    sv = cdd.Server()
    sid = sv.open(0, nchan, fcen, nchan * df, dm, n_int, max_block=B, fft_len=N, block_len=B)
    for seq in (0, 1, 2, 5, 6, 7):
        _push_retry(sv, sid, v[seq * B:(seq + 1) * B], seq)
    sv.close_stream(sid)
    sv.sync()
    u0, I = sv.poll(sid)
    spans = sv.invalid(sid)
    st = sv.stats()
    sv.close()
    z = v.copy()
    z[3 * B:5 * B] = 0
    assert u0 == 0 and len(I) == 8 * B // n_int
    g = cdd.dedisperse(to_dev(z), fcen, nchan * df, dm, N, n_int)
    torch.cuda.synchronize()
    assert rel_l2(I, g["I"].cpu().numpy()) <= 1e-6
    info = g["info"]
    o = O.dedisperse(z, fcen, nchan * df, dm, n_int, fft_len=N, overlap=info["overlap"],
                     nfront=info["nfront"])
    assert rel_l2(I, o["I"]) <= 1e-4
    after = slice(5 * B // n_int + info["d_max"] + 64, None)   # past the lost span's reach
    assert rel_l2(I[after], o["I"][after]) <= 1e-4
    assert st["gaps"] == 1 and len(spans) == 1
    b0, b1 = spans[0]
    d = O.channel_delays(fcen, nchan * df, nchan, dm, n_int)
    assert b0 <= 3 * B // n_int - int(d.max()) and b1 >= 5 * B // n_int
    assert 0 <= b0 < b1 <= len(I) + 1


def test_lost_blocks_of_unknown_length_join_and_are_marked():
    """Without a declared block length the block after a gap joins the data
    before it: the output equals the whole-record result of the joined
    record, and the outputs the junction reaches are reported."""
    import torch
    cdd = _cdd()
    fcen, nchan, df, dm, n_int, N = 325.0, 8, 0.0625, 40.0, 4, 1024
    v = _beam_int8(151, 9000, nchan, fcen, nchan * df, dm)
    sv = cdd.Server()
    sid = sv.open(0, nchan, fcen, nchan * df, dm, n_int, max_block=4000, fft_len=N)
    _push_retry(sv, sid, v[:4000], 0)
    _push_retry(sv, sid, v[4000:7000], 2)            # seq 1 lost, length unknown
    _push_retry(sv, sid, v[7000:], 3)
    sv.close_stream(sid)
    sv.sync()
    u0, I = sv.poll(sid)
    spans = sv.invalid(sid)
    sv.close()
    g = cdd.dedisperse(to_dev(v), fcen, nchan * df, dm, N, n_int)
    torch.cuda.synchronize()
    assert len(I) == 9000 // n_int
    assert rel_l2(I, g["I"].cpu().numpy()) <= 1e-6
    assert len(spans) == 1 and spans[0][0] < 4000 // n_int < spans[0][1]
