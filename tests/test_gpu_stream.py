"""GPU tests of the streaming search: a run in chunks (with the DM-overlap
carry) searches exactly the segments of one run over the whole data and
gives bit-identical powers and indices; FP8 e4m3 chunks with per-channel
scales give the result of the decoded data; the per-chunk Eq. 6 statistics
are those of the chunk's segments."""
import numpy as np
import pytest
import torch

from oracle import frb_oracle as O
from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

from gpu_helpers import note

pytestmark = pytest.mark.gpu


def _wl(K, R=2, precision="f32", n_mbd=64, n_if=4):
    # lattice positions 0, 1, 3, 6 (within the 8 first-pass rows of M = 64:
    # the one-pass MBD form), or with n_if = 5 also 10 (the two-pass form)
    f0 = [3000.0 + 32.0 * n * (n + 1) / 2 for n in range(n_if)]
    return W.custom_workload(
        if_freq_mhz=f0, n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=K, n_stations=3,
        config_id=130,
        search=dict(dm_lo=0.0, dm_step=120.0, n_dm=3, sbd_pad=4, n_mbd=n_mbd, n_rate=R,
                    windows=[2, 4, 8], threshold=3.0, n_win_min=2, n_bl_min=2,
                    precision=precision),
        signal=dict(pulses=dict(kind="fixed", list=[
            dict(t0_ms=210.0, dm=120.0, width_ms=4.0, snr=25.0, delay_us=0.01),
            dict(t0_ms=470.0, dm=240.0, width_ms=6.0, snr=25.0, delay_us=-0.02)])))


def _unsplit(wl, V):
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.load(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    s.run()
    P, I = s.power_cube()
    return s, P, I


def _stream(wl, chunks, kind="c64", scales=None, chunk=None):
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.stream_begin(chunk)
    nw = len(wl["search"]["windows"])
    got = [dict() for _ in range(nw)]
    stats = []
    for i, ch in enumerate(chunks):
        note(f"push {i} kind {kind}")
        if kind == "e4m3":
            s.stream_push(ch, "e4m3", scales[i])
        else:
            s.stream_push(ch, kind)
        pos = s.stream_position()
        P, I = s.power_cube()
        off = np.cumsum([0] + pos["n_seg"])
        for w in range(nw):
            for k in range(pos["n_seg"][w]):
                q = pos["first"][w] + k
                assert q not in got[w]
                got[w][q] = (P[:, :, off[w] + k].copy(), I[:, :, off[w] + k].copy())
        stats.append((pos, P, s.stats()))
    return s, got, stats


@pytest.mark.parametrize("chunk,n_if", [(150, 4), (97, 4), (97, 5)])
def test_stream_matches_unsplit_bitwise(chunk, n_if):
    K = 600
    wl = _wl(K, n_if=n_if)
    V, _ = W.generate(wl)
    s0, P0, I0 = _unsplit(wl, V)
    seg = s0.segments()
    n_chunks = K // chunk
    chunks = [np.ascontiguousarray(V[..., i * chunk:(i + 1) * chunk]) for i in range(n_chunks)]
    s, got, stats = _stream(wl, chunks, chunk=chunk)
    Kin = n_chunks * chunk
    off = np.cumsum([0] + seg["n_seg"])
    for w, l in enumerate(wl["search"]["windows"]):
        h = max(1, l // 2)
        q_max = (Kin - seg["dk_max"] - l) // h
        assert sorted(got[w]) == list(range(q_max + 1))
        for q, (P, I) in got[w].items():
            assert np.array_equal(P.view(np.uint32), P0[:, :, off[w] + q].view(np.uint32))
            assert np.array_equal(I, I0[:, :, off[w] + q])
    # per-chunk statistics: Eq. 6 over the chunk's segments of each window
    pos, P, (mean, sd, cnt) = stats[-1]
    D, nw = 3, 3
    offc = np.cumsum([0] + pos["n_seg"])
    for b in range(3):
        for d in range(D):
            for w in range(nw):
                if pos["n_seg"][w] == 0:
                    continue
                pn, mu, sdv = O.normalise(P[b, d, offc[w]:offc[w + 1]])
                row = (b * D + d) * nw + w
                assert mean[row] == pytest.approx(mu, rel=1e-12)
                assert sd[row] == pytest.approx(sdv, rel=1e-9)


def test_stream_fp8_chunks_match_decoded_data():
    K, chunk = 600, 150
    wl = _wl(K)
    V, _ = W.generate(wl)
    codes, scales, dec = [], [], []
    for i in range(K // chunk):
        c8, sc = W.to_e4m3(np.ascontiguousarray(V[..., i * chunk:(i + 1) * chunk]))
        codes.append(c8)
        scales.append(sc)
        dec.append(W.from_e4m3(c8, sc))
    Vd = np.concatenate(dec, axis=-1)
    s0, P0, I0 = _unsplit(wl, Vd)
    seg = s0.segments()
    dev = [torch.from_numpy(c).cuda() for c in codes]
    dsc = [torch.from_numpy(sc).cuda() for sc in scales]
    s, got, _ = _stream(wl, dev, kind="e4m3", scales=dsc, chunk=chunk)
    off = np.cumsum([0] + seg["n_seg"])
    n = 0
    for w in range(3):
        for q, (P, I) in got[w].items():
            assert np.array_equal(P.view(np.uint32), P0[:, :, off[w] + q].view(np.uint32))
            n += 1
    assert n > 100
    # the FP8 quantisation itself: detections of the pulses survive it
    assert any(abs(d["k0"] - 210) <= 8 for d in s.candidates())


def test_whole_run_fp8_load_equals_the_decoded_data():
    """frbx_load_e4m3 (device and host arrays) searches exactly the decoded
    values: the power cube equals a run on from_e4m3's complex64 bit for bit."""
    wl = _wl(400)
    V, _ = W.generate(wl)
    c8, sc = W.to_e4m3(V)
    _, P0, I0 = _unsplit(wl, W.from_e4m3(c8, sc))
    for dev in (True, False):
        s = frbx.Search(wl["layout"])
        s.configure(wl["search"])
        if dev:
            s.load_e4m3(torch.from_numpy(c8).cuda(), torch.from_numpy(sc).cuda())
        else:
            s.load_e4m3(c8, sc)
        s.run()
        P, I = s.power_cube()
        assert np.array_equal(P.view(np.uint32), P0.view(np.uint32)) and np.array_equal(I, I0)


def test_stream_in_the_matrix_core_form_matches_the_oracle():
    """Streaming with the f16x3 form (operand scale taken per push from the
    buffer): every pushed segment against the oracle at the float32 bar."""
    K, chunk = 600, 150
    wl = _wl(K, precision="f16x3", n_mbd=256)
    V, _ = W.generate(wl)
    chunks = [np.ascontiguousarray(V[..., i * chunk:(i + 1) * chunk]) for i in range(K // chunk)]
    s, got, _ = _stream(wl, chunks, chunk=chunk)
    g = O.build_grids(wl["layout"], wl["search"])
    N, J = wl["layout"]["n_if"], wl["layout"]["n_chan"]
    cal = np.ones((N, J))
    rng = np.random.default_rng(2)
    n = 0
    for w in range(3):
        qs = sorted(got[w])
        for q in rng.choice(qs, size=min(6, len(qs)), replace=False):
            P, I = got[w][int(q)]
            for b in range(P.shape[0]):
                d = int(rng.integers(P.shape[1]))
                po, io, s2 = O.search_row(V[b].astype(np.complex128), g, cal, d, w, q_list=[int(q)])
                assert abs(P[b, d] - po[0]) / po[0] <= 1e-4
                if (po[0] - s2[0]) / po[0] > 1e-3:
                    assert I[b, d] == io[0]
                n += 1
    assert n >= 40
