"""GPU tests of the float32 re-evaluation of the matrix-core forms: the
segments whose normalised power exceeds threshold - band (every crossing and
the segments near the threshold) are searched again by the float32 kernel
(one work-group per listed segment).
With a band that takes every segment, the cube must equal the float32
search's (to float32 rounding: the list kernel gathers the segment sums from
the input instead of a dedispersed copy, so the compiler may round a complex
product in another order); with a narrow band, the re-evaluated segments
carry float32 powers and cells, so the crossings and detections follow
float32 arithmetic."""
import numpy as np
import pytest
import torch

from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

from gpu_helpers import note

pytestmark = pytest.mark.gpu


def _wl(N, K=600, precision="f16", band=0.0, seed_id=140):
    # N = 4: lattice positions 0, 1, 3, 6 (one-pass f32 form); N = 9: spread (two-pass)
    f0 = [3000.0 + 32.0 * n * (n + 1) / 2 for n in range(N)]
    return W.custom_workload(
        if_freq_mhz=f0, n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=K, n_stations=3,
        config_id=seed_id + N,
        search=dict(dm_lo=0.0, dm_step=150.0, n_dm=3, sbd_pad=4, n_mbd=256, n_rate=2,
                    windows=[2, 4, 8], threshold=3.0, n_win_min=2, n_bl_min=2,
                    precision=precision, recheck_band=band),
        signal=dict(rfi_frac=0.05, rfi_amp=3.0, pulses=dict(kind="fixed", list=[
            dict(t0_ms=150.0, dm=150.0, width_ms=4.0, snr=12.0, delay_us=0.011),
            dict(t0_ms=400.0, dm=300.0, width_ms=6.0, snr=9.0, delay_us=-0.02)])))


def _run(wl, V):
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.load(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    note(f"run precision={wl['search']['precision']} band={wl['search']['recheck_band']}")
    s.run()
    P, I = s.power_cube()
    return s, P, I


def _key(c):
    return (c["baseline"], c["dm_index"], c["window_index"], c["segment"])


def _det(cands):
    return [(c["baseline"], c["dm_index"], c["window_len"], c["k0"], c["group_id"]) for c in cands]


REL = 1e-5   # list kernel vs the tiled float32 kernel


def _close(P, P32):
    return np.max(np.abs(P.astype(np.float64) - P32) / P32) <= REL


@pytest.mark.parametrize("N", [4, 9])
@pytest.mark.parametrize("prec", ["f16", "f16x3"])
def test_band_over_every_segment_reproduces_float32(prec, N):
    V, _ = W.generate(_wl(N))
    s32, P32, I32 = _run(_wl(N, precision="f32"), V)
    s, P, I = _run(_wl(N, precision=prec, band=1e9), V)
    assert s.recheck() == (1e9, P.size)
    assert _close(P, P32)
    assert np.mean(I == I32) > 0.99      # near-ties may take the other cell
    assert [_key(c) for c in s.crossings()] == [_key(c) for c in s32.crossings()]
    assert _det(s.candidates()) == _det(s32.candidates())


def test_narrow_band_takes_float32_crossings_and_detections():
    N = 9
    V, _ = W.generate(_wl(N))
    s32, P32, I32 = _run(_wl(N, precision="f32"), V)
    s16, P16, I16 = _run(_wl(N, precision="f16"), V)
    s, P, I = _run(_wl(N, precision="f16", band=0.05), V)
    band, n = s.recheck()
    assert band == 0.05 and n > 0
    changed = P.view(np.uint32) != P16.view(np.uint32)
    assert 0 < changed.sum() <= n
    # the re-evaluated segments hold the float32 search's values
    assert _close(P[changed], P32[changed])
    assert np.mean(I[changed] == I32[changed]) > 0.99
    # every crossing was re-evaluated: f32 values and cells
    cr = s.crossings()
    assert len(cr) <= n
    seg_vals = {_key(c): (c["power"], c["rate_idx"], c["sbd_idx"], c["mbd_idx"]) for c in s32.crossings()}
    common = [c for c in cr if _key(c) in seg_vals]
    assert all(abs(c["power"] - seg_vals[_key(c)][0]) <= REL * seg_vals[_key(c)][0] for c in common)
    assert np.mean([(c["rate_idx"], c["sbd_idx"], c["mbd_idx"]) == seg_vals[_key(c)][1:] for c in common]) > 0.99
    # crossings: as float32 except for ones within 1e-3 of the threshold
    a = {_key(c): c["power_norm"] for c in cr}
    b = {_key(c): c["power_norm"] for c in s32.crossings()}
    for k in set(a) ^ set(b):
        assert abs(a.get(k, b.get(k)) - 3.0) <= 1e-3
    assert _det(s.candidates()) == _det(s32.candidates())
    note(f"rechecked {n}; f16 crossings differing from f32 without recheck: "
         f"{len(set(a) ^ set(_key(c) for c in s16.crossings()))}")


def test_stream_with_full_band_equals_float32_stream():
    N, K, chunk = 4, 600, 150
    V, _ = W.generate(_wl(N, K=K))
    out = {}
    for prec, band in (("f32", 0.0), ("f16", 1e9)):
        wl = _wl(N, K=K, precision=prec, band=band)
        s = frbx.Search(wl["layout"])
        s.configure(wl["search"])
        s.stream_begin(chunk)
        cubes = []
        for i in range(K // chunk):
            s.stream_push(np.ascontiguousarray(V[..., i * chunk:(i + 1) * chunk]))
            cubes.append(s.power_cube())
        out[prec] = (cubes, s.candidates())
    for (P, I), (Q, J) in zip(out["f32"][0], out["f16"][0]):
        assert P.shape == Q.shape
        if P.size:
            assert _close(Q, P) and np.mean(I == J) > 0.99
    assert _det(out["f32"][1]) == _det(out["f16"][1])


def test_recheck_state_and_errors():
    wl = _wl(4)
    s = frbx.Search(wl["layout"])
    with pytest.raises(frbx.FrbxError):
        s._chk(frbx.lib().frbx_set_recheck(s._h, -1.0), "set_recheck")
    s.configure(wl["search"])
    assert s.recheck() == (0.0, 0)
