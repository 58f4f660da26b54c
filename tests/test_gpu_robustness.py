"""Failure handling on the GPU: non-finite input samples and device memory
that runs out.

* A NaN or infinite sample spoils exactly the segments whose dedispersed
  frames include it (their power is not finite; NaN ones carry packed index
  -1); Eq. 6 is taken
  over the remaining finite powers and a spoiled segment never crosses --
  against the FP64 oracle, which takes the same reading of Eq. 6.
* A tile budget below one DM trial's dedispersed tile, and an allocation
  the device refuses, both end the search with FRBX_E_NOMEM; the context
  stays usable."""
import numpy as np
import pytest
import torch

from oracle import frb_oracle as O
from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

from gpu_helpers import MARGIN, POWER_RTOL, compare_crossings, note, oracle_cube

pytestmark = pytest.mark.gpu


def _wl(precision="f32"):
    return W.custom_workload(
        if_freq_mhz=[3000.0, 3032.0, 3096.0, 3192.0], n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0,
        n_frames=300, n_stations=3, config_id=71,
        search=dict(dm_lo=0.0, dm_step=100.0, n_dm=3, sbd_pad=4, n_mbd=256, n_rate=2,
                    windows=[2, 4, 8], threshold=3.0, n_win_min=2, n_bl_min=2, precision=precision),
        signal=dict(pulses=dict(kind="fixed", list=[
            dict(t0_ms=150.0, dm=100.0, width_ms=4.0, snr=25.0, delay_us=0.013)])))


def _spoil(V):
    """NaN in two APs of one channel of baseline 0, +inf in one sample of
    baseline 1, NaN in the DC point of baseline 2 (not fitted: no effect)."""
    V = V.copy()
    V[0, 1, 5, 100:102] = np.nan
    V[1, 2, 17, 40] = np.inf
    V[2, 0, 0, 60:200] = np.nan
    return V


def test_non_finite_samples_spoil_their_segments_only():
    wl = _wl()
    V, _ = W.generate(wl)
    Vs = _spoil(V)
    lay, srch = wl["layout"], wl["search"]
    s = frbx.Search(lay)
    s.configure(srch)
    s.load(torch.from_numpy(Vs).to("cuda:0"))
    s.run()
    P, I = s.power_cube()
    mean, sd, cnt = s.stats()
    ora = O.search(Vs, lay, srch)
    B, D = lay["n_baselines"], srch["n_dm"]
    Po, Io, S2o = oracle_cube(ora, B, D, ora["grids"]["segs"])
    bad_o = ~np.isfinite(Po)
    assert np.array_equal(~np.isfinite(P), bad_o)
    assert bad_o[0].any() and bad_o[1].any() and not bad_o[2].any()
    # all-NaN segments carry no peak index (an infinite sample can leave an
    # infinite cell, whose index is reported)
    assert np.all(I[0][bad_o[0]] == -1)
    ok = ~bad_o
    rel = np.abs(P[ok].astype(np.float64) - Po[ok]) / Po[ok]
    assert rel.max() <= POWER_RTOL
    sel = ok & ((Po - np.where(ok, S2o, 0)) / np.where(ok, Po, 1) > MARGIN)
    assert np.all(I[sel] == Io[sel])
    # Eq. 6 over the finite powers of every (baseline, DM trial, window)
    segs = ora["grids"]["segs"]
    for (b, d, wi), (mu, sdv) in ora["stats"].items():
        row = (b * D + d) * len(segs) + wi
        assert mean[row] == pytest.approx(mu, rel=1e-6)
        assert sd[row] == pytest.approx(sdv, rel=1e-5)
        assert cnt[row] == np.isfinite(ora["cube"][(b, d, wi)][0]).sum()
    n_marg = compare_crossings(s.crossings(), ora["crossings"], srch["threshold"])
    cross = s.crossings()
    off = np.cumsum([0] + [q for (_, _, q) in segs])
    for c in cross:
        assert np.isfinite(P[c["baseline"], c["dm_index"], off[c["window_index"]] + c["segment"]])
    key = lambda d: (d["baseline"], d["dm_index"], d["k0"], d["window_len"])
    assert sorted(key(d) for d in s.candidates()) == sorted(
        (d["b"], d["d"], d["k0"], d["l"]) for d in ora["detections"])
    note(f"non-finite input: {int(bad_o.sum())} spoiled segments of {bad_o.size}, "
         f"worst power rel err {rel.max():.2e}, {len(cross)} crossings ({n_marg} marginal)")


def test_non_finite_samples_in_the_matrix_core_form():
    """The f16 form on complex32 input with NaN samples: the same segments are
    spoiled, the finite ones stay within the form's 1e-3 of the oracle."""
    wl = _wl("f16")
    V, _ = W.generate(wl)
    V[0, 1, 5, 100:102] = np.nan
    H = W.to_complex32(V)
    Vq = W.from_complex32(H)
    lay, srch = wl["layout"], wl["search"]
    s = frbx.Search(lay)
    s.configure(srch)
    s.load(torch.from_numpy(H).to("cuda:0"))
    s.run()
    P, I = s.power_cube()
    ora = O.search(Vq, lay, srch)
    Po, _, _ = oracle_cube(ora, lay["n_baselines"], srch["n_dm"], ora["grids"]["segs"])
    bad = ~np.isfinite(Po)
    assert bad.any() and np.array_equal(~np.isfinite(P), bad)
    assert np.all(I[bad] == -1)
    assert (np.abs(P[~bad] - Po[~bad]) / Po[~bad]).max() <= 1e-3


def test_tile_budget_below_one_dm_trial_is_e_nomem():
    wl = _wl()
    V, _ = W.generate(wl)
    lay, srch = wl["layout"], wl["search"]
    s = frbx.Search(lay)
    s.configure(srch)
    s.load(torch.from_numpy(V).to("cuda:0"))
    seg = s.segments()
    tile = (lay["n_frames"] - seg["dk_max"]) * lay["n_if"] * lay["n_chan"] * 8
    s.set_tile_budget(tile - 8)
    with pytest.raises(frbx.FrbxError) as e:
        s.run()
    assert e.value.status == frbx.E_NOMEM and str(tile) in str(e.value)
    # exactly one trial per tile, then the default: both searches equal a
    # fresh context's
    s.set_tile_budget(tile)
    s.run()
    P1, I1 = s.power_cube()
    s.set_tile_budget(0)
    s.run()
    P2, I2 = s.power_cube()
    f = frbx.Search(lay)
    f.configure(srch)
    f.load(torch.from_numpy(V).to("cuda:0"))
    f.run()
    P0, I0 = f.power_cube()
    assert np.array_equal(P1, P0) and np.array_equal(P2, P0)
    assert np.array_equal(I1, I0) and np.array_equal(I2, I0)
    with pytest.raises(frbx.FrbxError) as e:
        s.set_tile_budget(-1)
    assert e.value.status == frbx.E_INVAL


def test_allocation_refused_by_the_device_is_e_nomem():
    """512 DM trials in one tile of 512 x 58 000 APs x 2048 channels x 8 B
    (about 490 GB, more than the GPU holds): hipMalloc fails and the search
    returns FRBX_E_NOMEM; the context still answers afterwards."""
    K = 58000
    lay = dict(n_baselines=1, n_if=32, n_chan=64, n_frames=K, t_ap_ms=0.5, chan_bw_mhz=0.5,
               if_freq_mhz=[3000.0 + 32.0 * n for n in range(32)])
    srch = dict(dm_lo=0.0, dm_step=0.01, n_dm=512, k_dm=4.149e6, sbd_pad=4, n_mbd=256,
                mbd_step_us=0.0, f_ref_fit_mhz=float("nan"), n_rate=1, rate_step=0.0,
                windows=[2, 4], threshold=3.0, n_win_min=2, n_bl_min=1)
    s = frbx.Search(lay)
    s.configure(srch)
    s.load(torch.zeros((1, 32, 64, K), dtype=torch.complex64, device="cuda:0"))
    s.set_tile_budget(1 << 50)
    with pytest.raises(frbx.FrbxError) as e:
        s.run()
    assert e.value.status == frbx.E_NOMEM
    assert s.segments()["total"] > 0
    note(f"refused allocation: {e.value}")
