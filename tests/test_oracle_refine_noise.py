"""Noise floor of the refinement (the oracle's ascent, CPU): one VGOS-shaped
pulse (2 ms boxcar at DM 403.1, 0.31 us delay, window equal to its width)
under independent noise draws.  The refined SBD, MBD and DM scatter about
the truth without bias and their spread falls as 1/SNR -- the errors are
the statistical floor of the data, not of the method -- while a noise-free
pulse is recovered within 0.005 cell."""
import numpy as np
import pytest

from oracle import frb_oracle as O
from paper_1801_02391_amd import workloads as W

TAU, DM, WIDTH, T0 = 0.31, 403.1, 2.0, 150.0


def _refine(snr, seed, noise=True):
    f0 = W.get_workload("vgos-6bl-32x64-20000")["layout"]["if_freq_mhz"]
    wl = W.custom_workload(if_freq_mhz=f0, n_chan=64, chan_bw_mhz=0.5, t_ap_ms=0.5, n_frames=640,
                           n_stations=2, config_id=5000 + seed,
                           search=dict(dm_lo=0.0, dm_step=6.25, n_dm=80, sbd_pad=4, n_mbd=256, n_rate=8,
                                       windows=[2, 4, 8, 16], n_win_min=3, n_bl_min=1),
                           signal=dict(noise=noise, pulses=dict(kind="fixed", list=[
                               dict(t0_ms=T0, dm=DM, width_ms=WIDTH, snr=snr, delay_us=TAU)])))
    V, _ = W.generate(wl)
    lay, s = wl["layout"], wl["search"]
    g = O.build_grids(lay, s)
    cells = O.refine_cells(lay, s)
    sidx = int(np.argmin(np.abs(g["tau_s"] - TAU)))
    midx = int(np.argmin(np.abs(O.wrapped_diff(g["tau_m"], TAU, g["t_amb"]))))
    th0 = O.coarse_theta(lay, s, int(round(DM / s["dm_step"])), s["n_rate"] // 2, sidx, midx)
    cal = np.ones((lay["n_if"], lay["n_chan"]), complex)
    Vb = V[0].astype(np.complex128)
    k0, l = int(round(T0 / lay["t_ap_ms"])), int(round(WIDTH / lay["t_ap_ms"]))
    fn = lambda th: O.relaxed_power_grad(*O.relaxed_fringe(Vb, lay, s, cal, k0, l, th))
    th, _ = O.newton_ascent(fn, th0, cells, O.mean_dm_shift(lay), steps=20)
    return np.array([(th[0] - TAU) / cells[0], O.wrapped_diff(th[1], TAU, g["t_amb"]) / cells[1],
                     (th[3] - DM) / cells[3]])


def test_refined_parameters_scatter_at_the_noise_floor():
    n = 16
    e10 = np.array([_refine(10.0, k) for k in range(n)])
    e20 = np.array([_refine(20.0, 100 + k) for k in range(n)])
    for E in (e10, e20):
        rms = np.sqrt((E ** 2).mean(axis=0))
        # no bias beyond the standard error of the mean (3 sigma)
        assert np.all(np.abs(E.mean(axis=0)) < 3 * rms / np.sqrt(n))
    ratio = np.sqrt((e10 ** 2).mean(axis=0)) / np.sqrt((e20 ** 2).mean(axis=0))
    # doubling the SNR halves the spread of SBD, MBD and DM
    assert np.all((ratio > 1.3) & (ratio < 3.0)), ratio
    # MBD (7.5 GHz span) is within 0.05 cell already at SNR 10; SBD (32 MHz
    # IFs) is not, and at SNR 20 comes near it
    assert np.sqrt((e10[:, 1] ** 2).mean()) < 0.05
    assert 0.05 < np.sqrt((e10[:, 0] ** 2).mean()) < 0.2


def test_noise_free_pulse_is_recovered_within_0005_cell():
    e = _refine(10.0, 0, noise=False)
    assert np.all(np.abs(e) < 0.005), e
