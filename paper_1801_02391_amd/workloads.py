"""Seeded synthetic workloads for the cross-spectrum FRB search.

This module only describes workloads (array shapes, search grids, signal
recipe) and draws their input cross spectra. It holds none of the search
arithmetic (no dedispersion offsets, segment sums, fringe transforms or
peak finding); the HIP library and the FP64 oracle each implement those on
their own and both read the arrays produced here.

Input model (Liu et al. 2018, Sec. 2.2): a complex cross spectrum S(n, j, k)
per baseline, for IF n (sky frequency f0^n, lower edge, upper sideband),
frequency point j at baseband frequency j * chan_bw, and accumulation period
k of duration t_ap.  Arrays are complex64 with layout [B][N][J][K]
(time-contiguous per channel).

Signal model (ours; the paper's data are not available):
  * noise: iid circular complex Gaussian with E|z|^2 = 1 per channel/frame;
  * RFI: per station a fixed set of flagged channels; a baseline channel
    carries a tone of fixed amplitude and iid uniform phase per
    (frame, channel) iff either of its stations flags that channel;
  * pulses: a boxcar in time of width w at sky frequency f arrives at
    t0 + K_DM * DM * (f^-2 - f_top^-2) (cold-plasma dispersion, f_top the
    highest channel frequency); a frame receives amplitude A times the
    fraction of the frame the boxcar covers; the visibility phase of a
    baseline with geometric delay tau is exp(+2 pi i f tau) times a constant
    per (pulse, baseline) phase.  A = snr / sqrt(N (J - 1)) so that a single
    fully covered frame, coherently summed over the N (J - 1) fitted points,
    has the stated SNR against unit-power noise.
"""
from __future__ import annotations

import copy
import math
from itertools import combinations

import numpy as np

SEED_BASE = 1801023910
K_DM_PHYSICAL = 4.149e6  # ms MHz^2 / (pc cm^-3), cold-plasma dispersion constant


def _vgos_if_freqs():
    # 4 bands x 8 contiguous 32 MHz IFs, band lower edges in MHz.
    bases = (3000.0, 5240.0, 6360.0, 10200.0)
    return [b + 32.0 * i for b in bases for i in range(8)]


_WORKLOADS = {
    # One baseline, 8 IFs x 32 x 1 MHz from 3.0 GHz, 1 ms frames for 1 s.
    "single-1bl-8x32-1000": dict(
        config_id=1,
        layout=dict(n_stations=2, if_freq_mhz=[3000.0 + 32.0 * n for n in range(8)],
                    n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=1000),
        search=dict(dm_lo=0.0, dm_step=1000.0 / 64, n_dm=64, k_dm=4.149e6,
                    sbd_pad=4, n_mbd=256, mbd_step_us=0.0, f_ref_fit_mhz=float("nan"),
                    n_rate=1, rate_step=0.0, windows=[1, 2, 4, 8],
                    threshold=3.0, n_win_min=3, n_bl_min=1),
        signal=dict(noise=True, rfi_frac=0.0, rfi_amp=0.0,
                    pulses=dict(kind="fixed", list=[dict(t0_ms=400.0, dm=500.0, width_ms=2.0,
                                                         snr=10.0, delay_us=0.020)])),
    ),
    # VGOS-shaped: 4 stations -> 6 baselines; 4 bands x 8 IFs x 64 x 0.5 MHz;
    # 0.5 ms frames for 10 s; 5 % RFI channels; 20 pulses.
    "vgos-6bl-32x64-20000": dict(
        config_id=2,
        layout=dict(n_stations=4, if_freq_mhz=_vgos_if_freqs(), n_chan=64,
                    chan_bw_mhz=0.5, t_ap_ms=0.5, n_frames=20000),
        search=dict(dm_lo=0.0, dm_step=6.25, n_dm=256, k_dm=4.149e6,
                    sbd_pad=4, n_mbd=256, mbd_step_us=0.0, f_ref_fit_mhz=float("nan"),
                    n_rate=8, rate_step=0.0, windows=[2, 4, 8, 16],
                    threshold=3.0, n_win_min=3, n_bl_min=2),
        signal=dict(noise=True, rfi_frac=0.05, rfi_amp=3.0,
                    pulses=dict(kind="random", count=20, dm=(100.0, 1500.0),
                                width_ms=(1.0, 5.0), station_delay_us=0.5,
                                snr=(6.0, 15.0), min_sep_frames=32)),
    ),
    # Parity-sized VGOS shape: 2000 frames, 32 DM trials of 50, 4 pulses.
    "vgos-6bl-32x64-2000": dict(
        config_id=21,
        layout=dict(n_stations=4, if_freq_mhz=_vgos_if_freqs(), n_chan=64,
                    chan_bw_mhz=0.5, t_ap_ms=0.5, n_frames=2000),
        search=dict(dm_lo=0.0, dm_step=50.0, n_dm=32, k_dm=4.149e6,
                    sbd_pad=4, n_mbd=256, mbd_step_us=0.0, f_ref_fit_mhz=float("nan"),
                    n_rate=8, rate_step=0.0, windows=[2, 4, 8, 16],
                    threshold=3.0, n_win_min=3, n_bl_min=2),
        signal=dict(noise=True, rfi_frac=0.05, rfi_amp=3.0,
                    pulses=dict(kind="random", count=4, dm=(100.0, 500.0),
                                width_ms=(1.0, 5.0), station_delay_us=0.5,
                                snr=(6.0, 15.0), min_sep_frames=32)),
    ),
    # Precision form: 7 stations -> 21 baselines; the VGOS band layout with
    # 32 IFs x 128 x 0.25 MHz; 0.25 ms frames for 10 s; stored as complex32;
    # 50 pulses.
    "precision-21bl-32x128-40000": dict(
        config_id=4,
        layout=dict(n_stations=7, if_freq_mhz=_vgos_if_freqs(), n_chan=128,
                    chan_bw_mhz=0.25, t_ap_ms=0.25, n_frames=40000),
        search=dict(dm_lo=0.0, dm_step=6.25, n_dm=256, k_dm=4.149e6,
                    sbd_pad=4, n_mbd=256, mbd_step_us=0.0, f_ref_fit_mhz=float("nan"),
                    n_rate=8, rate_step=0.0, windows=[4, 8, 16, 32],
                    threshold=3.0, n_win_min=3, n_bl_min=2),
        signal=dict(noise=True, rfi_frac=0.05, rfi_amp=3.0,
                    pulses=dict(kind="random", count=50, dm=(100.0, 1500.0),
                                width_ms=(1.0, 5.0), station_delay_us=0.5,
                                snr=(6.0, 15.0), min_sep_frames=64)),
    ),
    # Streaming: 10 stations -> 45 baselines; 16 IFs x 256 x 0.125 MHz at
    # 768 MHz spacing from 2 GHz; 0.1 ms frames for 60 s, processed in 1 s
    # chunks stored as FP8 e4m3 with a per-channel scale; 2048 DM trials on
    # 0-3000; 10 % RFI channels; 200 pulses.
    "stream-45bl-16x256-600000": dict(
        config_id=5,
        layout=dict(n_stations=10, if_freq_mhz=[2000.0 + 768.0 * n for n in range(16)], n_chan=256,
                    chan_bw_mhz=0.125, t_ap_ms=0.1, n_frames=600000),
        search=dict(dm_lo=0.0, dm_step=3000.0 / 2048, n_dm=2048, k_dm=4.149e6,
                    sbd_pad=4, n_mbd=256, mbd_step_us=0.0, f_ref_fit_mhz=float("nan"),
                    n_rate=16, rate_step=0.0, windows=[10, 20, 40],
                    threshold=3.0, n_win_min=2, n_bl_min=2),
        signal=dict(noise=True, rfi_frac=0.10, rfi_amp=3.0,
                    pulses=dict(kind="random", count=200, dm=(100.0, 3000.0),
                                width_ms=(1.0, 5.0), station_delay_us=0.5,
                                snr=(5.0, 20.0), min_sep_frames=64)),
        chunk_frames=10000,
    ),
    # Paper-shaped (Sec. 3): 3 stations, 6 IFs x 32 x 0.5 MHz from 2192 MHz,
    # 1.024 ms APs, one DM trial at 26.833, windows 4..32 APs.  Shortened to
    # 20 s; periodic pulses of ~7 ms every 0.7145 s.
    "paper-3bl-6x32-19531": dict(
        config_id=3,
        layout=dict(n_stations=3, if_freq_mhz=[2192.0 + 16.0 * n for n in range(6)],
                    n_chan=32, chan_bw_mhz=0.5, t_ap_ms=1.024, n_frames=19531),
        search=dict(dm_lo=26.833, dm_step=1.0, n_dm=1, k_dm=4.149e6,
                    sbd_pad=4, n_mbd=256, mbd_step_us=0.0, f_ref_fit_mhz=float("nan"),
                    n_rate=1, rate_step=0.0, windows=[4, 8, 16, 24, 32],
                    threshold=3.0, n_win_min=3, n_bl_min=2),
        signal=dict(noise=True, rfi_frac=0.0, rfi_amp=0.0,
                    pulses=dict(kind="periodic", period_ms=714.5, first_ms=300.0,
                                dm=26.833, width_ms=7.0, snr=(4.0, 12.0),
                                station_delay_us=0.5)),
    ),
}


def to_complex32(V):
    """complex64 [..] -> float16 [.., 2] (re, im): the complex32 storage form."""
    out = np.empty(V.shape + (2,), dtype=np.float16)
    out[..., 0] = V.real
    out[..., 1] = V.imag
    return out


def from_complex32(H):
    """float16 [.., 2] -> the complex64 values it stores exactly."""
    return (H[..., 0].astype(np.float32) + 1j * H[..., 1].astype(np.float32)).astype(np.complex64)


def _e4m3_table():
    """Values of the 256 OCP FP8 e4m3 (e4m3fn) codes (NaN for 0x7f, 0xff)."""
    v = np.zeros(256)
    for b in range(256):
        e, m = (b >> 3) & 15, b & 7
        if e == 15 and m == 7:
            x = np.nan
        elif e == 0:
            x = m * 2.0 ** -9
        else:
            x = (1 + m / 8) * 2.0 ** (e - 7)
        v[b] = -x if b & 128 else x
    return v


E4M3 = _e4m3_table()


def to_e4m3(V):
    """complex64 [B][N][J][K] -> (uint8 codes [B][N][J][K][2], float32 scale
    [B][N][J]): the FP8 storage form, one scale per channel = max|re, im| / 448,
    each component rounded to the nearest e4m3 value (ties to even code)."""
    amax = np.maximum(np.abs(V.real), np.abs(V.imag)).max(axis=-1)
    scale = np.where(amax > 0, amax / 448.0, 1.0).astype(np.float32)
    pos = E4M3[:127]                        # codes 0..126, increasing
    out = np.empty(V.shape + (2,), dtype=np.uint8)
    for comp, part in ((0, V.real), (1, V.imag)):
        x = (part / scale[..., None]).astype(np.float64)
        a = np.minimum(np.abs(x), 448.0)
        hi = np.clip(np.searchsorted(pos, a, side="left"), 1, 126)
        lo = hi - 1
        dlo, dhi = a - pos[lo], pos[hi] - a
        pick = np.where((dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0)), hi, lo)
        pick = np.where(a <= 0.0, 0, pick)
        out[..., comp] = (pick | (np.signbit(x) << 7)).astype(np.uint8)
    return out, scale


def from_e4m3(codes, scale):
    """The complex64 values an FP8 chunk stores: decoded x scale in float32."""
    re = E4M3[codes[..., 0]].astype(np.float32) * scale[..., None]
    im = E4M3[codes[..., 1]].astype(np.float32) * scale[..., None]
    return (re + 1j * im).astype(np.complex64)


def workload_names():
    return list(_WORKLOADS)


def get_workload(name: str, **overrides) -> dict:
    """Return a deep copy of a named workload; `overrides` patch the
    `layout`, `search` and `signal` sections (e.g. search=dict(n_dm=4))."""
    wl = copy.deepcopy(_WORKLOADS[name])
    wl["name"] = name
    for sec, patch in overrides.items():
        wl[sec].update(patch)
    lay = wl["layout"]
    lay["n_if"] = len(lay["if_freq_mhz"])
    lay["stations"] = list(combinations(range(lay["n_stations"]), 2))
    lay["n_baselines"] = len(lay["stations"])
    return wl


def custom_workload(*, if_freq_mhz, n_chan, chan_bw_mhz, t_ap_ms, n_frames,
                    n_stations=2, search=None, signal=None, config_id=99, name="custom"):
    """Build a workload description for tests (small shapes, explicit grids)."""
    base = dict(dm_lo=0.0, dm_step=1.0, n_dm=1, k_dm=4.149e6, sbd_pad=4, n_mbd=64,
                mbd_step_us=0.0, f_ref_fit_mhz=float("nan"), n_rate=1, rate_step=0.0,
                windows=[2, 4], threshold=3.0, n_win_min=2, n_bl_min=1)
    base.update(search or {})
    sig = dict(noise=True, rfi_frac=0.0, rfi_amp=0.0, pulses=dict(kind="fixed", list=[]))
    sig.update(signal or {})
    lay = dict(n_stations=n_stations, if_freq_mhz=list(map(float, if_freq_mhz)),
               n_chan=int(n_chan), chan_bw_mhz=float(chan_bw_mhz), t_ap_ms=float(t_ap_ms),
               n_frames=int(n_frames))
    lay["n_if"] = len(lay["if_freq_mhz"])
    lay["stations"] = list(combinations(range(n_stations), 2))
    lay["n_baselines"] = len(lay["stations"])
    return dict(name=name, config_id=config_id, layout=lay, search=base, signal=sig)


def _rngs(wl):
    ss = np.random.SeedSequence(SEED_BASE + int(wl["config_id"]))
    kids = ss.spawn(2 + wl["layout"]["n_baselines"])
    return [np.random.Generator(np.random.Philox(k)) for k in kids]


def _draw_pulses(wl, rng_pulse, rng_station):
    lay, sig = wl["layout"], wl["signal"]
    t_ap, K = lay["t_ap_ms"], lay["n_frames"]
    ps = sig["pulses"]
    S = lay["n_stations"]
    out = []
    if ps["kind"] == "fixed":
        for p in ps["list"]:
            q = dict(p)
            q.setdefault("delay_us", 0.0)
            q.setdefault("rate", 0.0)
            q["baseline_delay_us"] = [q["delay_us"]] * lay["n_baselines"]
            q["phase_rad"] = [q.get("phase_rad", 0.0)] * lay["n_baselines"]
            out.append(q)
        return out
    f = _chan_freqs(lay)
    f_top = f.max()
    f_bot = f.min()
    if ps["kind"] == "periodic":
        t = ps["first_ms"]
        sweep = K_DM_PHYSICAL * ps["dm"] * (1.0 / f_bot ** 2 - 1.0 / f_top ** 2)
        while t + sweep + ps["width_ms"] + 2 * t_ap < K * t_ap:
            sd = rng_station.uniform(-ps["station_delay_us"], ps["station_delay_us"], S)
            out.append(dict(t0_ms=t, dm=ps["dm"], width_ms=ps["width_ms"],
                            snr=float(rng_pulse.uniform(*ps["snr"])),
                            baseline_delay_us=[float(sd[b] - sd[a]) for a, b in lay["stations"]],
                            phase_rad=list(rng_pulse.uniform(0, 2 * np.pi, lay["n_baselines"])),
                            rate=0.0))
            t += ps["period_ms"]
        return out
    # random pulses: DM, width, SNR uniform; arrival times separated by at
    # least min_sep_frames and fully inside the data for every channel.
    n = ps["count"]
    dms = rng_pulse.uniform(*ps["dm"], n)
    widths = rng_pulse.uniform(*ps["width_ms"], n)
    snrs = rng_pulse.uniform(*ps["snr"], n)
    sweep_max = K_DM_PHYSICAL * ps["dm"][1] * (1.0 / f_bot ** 2 - 1.0 / f_top ** 2)
    lo = 8 * t_ap
    hi = K * t_ap - sweep_max - ps["width_ms"][1] - 8 * t_ap
    if hi <= lo:
        raise ValueError("workload too short for its pulse DM range")
    sep = ps["min_sep_frames"] * t_ap
    t0s = []
    while len(t0s) < n:
        t = float(rng_pulse.uniform(lo, hi))
        if all(abs(t - u) >= sep for u in t0s):
            t0s.append(t)
    t0s.sort()
    for i in range(n):
        sd = rng_station.uniform(-ps["station_delay_us"], ps["station_delay_us"], S)
        out.append(dict(t0_ms=t0s[i], dm=float(dms[i]), width_ms=float(widths[i]),
                        snr=float(snrs[i]),
                        baseline_delay_us=[float(sd[b] - sd[a]) for a, b in lay["stations"]],
                        phase_rad=list(map(float, rng_pulse.uniform(0, 2 * np.pi, lay["n_baselines"]))),
                        rate=0.0))
    return out


def _chan_freqs(lay):
    f0 = np.asarray(lay["if_freq_mhz"], dtype=np.float64)
    j = np.arange(lay["n_chan"], dtype=np.float64)
    return f0[:, None] + j[None, :] * lay["chan_bw_mhz"]


def _add_pulse(Vb, lay, p, b):
    """Add one dispersed boxcar pulse to baseline array Vb [N][J][K]."""
    N, J, K = Vb.shape
    t_ap = lay["t_ap_ms"]
    f = _chan_freqs(lay)
    f_top = f.max()
    amp = p["snr"] / math.sqrt(N * (J - 1))
    t_start = p["t0_ms"] + K_DM_PHYSICAL * p["dm"] * (1.0 / f ** 2 - 1.0 / f_top ** 2)
    t_end = t_start + p["width_ms"]
    k_first = np.floor(t_start / t_ap).astype(np.int64)
    n_span = int(math.ceil(p["width_ms"] / t_ap)) + 2
    tau = p["baseline_delay_us"][b]
    phase = np.exp(1j * (2.0 * np.pi * (f * tau) + p["phase_rad"][b]))
    rate = p.get("rate", 0.0)
    for i in range(n_span):
        k = k_first + i
        lo = np.maximum(k * t_ap, t_start)
        hi = np.minimum((k + 1) * t_ap, t_end)
        frac = np.clip(hi - lo, 0.0, None) / t_ap
        ok = (frac > 0) & (k >= 0) & (k < K)
        if not ok.any():
            continue
        val = amp * frac * phase
        if rate != 0.0:
            # delay drifting at `rate` (s/s): extra fringe phase of the IF sky
            # frequency f0^n (MHz) at the frame centre (ms) -> cycles * 1e3
            tmid = (k + 0.5) * t_ap
            f0 = np.asarray(lay["if_freq_mhz"], dtype=np.float64)[:, None]
            val = val * np.exp(2j * np.pi * 1e3 * rate * f0 * tmid)
        nn, jj = np.nonzero(ok)
        Vb[nn, jj, k[nn, jj]] += val[nn, jj].astype(np.complex64)


def generate(wl: dict, baselines=None):
    """Draw the cross spectra of workload `wl`.

    Returns (V, truth): V is complex64 [B][N][J][K] (only the requested
    baselines, in the requested order, when `baselines` is given) and
    truth is a dict with the injected pulses and RFI masks.
    """
    lay, sig = wl["layout"], wl["signal"]
    N, J, K = lay["n_if"], lay["n_chan"], lay["n_frames"]
    B = lay["n_baselines"]
    rngs = _rngs(wl)
    rng_pulse, rng_station = rngs[0], rngs[1]
    pulses = _draw_pulses(wl, rng_pulse, rng_station)
    S = lay["n_stations"]
    n_flag = int(round(sig["rfi_frac"] * N * J))
    station_masks = []
    for s in range(S):
        m = np.zeros(N * J, dtype=bool)
        if n_flag:
            m[rng_station.choice(N * J, size=n_flag, replace=False)] = True
        station_masks.append(m)
    bl = list(range(B)) if baselines is None else list(baselines)
    V = np.zeros((len(bl), N, J, K), dtype=np.complex64)
    for out_i, b in enumerate(bl):
        rng = rngs[2 + b]
        Vb = V[out_i]
        if sig["noise"]:
            g = rng.standard_normal((2, N, J, K), dtype=np.float32)
            g *= np.float32(math.sqrt(0.5))
            Vb.real[...] = g[0]
            Vb.imag[...] = g[1]
            del g
        a, c = lay["stations"][b]
        flag = station_masks[a] | station_masks[c]
        if sig["rfi_amp"] and flag.any():
            idx = np.nonzero(flag)[0]
            ph = rng.uniform(0.0, 2.0 * np.pi, (idx.size, K))
            tone = (sig["rfi_amp"] * np.exp(1j * ph)).astype(np.complex64)
            flat = Vb.reshape(N * J, K)
            flat[idx] += tone
        for p in pulses:
            _add_pulse(Vb, lay, p, b)
    truth = dict(pulses=pulses, station_masks=station_masks)
    return V, truth
