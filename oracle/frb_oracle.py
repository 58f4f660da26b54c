"""FP64 CPU oracle of the cross-spectrum FRB search -- TEST INFRASTRUCTURE.

This is the plain, slow, obviously-correct reference that the HIP library is
checked against.  Only the test-suite, the package smoke check and the CPU
baseline leg of the benchmark may import or run it; the search product never
does.  It shares no code, table or constant generator with the HIP library:
everything below is written out from Liu et al. 2018 (arXiv:1801.02391),
in float64, with numpy matrix products as the only library primitive.

Steps and the passages they follow (section / equation of the paper):
  O1  reference frequency of dedispersion ......... Sec. 2.2, text after Eq. 1
  O2  dispersion offset and AP offset ............. Sec. 2.2, Eqs. 1 and 2
  O3  segment lists, half-overlapped .............. Sec. 2.2 Eq. 3; Sec. 2.4.1
  O4  channel-delay / initial-phase rotation ...... Sec. 2.3, Eq. 5
  O5  segment sum with optional rate rotation ..... Eq. 3; rate term of Eq. 4
  O6  single-band delay (SBD) transform ........... Eq. 5 (f_j SBD term), Sec. 5.1
  O7  multiband delay (MBD) transform ............. Eq. 5 (f0^n MBD term), Sec. 5.1
  O8  peak of |G| over the grid ................... Sec. 2.3 (fringe fitting maximises G)
  O9  normalised power ............................ Eq. 6
  O10 threshold ................................... Sec. 2.4.1 (threshold 3)
  O11 per-baseline multi-window filter, steps b-d . Sec. 2.4.1
  O12 best DM bin per detection ................... Sec. 5.3 (coarse search)
  O13 cross-baseline matching ..................... Sec. 2.4.1 (cross matching)
  PS  power-summation scheme ...................... Sec. 2.4.2
  CA  initial-phase / channel-delay extraction ..... Appendix A
  R1-R5 refinement of a coarse peak: |G| at continuous SBD, MBD and rate
      (Eq. 5 with the Eq. 4 rate term) and at a continuous DM (Eq. 1 without
      the rounding of Eq. 2, frames interpolated), with its gradient
  H1  DM resolution ............................... Eq. 10
  H2  noise level ................................. Eq. 7

Readings where the paper is silent (each also listed in the design notes):
  * SBD multiplies f_j and MBD multiplies (f0^n - f_ref,fit), as in Eq. 5
    (the prose after Eq. 4 swaps the two names).
  * f_ref,dm is the highest channel sky frequency, so every offset is >= 0.
  * segments are kept only where every channel is inside the data: one
    global maximum offset over all DM trials; hop h = max(1, floor(l/2)).
  * the rate term uses the IF sky frequency f0^n and the dedispersed frame
    index relative to the window centre, u - (l-1)/2; rate grid
    rho_r = (r - floor(R/2)) * step, default step 1/(2 f_max l_max t_ap).
  * SBD grid: PJ = sbd_pad * J points, tau_s = (s - PJ/2) / (PJ * chan_bw).
  * MBD grid: M points over one ambiguity T = 1/g (g = gcd of the IF offsets
    from the first IF, in whole kHz), tau_m = (m - M/2) * T / M.
  * power is |G| (the amplitude); ties in the peak take the lowest packed
    index (r * PJ + s) * M + m.
  * Eq. 6 statistics are per (baseline, DM trial, window) over all of that
    window's segments, population standard deviation; threshold strict ">".
  * grouping: insertion orders, the overlap rule on closed frame intervals
    [k0, k0 + l - 1], the circular MBD mean and the open +-T/4 interval as in
    group_windows(); best member by normalised power.
  * refinement (not in the paper, which grids every parameter): Eq. 2's
    rounding is relaxed by Keys' cubic interpolation (a = -1/2) of each
    channel's frames at the unrounded Eq. 1 shift plus a continuous arrival
    offset t; samples outside the data are zero; the ascent runs in grid-cell
    units with a diagonal Newton step (grid cells, DM decorrelated from t).
Units: MHz, ms, microseconds (so MHz * us = cycles), pc cm^-3; rate in s/s.
"""
from __future__ import annotations

import math
import numpy as np

TWO_PI = 2.0 * np.pi
K_DM_DEFAULT = 4.149e6  # ms MHz^2 per pc cm^-3


# ----------------------------------------------------------------------------
# Grid construction (O1-O4, rate grid, SBD / MBD grids)
# ----------------------------------------------------------------------------
def channel_sky_freq(f0, n_chan, chan_bw):
    """Sky frequency f0^n + f_j of frequency point j in IF n, f_j = j * chan_bw
    (Sec. 2.2: f0^n is the IF sky frequency, f_j the baseband frequency)."""
    f0 = np.asarray(f0, dtype=np.float64)
    return f0[:, None] + np.arange(n_chan, dtype=np.float64)[None, :] * chan_bw


def ref_freq_dm(f0, n_chan, chan_bw):
    """O1: f_ref,dm is the highest frequency of the band (Sec. 2.2)."""
    return float(channel_sky_freq(f0, n_chan, chan_bw).max())


def dispersion_offset_ms(dm, freq, f_ref, k_dm=K_DM_DEFAULT):
    """O2, Eq. 1: delay (ms) of sky frequency `freq` (MHz) behind f_ref."""
    return k_dm * dm * (1.0 / (freq * freq) - 1.0 / (f_ref * f_ref))


def ap_offsets(dm_grid, f0, n_chan, chan_bw, t_ap, k_dm=K_DM_DEFAULT):
    """O2, Eq. 2: dk = floor(0.5 + dt / t_ap) for every (DM trial, IF, point)."""
    f = channel_sky_freq(f0, n_chan, chan_bw)
    fr = ref_freq_dm(f0, n_chan, chan_bw)
    out = np.empty((len(dm_grid), f.shape[0], f.shape[1]), dtype=np.int64)
    for d, dm in enumerate(dm_grid):
        dt = dispersion_offset_ms(float(dm), f, fr, k_dm)
        out[d] = np.floor(0.5 + dt / t_ap).astype(np.int64)
    return out


def dm_trials(dm_lo, dm_step, n_dm):
    """DM_d = DM_lo + d * step (Sec. 5.3 coarse DM bins)."""
    return np.array([dm_lo + d * dm_step for d in range(n_dm)], dtype=np.float64)


def segment_layout(n_frames, dk_max, windows):
    """O3: for window l the hop is h = max(1, floor(l/2)) (half overlap,
    Sec. 2.4.1); segment q starts at k0 = q h and is kept iff every channel's
    frames k0 + dk .. k0 + dk + l - 1 lie inside the data (Eq. 3)."""
    out = []
    for l in windows:
        h = max(1, l // 2)
        span = n_frames - dk_max - l
        q = span // h + 1 if span >= 0 else 0
        out.append((int(l), int(h), int(q)))
    return out


def calibration_phasor(n_chan, chan_bw, tau0_us, phi0_rad):
    """O4, Eq. 5 terms: exp(-i [2 pi (f_j - f_bw/2) tau0^n + phi0^n]),
    f_bw = J * chan_bw.  tau0_us, phi0_rad: [N]."""
    fj = np.arange(n_chan, dtype=np.float64) * chan_bw
    fbw = n_chan * chan_bw
    tau0 = np.asarray(tau0_us, dtype=np.float64)[:, None]
    phi0 = np.asarray(phi0_rad, dtype=np.float64)[:, None]
    return np.exp(-1j * (TWO_PI * (fj[None, :] - fbw / 2.0) * tau0 + phi0))


def default_rate_step(f0, n_chan, chan_bw, t_ap, windows):
    """Rate-grid convention (the paper fixes none): half the fringe-rate
    resolution of the longest window at the top frequency, as a delay rate
    (s/s): 1 / (2 f_max l_max t_ap) with f in Hz and t_ap in s."""
    fmax_hz = ref_freq_dm(f0, n_chan, chan_bw) * 1e6
    return 1.0 / (2.0 * fmax_hz * max(windows) * t_ap * 1e-3)


def rate_grid(n_rate, rate_step):
    """rho_r = (r - floor(R/2)) * step; R = 1 gives rho = 0 (Sec. 2.3, the
    modification that drops the rate term)."""
    return np.array([(r - n_rate // 2) * rate_step for r in range(n_rate)], dtype=np.float64)


def rate_phasor(rates, f0, l, t_ap):
    """Rate term of Eq. 4 for a window of l frames:
    exp(-i 2 pi f0^n rho t_ap (u - (l-1)/2)), u = 0..l-1 -> [R][N][l].
    f0 in MHz and t_ap in ms, so the product carries a factor 1e3."""
    f0 = np.asarray(f0, dtype=np.float64)
    u = np.arange(l, dtype=np.float64) - (l - 1) / 2.0
    ph = TWO_PI * 1e3 * np.asarray(rates)[:, None, None] * f0[None, :, None] * t_ap * u[None, None, :]
    return np.exp(-1j * ph)


def _gcd_khz(offsets_mhz):
    g = 0
    for x in offsets_mhz:
        k = int(round(abs(x) * 1000.0))
        if abs(k - abs(x) * 1000.0) > 1e-6:
            raise ValueError("IF offsets are not whole kHz")
        g = math.gcd(g, k)
    return g


def mbd_grid(f0, n_mbd, mbd_step_us=0.0, f_ref_fit_mhz=float("nan"), chan_bw=None, n_chan=None):
    """MBD grid: tau_m = (m - M/2) * step.  Default step = T / M with the MBD
    ambiguity T = 1/g, g the gcd (whole kHz) of f0^n - f0^0 (Sec. 2.4.1 step c
    names the ambiguity; Sec. 5.1 grids MBD for a 2-D FFT).  With one IF
    (no offsets) g = J * chan_bw.  Returns (tau_m [M] us, T us, f_ref_fit)."""
    f0 = np.asarray(f0, dtype=np.float64)
    g_khz = _gcd_khz(f0 - f0[0])
    if g_khz == 0:
        g_mhz = n_chan * chan_bw
    else:
        g_mhz = g_khz / 1000.0
    t_amb = 1.0 / g_mhz
    step = mbd_step_us if mbd_step_us > 0 else t_amb / n_mbd
    f_ref = f0[0] if math.isnan(f_ref_fit_mhz) else f_ref_fit_mhz
    tau = (np.arange(n_mbd, dtype=np.float64) - n_mbd / 2.0) * step
    return tau, t_amb, float(f_ref)


def sbd_grid(n_chan, chan_bw, sbd_pad):
    """SBD grid of the zero-padded transform: tau_s = (s - PJ/2)/(PJ chan_bw)."""
    pj = sbd_pad * n_chan
    return (np.arange(pj, dtype=np.float64) - pj / 2.0) / (pj * chan_bw)


def build_grids(layout, search):
    """Everything the search needs from (layout, search parameters)."""
    f0 = np.asarray(layout["if_freq_mhz"], dtype=np.float64)
    J, df, t_ap, K = layout["n_chan"], layout["chan_bw_mhz"], layout["t_ap_ms"], layout["n_frames"]
    dms = dm_trials(search["dm_lo"], search["dm_step"], search["n_dm"])
    k_dm = search.get("k_dm", K_DM_DEFAULT) or K_DM_DEFAULT
    dk = ap_offsets(dms, f0, J, df, t_ap, k_dm)
    dk_max = int(dk.max())
    windows = list(search["windows"])
    segs = segment_layout(K, dk_max, windows)
    rstep = search.get("rate_step", 0.0)
    if search["n_rate"] > 1 and not rstep:
        rstep = default_rate_step(f0, J, df, t_ap, windows)
    rates = rate_grid(search["n_rate"], rstep)
    tau_s = sbd_grid(J, df, search["sbd_pad"])
    tau_m, t_amb, f_ref = mbd_grid(f0, search["n_mbd"], search.get("mbd_step_us", 0.0),
                                   search.get("f_ref_fit_mhz", float("nan")), df, J)
    fj = np.arange(J, dtype=np.float64) * df
    # Eq. 5 phase matrices, evaluated from their definitions in float64.
    e_sbd = np.exp(-1j * TWO_PI * fj[:, None] * tau_s[None, :])            # [J][PJ]
    e_mbd = np.exp(-1j * TWO_PI * (f0 - f_ref)[:, None] * tau_m[None, :])   # [N][M]
    return dict(f0=f0, dms=dms, dk=dk, dk_max=dk_max, windows=windows, segs=segs,
                rates=rates, rate_step=rstep, tau_s=tau_s, tau_m=tau_m, t_amb=t_amb,
                f_ref_fit=f_ref, e_sbd=e_sbd, e_mbd=e_mbd, t_ap=t_ap)


# ----------------------------------------------------------------------------
# Per-segment fringe search (O5-O8)
# ----------------------------------------------------------------------------
def segment_sums(Vb, dk_d, k0s, l, rph, cal):
    """O5 (Eq. 3 with the Eq. 4 rate term and the Eq. 5 calibration):
    Y[q, r, n, j] = cal[n,j] * sum_u rph[r,n,u] * V[n, j, k0_q + dk[n,j] + u],
    with the j = 0 point excluded from the fit (Sec. 2.3) by zeroing it."""
    N, J, _ = Vb.shape
    n_idx = np.arange(N)[:, None]
    j_idx = np.arange(J)[None, :]
    Q = len(k0s)
    R = rph.shape[0]
    Y = np.zeros((Q, R, N, J), dtype=np.complex128)
    for u in range(l):
        frames = np.asarray(k0s)[:, None, None] + dk_d[None, :, :] + u      # [Q][N][J]
        v = Vb[n_idx[None], j_idx[None], frames].astype(np.complex128)      # [Q][N][J]
        Y += rph[None, :, :, u, None] * v[:, None, :, :]
    Y *= cal[None, None, :, :]
    Y[..., 0] = 0.0
    return Y


def fringe_matrix(Y, e_sbd, e_mbd):
    """O6-O7: G[q, r, s, m] = sum_n e_mbd[n,m] sum_j e_sbd[j,s] Y[q,r,n,j]
    -- the double sum of Eq. 5 with its phase split into the SBD and MBD
    terms, evaluated as two matrix products."""
    X = Y @ e_sbd                                  # [Q][R][N][PJ]
    return np.swapaxes(X, -1, -2) @ e_mbd          # [Q][R][PJ][M]


def peak(G):
    """O8: P = max |G| over (r, s, m); index = lowest flat (r, s, m) index
    among the maxima (numpy argmax returns the first); also the second-largest
    cell value, for the peak-margin rule of the parity checks."""
    Q = G.shape[0]
    A = np.abs(G).reshape(Q, -1)
    idx = np.argmax(A, axis=1)
    best = A[np.arange(Q), idx]
    if A.shape[1] > 1:
        second = np.partition(A, -2, axis=1)[:, -2]
    else:
        second = np.zeros(Q)
    return best, idx.astype(np.int64), second


def search_row(Vb, grids, cal, d, wi, q_list=None, chunk=16):
    """Fringe search of every (or the listed) segment of one (DM trial d,
    window index wi) on one baseline.  Returns (P, idx, second) per segment."""
    l, h, Q = grids["segs"][wi]
    qs = np.arange(Q) if q_list is None else np.asarray(q_list, dtype=np.int64)
    rph = rate_phasor(grids["rates"], grids["f0"], l, grids["t_ap"])
    P = np.zeros(len(qs))
    I = np.zeros(len(qs), dtype=np.int64)
    S2 = np.zeros(len(qs))
    for a in range(0, len(qs), chunk):
        qq = qs[a:a + chunk]
        Y = segment_sums(Vb, grids["dk"][d], qq * h, l, rph, cal)
        G = fringe_matrix(Y, grids["e_sbd"], grids["e_mbd"])
        P[a:a + chunk], I[a:a + chunk], S2[a:a + chunk] = peak(G)
    return P, I, S2


def unpack_index(idx, n_sbd, n_mbd):
    """packed = (r * PJ + s) * M + m -> (r, s, m)."""
    m = idx % n_mbd
    s = (idx // n_mbd) % n_sbd
    r = idx // (n_mbd * n_sbd)
    return r, s, m


# ----------------------------------------------------------------------------
# Normalisation and threshold (O9, O10)
# ----------------------------------------------------------------------------
def normalise(P):
    """O9, Eq. 6: (|G| - mean) / std over the row, population std.  A segment
    whose power is not finite (its data hold a NaN or infinity) takes no part
    in the statistics and has no normalised power (NaN), so it never crosses.
    Returns (P_norm or None when std == 0, mean, std)."""
    P = np.asarray(P, dtype=np.float64)
    ok = np.isfinite(P)
    if not ok.any():
        return None, 0.0, 0.0
    mu = P[ok].mean()
    sd = math.sqrt(((P[ok] - mu) ** 2).mean())
    if sd == 0.0:
        return None, mu, sd
    return np.where(ok, (np.where(ok, P, mu) - mu) / sd, np.nan), mu, sd


def crossings(P_norm, threshold):
    """O10: segments whose normalised power is strictly above the threshold
    (a NaN normalised power is not)."""
    if P_norm is None:
        return np.zeros(0, dtype=np.int64)
    return np.nonzero(np.nan_to_num(P_norm, nan=-np.inf) > threshold)[0]


# ----------------------------------------------------------------------------
# Grouping (O11-O13, power summation)
# ----------------------------------------------------------------------------
def _overlap(a0, a1, b0, b1):
    return a0 <= b1 and b0 <= a1


def _insert(groups, item, lo, hi):
    """Join the lowest-numbered group holding a member whose closed interval
    overlaps [lo, hi]; else open a new group (Sec. 2.4.1 step b)."""
    for g in groups:
        for (_, glo, ghi) in g:
            if _overlap(lo, hi, glo, ghi):
                g.append((item, lo, hi))
                return
    groups.append([(item, lo, hi)])


def circular_mean(values, period):
    """Mean of values defined modulo `period` (Sec. 2.4.1 step c: the MBD
    ambiguity must be taken into account when averaging)."""
    z = np.exp(1j * TWO_PI * np.asarray(values, dtype=np.float64) / period).sum()
    return period * math.atan2(z.imag, z.real) / TWO_PI


def wrapped_diff(a, b, period):
    """a - b wrapped into [-period/2, period/2)."""
    return ((a - b + period / 2.0) % period) - period / 2.0


def group_windows(cands, t_amb, n_win_min, use_mbd=True):
    """O11, Sec. 2.4.1 steps b-d for one baseline and DM trial.

    cands: list of dicts with keys l, k0, p_norm, mbd_us (any extra keys are
    carried along).  Insertion order: window descending, then k0 ascending.
    Step c keeps members with wrapped |MBD - circular mean| < T/4 (skipped
    when use_mbd is False, the power-summation scheme, Sec. 2.4.2).
    Step d: N_win = number of distinct windows among the survivors; a single
    pulse needs N_win >= n_win_min and is represented by the survivor with
    the highest normalised power (earliest inserted on ties).
    Returns a list of (detection dict with 'n_windows', members)."""
    order = sorted(range(len(cands)), key=lambda i: (-cands[i]["l"], cands[i]["k0"], i))
    groups = []
    for i in order:
        c = cands[i]
        _insert(groups, i, c["k0"], c["k0"] + c["l"] - 1)
    out = []
    for g in groups:
        members = [i for (i, _, _) in g]
        if use_mbd:
            mbar = circular_mean([cands[i]["mbd_us"] for i in members], t_amb)
            surv = [i for i in members
                    if abs(wrapped_diff(cands[i]["mbd_us"], mbar, t_amb)) < t_amb / 4.0]
        else:
            surv = members
        n_win = len({cands[i]["l"] for i in surv})
        if n_win >= n_win_min and surv:
            best = surv[0]
            for i in surv[1:]:
                if cands[i]["p_norm"] > cands[best]["p_norm"]:
                    best = i
            det = dict(cands[best])
            det["n_windows"] = n_win
            out.append((det, members))
    return out


def merge_dm(dets):
    """O12, Sec. 5.3: a pulse found in several DM bins keeps the bin with the
    highest power.  dets: detections of one baseline over all DM trials (keys
    d, k0, l, p_norm).  Insertion order DM ascending then k0; the overlap rule
    of step b; the best member by normalised power survives."""
    order = sorted(range(len(dets)), key=lambda i: (dets[i]["d"], dets[i]["k0"], i))
    groups = []
    for i in order:
        c = dets[i]
        _insert(groups, i, c["k0"], c["k0"] + c["l"] - 1)
    out = []
    for g in groups:
        members = [i for (i, _, _) in g]
        best = members[0]
        for i in members[1:]:
            if dets[i]["p_norm"] > dets[best]["p_norm"]:
                best = i
        out.append(dets[best])
    return out


def cross_match(dets, n_bl_min):
    """O13, Sec. 2.4.1 cross matching: insert the single pulses of every
    baseline (baseline ascending, then k0) into matching groups with the
    overlap rule; count distinct baselines per group.  Returns (groups,
    assignment) where each group is dict(n_baselines, k_start, k_end, best,
    members) and assignment[i] is the group of detection i.  Groups with
    n_baselines >= n_bl_min are the reported ones."""
    order = sorted(range(len(dets)), key=lambda i: (dets[i]["b"], dets[i]["k0"], i))
    groups = []
    for i in order:
        c = dets[i]
        _insert(groups, i, c["k0"], c["k0"] + c["l"] - 1)
    res = []
    assign = [-1] * len(dets)
    for gi, g in enumerate(groups):
        members = [i for (i, _, _) in g]
        for i in members:
            assign[i] = gi
        best = members[0]
        for i in members[1:]:
            if dets[i]["p_norm"] > dets[best]["p_norm"]:
                best = i
        res.append(dict(n_baselines=len({dets[i]["b"] for i in members}),
                        k_start=min(lo for (_, lo, _) in g), k_end=max(hi for (_, _, hi) in g),
                        best=best, members=members, reported=None))
    for r in res:
        r["reported"] = r["n_baselines"] >= n_bl_min
    return res, assign


# ----------------------------------------------------------------------------
# Full search
# ----------------------------------------------------------------------------
def search(V, layout, search_params, tau0_us=None, phi0_rad=None, baselines=None,
           dm_indices=None, chunk=16):
    """Run O1-O13 on cross spectra V [B][N][J][K] (any complex dtype; the
    stored values are promoted to complex128).  Returns a dict with the grids,
    the power cube (per baseline, DM trial and window: P, packed index and the
    second-best cell), the Eq. 6 statistics, the crossings, the per-baseline
    detections and the cross-baseline groups."""
    g = build_grids(layout, search_params)
    B, N, J, K = V.shape
    bls = list(range(B)) if baselines is None else list(baselines)
    dis = list(range(len(g["dms"]))) if dm_indices is None else list(dm_indices)
    PJ, M = len(g["tau_s"]), len(g["tau_m"])
    thr = search_params["threshold"]
    cube = {}
    stats = {}
    cross = []
    for b in bls:
        t0 = np.zeros(N) if tau0_us is None else np.asarray(tau0_us)[b]
        p0 = np.zeros(N) if phi0_rad is None else np.asarray(phi0_rad)[b]
        cal = calibration_phasor(J, layout["chan_bw_mhz"], t0, p0)
        for d in dis:
            for wi, (l, h, Q) in enumerate(g["segs"]):
                P, I, S2 = search_row(V[b], g, cal, d, wi, chunk=chunk)
                cube[(b, d, wi)] = (P, I, S2)
                pn, mu, sd = normalise(P)
                stats[(b, d, wi)] = (mu, sd)
                for q in crossings(pn, thr):
                    r, s, m = unpack_index(int(I[q]), PJ, M)
                    cross.append(dict(b=b, d=d, wi=wi, l=l, q=int(q), k0=int(q) * h,
                                      power=float(P[q]), p_norm=float(pn[q]), idx=int(I[q]),
                                      r=int(r), s=int(s), m=int(m),
                                      sbd_us=float(g["tau_s"][s]), mbd_us=float(g["tau_m"][m]),
                                      rate=float(g["rates"][r])))
    dets, groups, assign = detect(cross, g["t_amb"], search_params["n_win_min"],
                                  search_params["n_bl_min"])
    return dict(grids=g, cube=cube, stats=stats, crossings=cross, detections=dets,
                groups=groups, assign=assign)


def detect(cross, t_amb, n_win_min, n_bl_min):
    """O11-O13 over a list of crossings (dicts as produced by search())."""
    by_bd = {}
    for c in cross:
        by_bd.setdefault((c["b"], c["d"]), []).append(c)
    per_b = {}
    for (b, d) in sorted(by_bd):
        for det, _ in group_windows(by_bd[(b, d)], t_amb, n_win_min):
            per_b.setdefault(b, []).append(det)
    dets = []
    for b in sorted(per_b):
        dets.extend(merge_dm(per_b[b]))
    groups, assign = cross_match(dets, n_bl_min)
    return dets, groups, assign


def power_sum_detect(cube_rows, segs, t_amb, threshold, n_win_min):
    """PS, Sec. 2.4.2 for one DM trial: sum |G| of corresponding segments over
    the given baselines per window, normalise (Eq. 6), threshold, then steps b
    and d of the multi-window filter (step c skipped: MBD is meaningless for
    the combined baseline).  cube_rows[wi] = list of per-baseline P arrays."""
    cands = []
    for wi, (l, h, Q) in enumerate(segs):
        tot = np.sum(np.asarray(cube_rows[wi], dtype=np.float64), axis=0)
        pn, _, _ = normalise(tot)
        for q in crossings(pn, threshold):
            cands.append(dict(wi=wi, l=l, q=int(q), k0=int(q) * h, p_norm=float(pn[q]),
                              power=float(tot[q]), mbd_us=0.0))
    return [det for det, _ in group_windows(cands, t_amb, n_win_min, use_mbd=False)]


def power_sum_search(cube_P, segs, t_amb, threshold, n_win_min, baselines):
    """PS over DM trials: cube_P[b][d][seg] (window-major segments).  For
    every DM trial, the Sec. 2.4.2 steps on the summed power of the listed
    baselines; then the best DM bin per pulse (Sec. 5.3).  Returns the
    detections (dicts with d, wi, l, q, k0, power, p_norm, n_windows)."""
    cube_P = np.asarray(cube_P, dtype=np.float64)
    off = np.cumsum([0] + [q for (_, _, q) in segs])
    dets = []
    for d in range(cube_P.shape[1]):
        rows = [[cube_P[b, d, off[wi]:off[wi + 1]] for b in baselines] for wi in range(len(segs))]
        for det in power_sum_detect(rows, segs, t_amb, threshold, n_win_min):
            det["d"] = d
            dets.append(det)
    return merge_dm(dets)


def calibrate(Y, f0, chan_bw, e_sbd, e_mbd, tau_s, tau_m, f_ref, n_fine=64):
    """CA, Appendix A on one calibrator segment Y[N][J] (the window sum,
    j = 0 unused), starting from zero calibration (step a):
      * the (SBD, MBD) cell maximising |G| of Eq. 5;
      * channel delay of IF n: the delay tau maximising
        |sum_{j>=1} Y(n,j) exp(-2 pi i f_j SBD) exp(-2 pi i (f_j - f_bw/2) tau)|
        (the fit of Y exp(-2 pi i f_j SBD) of step c), on a grid n_fine times
        finer than 1/(J chan_bw) over +-1/(2 chan_bw), refined by
        golden-section search;
      * initial phase of IF n: the angle of
        sum_{j>=1} Y(n,j) exp(-2 pi i [f_j SBD + (f0^n - f_ref) MBD
                                       + (f_j - f_bw/2) tau0^n]),
        i.e. step c's formula taken after the channel delay is removed (the
        reading that keeps the pair consistent with the Eq. 5 rotation; it
        equals the printed order when channel delays are small).
    Returns (tau0_us[N], phi0_rad[N], sbd_us, mbd_us)."""
    Y = np.array(Y, dtype=np.complex128)
    Y[:, 0] = 0.0
    N, J = Y.shape
    G = np.abs((Y @ e_sbd).T @ e_mbd)                       # [PJ][M]
    s, m = np.unravel_index(int(np.argmax(G)), G.shape)
    sbd, mbd = float(tau_s[s]), float(tau_m[m])
    fj = np.arange(J, dtype=np.float64) * chan_bw
    fbw = J * chan_bw
    f0 = np.asarray(f0, dtype=np.float64)
    Z = Y * np.exp(-2j * np.pi * fj * sbd)[None, :]
    grid = np.linspace(-0.5 / chan_bw, 0.5 / chan_bw, n_fine * J + 1)
    tau0 = np.zeros(N)

    def amp(n, t):
        return abs((Z[n] * np.exp(-2j * np.pi * (fj - fbw / 2) * t)).sum())

    for n in range(N):
        vals = np.abs(Z[n][None, :] @ np.exp(-2j * np.pi * (fj[:, None] - fbw / 2) * grid[None, :]))[0]
        i = int(np.argmax(vals))
        a, b = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
        gr = (math.sqrt(5) - 1) / 2
        c, d = b - gr * (b - a), a + gr * (b - a)
        for _ in range(80):
            if amp(n, c) > amp(n, d):
                b = d
            else:
                a = c
            c, d = b - gr * (b - a), a + gr * (b - a)
        tau0[n] = 0.5 * (a + b)
    rot = np.exp(-2j * np.pi * (fj[None, :] * sbd + (f0 - f_ref)[:, None] * mbd
                                + (fj[None, :] - fbw / 2) * tau0[:, None]))
    phi0 = np.angle((Y * rot).sum(axis=1))
    return tau0, phi0, sbd, mbd


# ----------------------------------------------------------------------------
# Helper closed forms (not on the search path)
# ----------------------------------------------------------------------------
def dm_resolution(t_win_min_ms, f_low_mhz, f_high_mhz):
    """H1, Eq. 10: DM_res = 2.41e-7 t_win,min / (f_low^-2 - f_high^-2)."""
    return 2.41e-7 * t_win_min_ms / (1.0 / f_low_mhz ** 2 - 1.0 / f_high_mhz ** 2)


def noise_level_jy(sefd1, sefd2, bandwidth_hz, t_s):
    """H2, Eq. 7: S_noise = sqrt(SEFD1 SEFD2 / (2 B T))."""
    return math.sqrt(sefd1 * sefd2 / (2.0 * bandwidth_hz * t_s))


# ----------------------------------------------------------------------------
# Refinement of a coarse peak (R1-R4): |G| as a function of continuous
# (SBD, MBD, rate, DM, arrival offset) and its analytic gradient.
# ----------------------------------------------------------------------------
REFINE_PARAMS = ("sbd_us", "mbd_us", "rate", "dm", "t_frames")


def keys_kernel(s):
    """R1: Keys' cubic convolution kernel with a = -1/2 (Catmull-Rom):
    phi(s) = 3/2 |s|^3 - 5/2 |s|^2 + 1 for |s| <= 1,
    -1/2 |s|^3 + 5/2 |s|^2 - 4 |s| + 2 for 1 < |s| < 2, 0 beyond.
    Interpolating, continuously differentiable, exact for quadratics.  It
    relaxes the rounding of Eq. 2 so that the fringe amplitude becomes a
    differentiable function of DM."""
    a = np.abs(np.asarray(s, dtype=np.float64))
    inner = 1.5 * a ** 3 - 2.5 * a ** 2 + 1.0
    outer = -0.5 * a ** 3 + 2.5 * a ** 2 - 4.0 * a + 2.0
    return np.where(a <= 1.0, inner, np.where(a < 2.0, outer, 0.0))


def keys_kernel_deriv(s):
    """d phi / d s of keys_kernel."""
    s = np.asarray(s, dtype=np.float64)
    a = np.abs(s)
    inner = 4.5 * a ** 2 - 5.0 * a
    outer = -1.5 * a ** 2 + 5.0 * a - 4.0
    return np.sign(s) * np.where(a <= 1.0, inner, np.where(a < 2.0, outer, 0.0))


def keys_kernel_deriv2(s):
    """d^2 phi / d s^2 of keys_kernel (piecewise linear, even)."""
    a = np.abs(np.asarray(s, dtype=np.float64))
    return np.where(a <= 1.0, 9.0 * a - 5.0, np.where(a < 2.0, -3.0 * a + 5.0, 0.0))


def relaxed_offsets(dm, f0, n_chan, chan_bw, t_ap, k_dm=K_DM_DEFAULT):
    """R2: the dispersion shift of Eq. 1 in frames, dt / t_ap, without the
    rounding of Eq. 2, and its derivative with respect to DM ([N][J] each)."""
    f = channel_sky_freq(f0, n_chan, chan_bw)
    fr = ref_freq_dm(f0, n_chan, chan_bw)
    dxd = k_dm * (1.0 / (f * f) - 1.0 / (fr * fr)) / t_ap
    return dm * dxd, dxd


def interpolated_frames(Vb, pos):
    """R1 applied to every channel: the value at the continuous frame position
    pos[n, j] of channel (n, j) of Vb [N][J][K], as sum_i V[n, j, i] phi(pos - i)
    over the four samples i = floor(pos) - 1 .. floor(pos) + 2 (samples outside
    the data count as zero), and its first and second derivatives with
    respect to pos."""
    N, J, K = Vb.shape
    base = np.floor(pos).astype(np.int64)
    nn, jj = np.meshgrid(np.arange(N), np.arange(J), indexing="ij")
    val = np.zeros((N, J), dtype=np.complex128)
    der = np.zeros((N, J), dtype=np.complex128)
    der2 = np.zeros((N, J), dtype=np.complex128)
    for m in range(-1, 3):
        i = base + m
        ok = (i >= 0) & (i < K)
        v = np.where(ok, Vb[nn, jj, np.clip(i, 0, K - 1)], 0.0)
        val += v * keys_kernel(pos - i)
        der += v * keys_kernel_deriv(pos - i)
        der2 += v * keys_kernel_deriv2(pos - i)
    return val, der, der2


def relaxed_fringe(Vb, layout, search, cal, k0, l, theta, k_dm=K_DM_DEFAULT):
    """R3: G(theta) for one segment of one baseline, theta = (SBD us, MBD us,
    rate, DM, t frames):
        G = sum_{n, j >= 1} cal[n,j] exp(-i 2 pi (f_j tau_s + (f0^n - f0^0) tau_m))
              sum_u exp(-i 2 pi f0^n rho t_ap (u - (l-1)/2)) V~[n, j, k0 + t + x_nj(DM) + u]
    -- Eq. 5 with the rate term of Eq. 4 (as in O5-O7) at continuous delays
    and rate, and the dedispersed frame of Eq. 3 taken at the unrounded Eq. 1
    shift plus an arrival offset t, interpolated by R1.  Returns G, the five
    partial derivatives dG/dtheta_i and the second derivatives
    d2G[i] = d^2 G / d theta_i^2 (i = 0..4) with d2G[5] = d^2 G / d DM d t
    (complex)."""
    tau_s, tau_m, rho, dm, t = (float(v) for v in theta)
    f0 = np.asarray(layout["if_freq_mhz"], dtype=np.float64)
    J, df, t_ap = layout["n_chan"], layout["chan_bw_mhz"], layout["t_ap_ms"]
    x, dxd = relaxed_offsets(dm, f0, J, df, t_ap, k_dm)
    fj = np.arange(J, dtype=np.float64) * df
    # phase of Eq. 5 at continuous delays; the j = 0 point is left out (Sec. 2.3)
    e = cal * np.exp(-1j * TWO_PI * (fj[None, :] * tau_s + (f0 - f0[0])[:, None] * tau_m))
    e[:, 0] = 0.0
    S0 = np.zeros(e.shape, dtype=np.complex128)   # sum_u r V~
    S1 = np.zeros(e.shape, dtype=np.complex128)   # sum_u d(r)/d(rho) V~
    S11 = np.zeros(e.shape, dtype=np.complex128)  # sum_u d2(r)/d(rho)2 V~
    S2 = np.zeros(e.shape, dtype=np.complex128)   # sum_u r dV~/dpos
    S3 = np.zeros(e.shape, dtype=np.complex128)   # sum_u r d2V~/dpos2
    for u in range(l):
        # rate phasor of Eq. 4 for frame u (f0 in MHz, t_ap in ms: factor 1e3)
        w_rate = TWO_PI * 1e3 * f0 * t_ap * (u - (l - 1) / 2.0)
        r = np.exp(-1j * rho * w_rate)[:, None]
        val, der, der2 = interpolated_frames(Vb, k0 + t + x + u)
        S0 += r * val
        S1 += (-1j * w_rate)[:, None] * r * val
        S11 += (-1j * w_rate)[:, None] ** 2 * r * val
        S2 += r * der
        S3 += r * der2
    term = e * S0
    G = term.sum()
    ws = -1j * TWO_PI * fj[None, :]
    wm = -1j * TWO_PI * (f0 - f0[0])[:, None]
    dG = np.array([
        np.sum(ws * term),
        np.sum(wm * term),
        np.sum(e * S1),
        np.sum(e * S2 * dxd),
        np.sum(e * S2),
    ])
    d2G = np.array([
        np.sum(ws * ws * term),
        np.sum(wm * wm * term),
        np.sum(e * S11),
        np.sum(e * S3 * dxd * dxd),
        np.sum(e * S3),
        np.sum(e * S3 * dxd),
    ])
    return G, dG, d2G


def relaxed_power_grad(G, dG, d2G=None):
    """R4: P = |G|, dP/dtheta_a = Re(conj(G) G_a) / P and (with d2G) the
    second derivatives
    P_ab = [Re(conj(G_a) G_b) + Re(conj(G) G_ab)] / P - P_a P_b / P
    for the five diagonal entries and (DM, t): returns (P, grad[5]) or
    (P, grad[5], H[6])."""
    P = abs(G)
    if P == 0.0:
        z = np.zeros(len(dG))
        return (0.0, z) if d2G is None else (0.0, z, np.zeros(6))
    g = np.real(np.conj(G) * dG) / P
    if d2G is None:
        return P, g
    H = np.empty(6)
    for i in range(5):
        H[i] = (abs(dG[i]) ** 2 + np.real(np.conj(G) * d2G[i])) / P - g[i] * g[i] / P
    H[5] = (np.real(np.conj(dG[3]) * dG[4]) + np.real(np.conj(G) * d2G[5])) / P - g[3] * g[4] / P
    return P, g, H


def refine_cells(layout, search):
    """Grid cell of each refined parameter: SBD and MBD grid steps, the rate
    step (0 when the grid has one rate: the rate is then held), the DM step,
    one frame for the arrival offset."""
    g = build_grids(layout, search)
    J, df = layout["n_chan"], layout["chan_bw_mhz"]
    sbd_cell = 1.0 / (search["sbd_pad"] * J * df)
    mbd_cell = g["tau_m"][1] - g["tau_m"][0] if len(g["tau_m"]) > 1 else g["t_amb"]
    rate_cell = g["rate_step"] if search["n_rate"] > 1 else 0.0
    return np.array([sbd_cell, mbd_cell, rate_cell, search["dm_step"], 1.0])


def coarse_theta(layout, search, d, r, s, m):
    """The grid point of a coarse peak as a refinement start: (tau_s[s],
    tau_m[m], rho[r], DM_d, 0)."""
    g = build_grids(layout, search)
    return np.array([g["tau_s"][s], g["tau_m"][m], g["rates"][r], g["dms"][d], 0.0])


def mean_dm_shift(layout, k_dm=K_DM_DEFAULT):
    """Mean over the fitted points (j >= 1) of d x / d DM (frames per pc cm^-3):
    the arrival offset that a DM change moves on average."""
    f0 = np.asarray(layout["if_freq_mhz"], dtype=np.float64)
    _, dxd = relaxed_offsets(1.0, f0, layout["n_chan"], layout["chan_bw_mhz"], layout["t_ap_ms"], k_dm)
    return float(dxd[:, 1:].mean())


def newton_ascent(fn, theta0, cells, xbar, steps=20, max_step=0.5):
    """R5: ascent of P(theta) from a coarse grid point.  Coordinates z in
    grid cells, theta = theta0 + cells * (A z) with A the identity except
    that a DM step moves the arrival offset by -xbar per unit DM (the time
    reference follows the mean dispersion shift, which decorrelates DM from
    t).  The proposed move of every live coordinate is -g_i / H_ii (gradient
    over curvature of P in z) where H_ii < 0, else max_step along the
    gradient, clipped to +-max_step; coordinates whose cell is 0 are held.
    A trust region keeps it monotone: each evaluation that does not lower P
    below the best so far is accepted (best point, its proposed move, radius
    doubled up to max_step) and the move is taken clipped to the radius;
    otherwise the radius is halved and the best point's move is retried,
    clipped to the new radius.  After the steps the better of the last point
    and the best one is returned.  fn(theta) returns (P, grad[5], H[6]).
    Returns (theta, P history)."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.float64)
    live = cells > 0
    a = -xbar * cells[3] / cells[4] if cells[4] > 0 else 0.0

    def move(base, dz):
        d = dz.copy()
        d[4] += a * d[3]
        return base + cells * d

    theta = theta0.copy()
    best_t, best_p, best_s = theta0.copy(), -1.0, np.zeros(5)
    radius = max_step
    hist = []
    for _ in range(steps):
        P, g, H = fn(theta)
        hist.append(P)
        if P >= best_p:
            gc = g * cells
            gz = gc.copy()
            gz[3] += a * gc[4]
            hz = np.array([H[i] * cells[i] ** 2 for i in range(5)])
            hz[3] = (H[3] * cells[3] ** 2 + 2 * a * H[5] * cells[3] * cells[4]
                     + a * a * H[4] * cells[4] ** 2)
            st = np.where(hz < 0, -gz / np.where(hz < 0, hz, -1.0), max_step * np.sign(gz))
            best_s = np.where(live, np.clip(st, -max_step, max_step), 0.0)
            best_t, best_p = theta.copy(), P
            radius = min(max_step, 2.0 * radius)
        else:
            radius *= 0.5
        theta = move(best_t, np.clip(best_s, -radius, radius))
    P = fn(theta)[0]
    if P < best_p:
        theta, P = best_t, best_p
    hist.append(P)
    return theta, np.array(hist)
