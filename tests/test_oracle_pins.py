"""Pins of the FP64 oracle against things other than itself: closed forms,
exact arithmetic, numbers the paper prints, invariants and brute force.
Each test names the passage of Liu et al. 2018 that fixes the expectation."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import frb_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _layout(f0, J, df, t_ap, K):
    return dict(if_freq_mhz=list(f0), n_chan=J, chan_bw_mhz=df, t_ap_ms=t_ap, n_frames=K,
                n_if=len(f0))


def _search(**kw):
    s = dict(dm_lo=0.0, dm_step=1.0, n_dm=1, k_dm=4.149e6, sbd_pad=4, n_mbd=64,
             mbd_step_us=0.0, f_ref_fit_mhz=float("nan"), n_rate=1, rate_step=0.0,
             windows=[2, 4], threshold=3.0, n_win_min=2, n_bl_min=1)
    s.update(kw)
    return s


def _exact_dk(dm, freq, f_ref, t_ap, k_dm):
    """Eq. 2 in exact rational arithmetic on the float64 inputs."""
    F = Fraction
    x = F(k_dm) * F(dm) * (1 / (F(freq) * F(freq)) - 1 / (F(f_ref) * F(f_ref))) / F(t_ap)
    return math.floor(F(1, 2) + x), x


# ---------------------------------------------------------------- P13 helpers
def test_paper_printed_helper_values():
    """Eq. 10 (Sec. 5.3) and Eq. 7 (Sec. 4.1): the printed example values."""
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))
    a = g["dm_resolution_pulsar"]
    v = O.dm_resolution(a["t_win_min_ms"], a["f_low_mhz"], a["f_high_mhz"])
    assert round(v, a["printed_digits"]) == a["printed"]
    b = g["dm_resolution_vgos"]
    v = O.dm_resolution(b["t_win_min_ms"], b["f_low_mhz"], b["f_high_mhz"])
    assert round(v, b["printed_digits"]) == b["printed"]
    # the printed bin count is the range over the resolution, rounded (72.03)
    assert round(b["dm_range"] / v) == b["printed_bins"]
    c = g["noise_level_sh_ur"]
    v = O.noise_level_jy(c["sefd1"], c["sefd2"], c["bandwidth_hz"], c["t_s"])
    assert round(v, c["printed_digits"]) == c["printed"]


# ---------------------------------------------------------------- P2 dk table
@pytest.mark.parametrize("name", ["single", "vgos"])
def test_dk_table_matches_exact_rational(name):
    """Eqs. 1-2: the float64 table equals floor(1/2 + x) with x exact, for
    every (DM trial, IF, point) of the two benchmark grids; no near-ties."""
    if name == "single":
        f0 = [3000.0 + 32 * n for n in range(8)]
        J, df, t_ap = 32, 1.0, 1.0
        dms = O.dm_trials(0.0, 1000.0 / 64, 64)
    else:
        f0 = [b + 32.0 * i for b in (3000.0, 5240.0, 6360.0, 10200.0) for i in range(8)]
        J, df, t_ap = 64, 0.5, 0.5
        dms = O.dm_trials(0.0, 6.25, 256)[::9]
    tab = O.ap_offsets(dms, f0, J, df, t_ap, 4.149e6)
    f = O.channel_sky_freq(f0, J, df)
    fr = O.ref_freq_dm(f0, J, df)
    near = 0
    for d, dm in enumerate(dms):
        for n in range(len(f0)):
            for j in range(0, J, 3):
                k, x = _exact_dk(float(dm), float(f[n, j]), fr, t_ap, 4.149e6)
                assert tab[d, n, j] == k
                frac = x - math.floor(x)
                near += abs(frac - Fraction(1, 2)) < Fraction(1, 10 ** 9)
    assert near == 0
    # top channel is the reference: zero offset; offsets are non-negative
    assert (tab[:, :, :] >= 0).all()
    n_top, j_top = np.unravel_index(np.argmax(f), f.shape)
    assert (tab[:, n_top, j_top] == 0).all()


def test_single_baseline_dm_grid_hits_500():
    """Config of Sec. 5.3-style coarse bins: 64 trials over 0-1000 put DM 500
    on trial 32 exactly."""
    assert O.dm_trials(0.0, 1000.0 / 64, 64)[32] == 500.0


# ---------------------------------------------------------------- P1 DM = 0
def test_dm_zero_is_plain_window_sum():
    """Eq. 3 with DM = 0: every offset is zero and a segment is the plain sum
    of l consecutive APs (checked against slicing)."""
    rng = np.random.default_rng(1)
    N, J, K = 3, 8, 40
    V = rng.standard_normal((N, J, K)) + 1j * rng.standard_normal((N, J, K))
    dk = O.ap_offsets([0.0], [2000.0, 2016.0, 2048.0], J, 1.0, 1.0)[0]
    assert (dk == 0).all()
    rph = O.rate_phasor([0.0], [2000.0, 2016.0, 2048.0], 5, 1.0)
    cal = np.ones((N, J))
    k0s = [0, 3, 17, 35]
    Y = O.segment_sums(V, dk, k0s, 5, rph, cal)
    for qi, k0 in enumerate(k0s):
        ref = V[:, :, k0:k0 + 5].sum(axis=2)
        ref[:, 0] = 0
        assert np.allclose(Y[qi, 0], ref, rtol=0, atol=1e-13)


# ------------------------------------------------------------ P3/P4 tones
def _tone(f0, J, df, K, tau_us, amp=1.0):
    f = O.channel_sky_freq(f0, J, df)
    return np.broadcast_to((amp * np.exp(2j * np.pi * f * tau_us))[:, :, None],
                           (len(f0), J, K)).copy()


def _unit_G(V, g, d, l, k0, cal=None):
    N, J, _ = V.shape
    cal = np.ones((N, J)) if cal is None else cal
    rph = O.rate_phasor(g["rates"], g["f0"], l, g["t_ap"])
    Y = O.segment_sums(V, g["dk"][d], [k0], l, rph, cal)
    return O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])[0]


def test_on_grid_tone_peaks_at_amplitude_N_ch():
    """Eq. 5 with a delay on both grids: |G| = A l N (J-1) at the unique
    cell of that delay (sign convention: exp(+i 2 pi f tau) peaks at +tau)."""
    f0 = [3000.0 + 32 * n for n in range(8)]
    J, df, K = 32, 1.0, 64
    lay = _layout(f0, J, df, 1.0, K)
    g = O.build_grids(lay, _search(n_mbd=256, windows=[4]))
    tau = 3 * (1.0 / (128 * df))            # 3 SBD cells = 64 MBD cells
    V = _tone(f0, J, df, K, tau, amp=0.5)
    G = _unit_G(V, g, 0, 4, 10)
    A = np.abs(G[0])
    s, m = np.unravel_index(np.argmax(A), A.shape)
    assert A[s, m] == pytest.approx(0.5 * 4 * 8 * 31, rel=1e-12)
    assert g["tau_s"][s] == pytest.approx(tau, abs=1e-12)
    assert O.wrapped_diff(g["tau_m"][m], tau, g["t_amb"]) == pytest.approx(0, abs=1e-12)
    flat = np.sort(A.ravel())
    assert flat[-2] < flat[-1] * (1 - 1e-3)


def test_off_grid_tone_matches_dirichlet_product():
    """Eq. 5 for a pure delay factorises into two Dirichlet sums (one over the
    points j >= 1 of an IF, one over IFs); the oracle reproduces the product at
    every (SBD, MBD) cell, including the 20 ns residual delay case."""
    f0 = [3000.0 + 32 * n for n in range(8)]
    J, df, K = 32, 1.0, 16
    lay = _layout(f0, J, df, 1.0, K)
    g = O.build_grids(lay, _search(n_mbd=256, windows=[2]))
    tau = 0.020
    V = _tone(f0, J, df, K, tau)
    A = np.abs(_unit_G(V, g, 0, 2, 3)[0])
    j = np.arange(1, J)
    sbd = np.abs(np.exp(2j * np.pi * j[None, :] * df * (tau - g["tau_s"][:, None])).sum(axis=1))
    f0a = np.array(f0)
    mbd = np.abs(np.exp(2j * np.pi * (f0a[None, :] - f0a[0]) * (tau - g["tau_m"][:, None])).sum(axis=1))
    ref = 2 * sbd[:, None] * mbd[None, :]
    assert np.max(np.abs(A - ref)) < 1e-9 * ref.max()


# ---------------------------------------------------------------- P6 Parseval
def test_parseval_sbd_and_mbd():
    """The SBD grid is a PJ-point DFT over j, so sum_s |X|^2 = PJ sum_j |Y|^2;
    the default MBD grid is an M-point DFT over distinct lattice positions of
    the IFs, so sum_m |G|^2 = M sum_n |X|^2."""
    rng = np.random.default_rng(7)
    f0 = [3000.0, 3032.0, 3096.0, 3224.0, 3256.0]
    J, df = 16, 1.0
    lay = _layout(f0, J, df, 1.0, 8)
    g = O.build_grids(lay, _search(n_mbd=32))
    Y = rng.standard_normal((1, 1, 5, J)) + 1j * rng.standard_normal((1, 1, 5, J))
    Y[..., 0] = 0
    X = Y @ g["e_sbd"]
    assert np.allclose((np.abs(X) ** 2).sum(-1), 64 * (np.abs(Y) ** 2).sum(-1), rtol=1e-12)
    G = O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])
    lhs = (np.abs(G[0, 0]) ** 2).sum(axis=1)
    rhs = 32 * (np.abs(X[0, 0]) ** 2).sum(axis=0)
    assert np.allclose(lhs, rhs, rtol=1e-12)


# ---------------------------------------------------------------- P8 Eq. 9
def test_additive_window_property():
    """Eq. 9 (Sec. 5.1): without the rate term G_{k0,l1} + G_{k0+l1,l2} =
    G_{k0,l1+l2}, cell by cell, with dispersion offsets in place."""
    rng = np.random.default_rng(3)
    f0 = [3000.0 + 32 * n for n in range(4)]
    J, df, K = 16, 1.0, 200
    lay = _layout(f0, J, df, 1.0, K)
    g = O.build_grids(lay, _search(dm_lo=300.0, n_dm=1, n_mbd=32))
    assert g["dk"].max() > 3
    V = rng.standard_normal((4, J, K)) + 1j * rng.standard_normal((4, J, K))
    a = _unit_G(V, g, 0, 3, 20)
    b = _unit_G(V, g, 0, 5, 23)
    c = _unit_G(V, g, 0, 8, 20)
    assert np.max(np.abs(a + b - c)) < 1e-10 * np.abs(c).max()


# ---------------------------------------------------------------- P9 f_ref,fit
def test_fit_reference_frequency_only_rotates_phase():
    """Eq. 5: changing f_ref,fit multiplies G(s, m) by exp(i 2 pi df_ref tau_m)
    and leaves |G| unchanged."""
    rng = np.random.default_rng(5)
    f0 = [3000.0 + 32 * n for n in range(4)]
    J, df = 16, 1.0
    lay = _layout(f0, J, df, 1.0, 30)
    g1 = O.build_grids(lay, _search(n_mbd=32))
    g2 = O.build_grids(lay, _search(n_mbd=32, f_ref_fit_mhz=3050.0))
    V = rng.standard_normal((4, J, 30)) + 1j * rng.standard_normal((4, J, 30))
    G1 = _unit_G(V, g1, 0, 4, 2)
    G2 = _unit_G(V, g2, 0, 4, 2)
    assert np.allclose(np.abs(G1), np.abs(G2), rtol=1e-12, atol=1e-12)
    rot = np.exp(2j * np.pi * (3050.0 - 3000.0) * g1["tau_m"])
    assert np.allclose(G2, G1 * rot[None, None, :], rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------- P10 calibration
def test_calibration_round_trip():
    """Eq. 5: a tone carrying per-IF channel delays tau0^n and phases phi0^n
    is restored to the full A l N (J-1) once the same values are applied;
    without them the peak is lower."""
    rng = np.random.default_rng(11)
    f0 = [3000.0 + 32 * n for n in range(6)]
    J, df, K = 32, 1.0, 20
    lay = _layout(f0, J, df, 1.0, K)
    g = O.build_grids(lay, _search(n_mbd=64, windows=[4]))
    tau0 = rng.uniform(-0.05, 0.05, 6)
    phi0 = rng.uniform(-np.pi, np.pi, 6)
    fj = np.arange(J) * df
    inst = np.exp(1j * (2 * np.pi * (fj[None, :] - J * df / 2) * tau0[:, None] + phi0[:, None]))
    V = _tone(f0, J, df, K, 0.0) * inst[:, :, None]
    cal = O.calibration_phasor(J, df, tau0, phi0)
    full = 4 * 6 * 31
    with_cal = np.abs(_unit_G(V, g, 0, 4, 3, cal)).max()
    without = np.abs(_unit_G(V, g, 0, 4, 3)).max()
    assert with_cal == pytest.approx(full, rel=1e-12)
    assert without < 0.95 * full


# ---------------------------------------------------------------- P12 rate
def test_on_grid_rate_peaks_at_its_bin():
    """Rate term of Eq. 4: a fringe rotating at a grid rate rho* (phase
    +2 pi f0^n rho* t about the window centre) gives full amplitude in bin r*
    and less in the others."""
    f0 = [3000.0 + 32 * n for n in range(4)]
    J, df, K, t_ap, l = 16, 1.0, 40, 1.0, 8
    lay = _layout(f0, J, df, t_ap, K)
    g = O.build_grids(lay, _search(n_mbd=32, n_rate=5, windows=[l]))
    r_star = 3
    rho = g["rates"][r_star]
    assert rho != 0
    k0 = 10
    kc = k0 + (l - 1) / 2.0
    k = np.arange(K)
    ph = np.exp(2j * np.pi * 1e3 * rho * np.array(f0)[:, None, None] * t_ap * (k[None, None, :] - kc))
    V = np.broadcast_to(ph, (4, J, K)).copy()
    G = _unit_G(V, g, 0, l, k0)
    A = np.abs(G).reshape(5, -1).max(axis=1)
    assert A[r_star] == pytest.approx(l * 4 * (J - 1), rel=1e-12)
    assert np.all(np.delete(A, r_star) < 0.99 * A[r_star])


def test_default_rate_step_hand_values():
    """The rate-grid default (a convention; the paper drops the rate term of
    Eq. 4): 1 / (2 f_max l_max t_ap) in Hz and seconds, f_max the highest
    channel sky frequency.  Values worked by hand:
      3000 MHz + 31 x 1 MHz points = 3.031e9 Hz, l_max 8, t_ap 1 ms:
        1 / (2 x 3.031e9 x 8 x 1e-3) = 1 / 48 496 000 s/s;
      VGOS top 10200 + 7 x 32 + 63 x 0.5 = 10455.5 MHz, l_max 16, 0.5 ms:
        1 / (2 x 10455.5e6 x 16 x 5e-4) = 1 / 167 288 000 s/s."""
    f0 = [3000.0 + 32 * n for n in range(1)]
    step = O.default_rate_step(f0, 32, 1.0, 1.0, [2, 8, 4])
    assert step == pytest.approx(1.0 / 48_496_000.0, rel=1e-14)
    f0 = [b + 32 * i for b in (3000.0, 5240.0, 6360.0, 10200.0) for i in range(8)]
    step = O.default_rate_step(f0, 64, 0.5, 0.5, [2, 4, 8, 16])
    assert step == pytest.approx(1.0 / 167_288_000.0, rel=1e-14)


@pytest.mark.parametrize("f0,J,df,t_ap,windows", [
    ([3000.0 + 32 * n for n in range(8)], 32, 1.0, 1.0, [1, 2, 4, 8]),
    ([2192.0 + 16 * n for n in range(6)], 32, 0.5, 1.024, [4, 8, 16, 24, 32]),
    ([2000.0 + 768 * n for n in range(16)], 256, 0.125, 0.1, [10, 20, 40]),
])
def test_default_rate_step_is_half_a_cycle_over_the_longest_window(f0, J, df, t_ap, windows):
    """The definition of the default rate step, checked physically: a delay
    rate rho turns the fringe of sky frequency f by f rho seconds of phase
    per second (a delay tau = rho t), so over the longest window (l_max APs
    of t_ap) at the top channel frequency one step turns it by exactly half a
    cycle; the grid built for a search uses that step, and the Eq. 4 rate
    phasor at the top frequency advances by the same half cycle across
    l_max APs."""
    step = O.default_rate_step(f0, J, df, t_ap, windows)
    f_top_hz = (max(f0) + (J - 1) * df) * 1e6       # MHz -> Hz
    window_s = max(windows) * t_ap * 1e-3           # ms -> s
    assert f_top_hz * step * window_s == pytest.approx(0.5, rel=1e-13)
    lay = _layout(f0, J, df, t_ap, 4 * max(windows) + 10)
    g = O.build_grids(lay, _search(n_mbd=256, n_rate=4, windows=windows))
    assert g["rates"][3] - g["rates"][2] == pytest.approx(step, rel=1e-13)
    assert g["rates"][2] == 0.0
    ph = O.rate_phasor([step], [max(f0) + (J - 1) * df], max(windows), t_ap)[0, 0]
    per_ap = -np.angle(ph[1] / ph[0]) / (2 * np.pi)  # cycles per AP (e^{-i phase})
    assert per_ap * max(windows) == pytest.approx(0.5, rel=1e-12)


# ---------------------------------------------------------------- P5 DM pulse
def test_pulse_at_dm0_full_power_only_at_dm0():
    """Eqs. 1-3: a noise-free boxcar of w frames placed along the exact Eq. 2
    sweep of DM0 (offsets from rational arithmetic) is summed in full by the
    DM0 trial with l = w: P = A w N (J-1); every other trial whose offsets are
    not a constant shift of DM0's collects strictly less."""
    f0 = [2000.0 + 16 * n for n in range(4)]
    J, df, t_ap, K = 16, 1.0, 1.0, 200
    dms = [0.0, 40.0, 80.0, 120.0, 160.0]
    d0 = 2
    lay = _layout(f0, J, df, t_ap, K)
    g = O.build_grids(lay, _search(dm_lo=0.0, dm_step=40.0, n_dm=5, n_mbd=32, windows=[4]))
    f = O.channel_sky_freq(f0, J, df)
    fr = f.max()
    w, k_p, A = 4, 60, 0.7
    V = np.zeros((4, J, K), dtype=np.complex128)
    for n in range(4):
        for j in range(J):
            dk, _ = _exact_dk(dms[d0], float(f[n, j]), fr, t_ap, 4.149e6)
            V[n, j, k_p + dk:k_p + dk + w] = A
    h = 2
    powers = []
    for d in range(5):
        q = k_p // h
        G = _unit_G(V, g, d, w, q * h)
        powers.append(np.abs(G).max())
    assert powers[d0] == pytest.approx(A * w * 4 * (J - 1), rel=1e-12)
    for d in range(5):
        if d != d0:
            shift = g["dk"][d] - g["dk"][d0]
            if not np.all(shift == shift.flat[0]):
                assert powers[d] < powers[d0] * (1 - 1e-6)


# ---------------------------------------------------------------- P11 noise
def test_noise_cell_power_expectation():
    """For CN(0,1) input, E|G(cell)|^2 = l N (J-1) at any fixed cell (the
    sum of l N (J-1) unit-power terms with unit-modulus phases)."""
    rng = np.random.default_rng(21)
    f0 = [3000.0 + 32 * n for n in range(4)]
    J, df, K, l = 8, 1.0, 2000, 4
    lay = _layout(f0, J, df, 1.0, K)
    g = O.build_grids(lay, _search(n_mbd=16, windows=[l]))
    V = (rng.standard_normal((4, J, K)) + 1j * rng.standard_normal((4, J, K))) / np.sqrt(2)
    rph = O.rate_phasor(g["rates"], g["f0"], l, 1.0)
    k0s = np.arange(0, K - l, l)
    Y = O.segment_sums(V, g["dk"][0], k0s, l, rph, np.ones((4, J)))
    G = O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])
    p = np.abs(G[:, 0, 5, 3]) ** 2
    expect = l * 4 * (J - 1)
    se = p.std() / np.sqrt(len(p))
    assert abs(p.mean() - expect) < 4 * se
    pn, mu, sd = O.normalise(np.abs(G).reshape(len(k0s), -1).max(axis=1))
    assert abs(pn.mean()) < 1e-12 and abs(pn.std() - 1) < 1e-12


# ---------------------------------------------------------------- segments
def test_segment_layout_bounds():
    """Eq. 3 bounds and the half-overlap hop: the last kept segment ends inside
    the data for the channel with the largest offset, the next would not."""
    K, dkm = 1000, 68
    for (l, h, Q) in O.segment_layout(K, dkm, [1, 2, 4, 8, 3]):
        assert h == max(1, l // 2)
        last = (Q - 1) * h + dkm + l - 1
        assert last <= K - 1
        assert Q * h + dkm + l - 1 > K - 1
    # the survey's count of segment positions for the single-baseline case
    assert sum(q for (_, _, q) in O.segment_layout(1000, 68, [1, 2, 4, 8])) == 2560


# ---------------------------------------------------------------- App. A
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_calibration_extraction_restores_full_power(seed):
    """Appendix A: channel delays and initial phases extracted from a
    calibrator segment, applied through Eq. 5, flatten the fringe phase: the
    calibrated peak equals the closed form A N (J-1) of a coherent sum, while
    the uncalibrated peak is clearly lower."""
    rng = np.random.default_rng(seed)
    f0 = [3000.0 + 32 * n for n in range(8)]
    J, df = 32, 1.0
    lay = _layout(f0, J, df, 1.0, 10)
    g = O.build_grids(lay, _search(n_mbd=256, windows=[2]))
    tau_n = rng.uniform(-0.05, 0.05, 8)
    psi = rng.uniform(-3, 3, 8)
    fj = np.arange(J) * df
    f = O.channel_sky_freq(f0, J, df)
    A = 100.0
    Y = A * np.exp(1j * (2 * np.pi * f * 0.013 + 2 * np.pi * fj[None, :] * tau_n[:, None] + psi[:, None]))
    tau0, phi0, sbd, mbd = O.calibrate(Y, f0, df, g["e_sbd"], g["e_mbd"], g["tau_s"], g["tau_m"],
                                       g["f_ref_fit"])
    Yc = Y * O.calibration_phasor(J, df, tau0, phi0)
    Yc[:, 0] = 0
    full = np.abs(O.fringe_matrix(Yc[None, None], g["e_sbd"], g["e_mbd"])).max()
    Y0 = Y.copy()
    Y0[:, 0] = 0
    raw = np.abs(O.fringe_matrix(Y0[None, None], g["e_sbd"], g["e_mbd"])).max()
    assert full == pytest.approx(A * 8 * (J - 1), rel=1e-9)
    assert raw < 0.7 * full
    # channel delays are recovered up to one common shift (absorbed by SBD)
    d = tau0 - tau_n
    assert np.ptp(d) < 1e-9


def test_power_summation_over_dm_trials():
    """Sec. 2.4.2 with the Sec. 5.3 merge: a pulse split evenly over two
    baselines, below threshold on each (2.8 sigma) but above it in the sum
    (~2.8 sqrt 2 sigma for independent noise), is detected in the summed
    power, at the DM trial where it is strongest."""
    rng = np.random.default_rng(4)
    segs = [(8, 4, 60), (4, 2, 120)]
    S = sum(q for (_, _, q) in segs)
    P = rng.uniform(1.0, 1.1, (2, 3, S))
    sig = 0.1 / np.sqrt(12.0)
    off = [0, 60]
    for d, k in [(0, 2.2), (1, 2.8), (2, 2.5)]:
        for wi, (l, h, Q) in enumerate(segs):
            P[:, d, off[wi] + 100 // h] = 1.05 + k * sig
    for b in range(2):
        assert O.normalise(P[b, 1, 0:60])[0].max() < 3.0
    assert O.normalise(P[0, 1, 0:60] + P[1, 1, 0:60])[0].max() > 3.0
    dets = O.power_sum_search(P, segs, 1.0, 3.0, 2, [0, 1])
    assert len(dets) == 1
    assert dets[0]["d"] == 1 and dets[0]["k0"] == 100 and dets[0]["n_windows"] == 2


# ---------------------------------------------------------------- non-finite data
def test_eq6_statistics_skip_non_finite_segments():
    """Eq. 6 with missing data: the mean and population standard deviation of
    a row are those of its finite powers alone (computed here with the
    standard library), a non-finite power gets no normalised power and never
    crosses, and the finite segments cross exactly as in the row without
    the missing ones."""
    import statistics
    rng = np.random.default_rng(5)
    P = rng.rayleigh(1.0, 400)
    P[[7, 100]] = 9.0                       # two strong segments
    bad = [3, 50, 51, 399]
    Pm = P.copy()
    Pm[bad[:2]] = np.nan
    Pm[bad[2]] = np.inf
    Pm[bad[3]] = -np.inf
    pn, mu, sd = O.normalise(Pm)
    fin = [float(x) for x in Pm if math.isfinite(x)]
    assert mu == pytest.approx(statistics.fmean(fin), rel=1e-13)
    assert sd == pytest.approx(statistics.pstdev(fin), rel=1e-12)
    assert np.all(np.isnan(pn[bad]))
    keep = np.setdiff1d(np.arange(400), bad)
    pk, _, _ = O.normalise(P[keep])
    assert np.allclose(pn[keep], pk, rtol=0, atol=1e-12)
    cr = O.crossings(pn, 3.0)
    assert not set(cr.tolist()) & set(bad)
    assert cr.tolist() == keep[O.crossings(pk, 3.0)].tolist()
    assert 7 in cr and 100 in cr
    # a row with no finite power has no statistics and no crossings
    pn0, mu0, sd0 = O.normalise(np.full(5, np.nan))
    assert pn0 is None and O.crossings(pn0, 3.0).size == 0


def test_nan_sample_makes_exactly_its_segments_non_finite():
    """A NaN sample in channel (n, j) at AP k spoils exactly the segments
    whose dedispersed frames include it (Eq. 3: AP k0 + dk_d(n, j) + u for
    u < l), counted here by brute force over the segment list; every other
    segment keeps its power, and a NaN in the DC point j = 0 (not fitted,
    Sec. 2.3) spoils nothing."""
    f0 = [3000.0, 3064.0]
    J, K = 8, 60
    lay = _layout(f0, J, 1.0, 1.0, K)
    lay["n_baselines"] = 1
    srch = _search(dm_lo=0.0, dm_step=300.0, n_dm=2, n_mbd=32, windows=[2, 4])
    rng = np.random.default_rng(6)
    V = (rng.standard_normal((1, 2, J, K)) + 1j * rng.standard_normal((1, 2, J, K))) / np.sqrt(2)
    clean = O.search(V, lay, srch)
    n, j, k = 1, 3, 20
    Vn = V.copy()
    Vn[0, n, j, k] = np.nan
    res = O.search(Vn, lay, srch)
    g = res["grids"]
    for d in range(2):
        for wi, (l, h, Q) in enumerate(g["segs"]):
            P = res["cube"][(0, d, wi)][0]
            dk = int(g["dk"][d][n][j])
            hit = np.array([q * h + dk <= k <= q * h + dk + l - 1 for q in range(Q)])
            assert hit.any()
            assert np.array_equal(np.isnan(P), hit)
            assert np.array_equal(P[~hit], clean["cube"][(0, d, wi)][0][~hit])
    Vd = V.copy()
    Vd[0, n, 0, k] = np.nan
    res_dc = O.search(Vd, lay, srch)
    for key, (P, _, _) in clean["cube"].items():
        assert np.array_equal(res_dc["cube"][key][0], P)
