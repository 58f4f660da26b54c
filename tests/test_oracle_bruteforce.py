"""P7: on tiny inputs the oracle's factored two-matrix-product form equals
the direct triple sum over (IF n, point j >= 1, AP u) of the paper's delay
resolution function (Eq. 4 with its rate term, Eq. 5 with the calibration
terms), evaluated cell by cell with the AP offsets of Eq. 2 taken from exact
rational arithmetic."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import frb_oracle as O


def _exact_dk(dm, freq, f_ref, t_ap, k_dm):
    F = Fraction
    x = F(k_dm) * F(dm) * (1 / (F(freq) * F(freq)) - 1 / (F(f_ref) * F(f_ref))) / F(t_ap)
    return math.floor(F(1, 2) + x)


@pytest.mark.parametrize("seed", [0, 1])
def test_bruteforce_triple_sum(seed):
    rng = np.random.default_rng(100 + seed)
    f0 = [2000.0, 2016.0, 2048.0]          # offsets 16, 48 MHz -> g = 16 MHz
    N, J, df, t_ap, K = 3, 8, 1.0, 1.0, 60
    P, M, R = 2, 16, 3
    PJ = P * J
    dms = [0.0, 150.0, 300.0]
    l = 3
    layout = dict(if_freq_mhz=f0, n_chan=J, chan_bw_mhz=df, t_ap_ms=t_ap, n_frames=K, n_if=N)
    search = dict(dm_lo=0.0, dm_step=150.0, n_dm=3, k_dm=4.149e6, sbd_pad=P, n_mbd=M,
                  mbd_step_us=0.0, f_ref_fit_mhz=float("nan"), n_rate=R, rate_step=2e-9,
                  windows=[l], threshold=3.0, n_win_min=1, n_bl_min=1)
    g = O.build_grids(layout, search)
    V = rng.standard_normal((N, J, K)) + 1j * rng.standard_normal((N, J, K))
    tau0 = rng.uniform(-0.03, 0.03, N)
    phi0 = rng.uniform(-3, 3, N)
    cal = O.calibration_phasor(J, df, tau0, phi0)
    rph = O.rate_phasor(g["rates"], g["f0"], l, t_ap)

    # grid values straight from their definitions
    tau_s = [(s - PJ / 2) / (PJ * df) for s in range(PJ)]
    T = 1.0 / 16.0
    tau_m = [(m - M / 2) * T / M for m in range(M)]
    rho = [(r - R // 2) * 2e-9 for r in range(R)]
    fref_dm = max(f0) + (J - 1) * df
    fbw = J * df

    for d, dm in enumerate(dms):
        dk = [[_exact_dk(dm, f0[n] + j * df, fref_dm, t_ap, 4.149e6) for j in range(J)]
              for n in range(N)]
        assert np.array_equal(np.array(dk), g["dk"][d])
        for k0 in (0, 7):
            Y = O.segment_sums(V, g["dk"][d], [k0], l, rph, cal)
            G = O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])[0]
            B = np.zeros((R, PJ, M), dtype=np.complex128)
            for r in range(R):
                for s in range(PJ):
                    for m in range(M):
                        acc = 0j
                        for n in range(N):
                            for j in range(1, J):
                                fj = j * df
                                for u in range(l):
                                    phi = (2 * math.pi * fj * tau_s[s]
                                           + 2 * math.pi * (f0[n] - f0[0]) * tau_m[m]
                                           + 2 * math.pi * f0[n] * rho[r] * t_ap * 1e3 * (u - (l - 1) / 2)
                                           + 2 * math.pi * (fj - fbw / 2) * tau0[n] + phi0[n])
                                    acc += V[n, j, k0 + dk[n][j] + u] * complex(math.cos(phi), -math.sin(phi))
                        B[r, s, m] = acc
            assert np.max(np.abs(G - B)) < 1e-10 * np.abs(B).max()
            # the oracle's peak: value and lowest flat index of the maximum
            pk, idx, _ = O.peak(G[None])
            A = np.abs(B).ravel()
            assert pk[0] == pytest.approx(A.max(), rel=1e-12)
            assert idx[0] == int(np.argmax(A))
