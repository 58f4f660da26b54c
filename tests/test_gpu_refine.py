"""GPU tests of the refinement of coarse peaks: the forward, backward and
curvature kernels against the FP64 oracle (R3-R4), the gradient against
central finite differences, the library's ascent against the same ascent
driven through the torch.autograd.Function, and recovery of injected
pulses within 0.05 grid cell."""
import math

import numpy as np
import pytest
import torch

from oracle import frb_oracle as O
from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

from gpu_helpers import note

pytestmark = pytest.mark.gpu

F0_8 = [3000.0 + 32.0 * n for n in range(8)]


def _search(wl, V, f16=False):
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    if f16:
        s.load(torch.from_numpy(W.to_complex32(V)).cuda())
    else:
        s.load(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    s.run()
    return s


def _noisy_workload():
    return W.custom_workload(
        if_freq_mhz=F0_8, n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=700, n_stations=3,
        config_id=150,
        search=dict(dm_lo=0.0, dm_step=15.625, n_dm=24, sbd_pad=4, n_mbd=256, n_rate=3,
                    windows=[2, 4, 8], threshold=3.0, n_win_min=2, n_bl_min=2),
        signal=dict(pulses=dict(kind="fixed", list=[
            dict(t0_ms=150.2, dm=180.0, width_ms=4.0, snr=20.0, delay_us=0.011),
            dict(t0_ms=380.7, dm=290.0, width_ms=2.0, snr=25.0, delay_us=-0.023)])))


@pytest.fixture(scope="module")
def noisy():
    wl = _noisy_workload()
    V, _ = W.generate(wl)
    s = _search(wl, V)
    peaks = s.top_peaks(48)
    assert len(peaks) == 48
    return wl, V, s, peaks


def _oracle_eval(wl, V, p, th, cal=None):
    lay, srch = wl["layout"], wl["search"]
    N, J = len(lay["if_freq_mhz"]), lay["n_chan"]
    cal = np.ones((N, J), complex) if cal is None else cal
    G, dG, d2G = O.relaxed_fringe(V[p["baseline"]].astype(np.complex128), lay, srch, cal, p["k0"],
                                  p["window_len"], th)
    return O.relaxed_power_grad(G, dG, d2G)


def test_top_peaks_are_the_crossings_by_normalised_power(noisy):
    _, _, s, peaks = noisy
    cr = sorted(s.crossings(), key=lambda c: (-c["power_norm"], c["baseline"], c["dm_index"],
                                              c["window_index"], c["segment"]))
    assert [(p["baseline"], p["dm_index"], p["window_index"], p["segment"]) for p in peaks] == \
           [(c["baseline"], c["dm_index"], c["window_index"], c["segment"]) for c in cr[:48]]


def test_forward_backward_curvature_match_the_oracle(noisy):
    wl, V, s, peaks = noisy
    th0 = s.refine_begin(peaks)
    cells, _ = s.refine_cells()
    assert np.allclose(cells, O.refine_cells(wl["layout"], wl["search"]), rtol=1e-12)
    rng = np.random.default_rng(7)
    th = th0 + rng.uniform(-0.45, 0.45, th0.shape) * np.where(cells > 0, cells, 0.0)
    th[::5, 4] -= 3.0                        # some windows partly before their segment start
    tt = torch.tensor(th, dtype=torch.float64, device="cuda")
    note("refine forward/backward/curvature")
    P = s.refine_forward(tt).cpu().numpy()
    g = s.refine_backward(tt, torch.ones(len(peaks), dtype=torch.float32, device="cuda")).cpu().numpy()
    H = s.refine_curvature(tt).cpu().numpy()
    worst = np.zeros(3)
    for i in range(0, len(peaks), 3):
        Po, go, Ho = _oracle_eval(wl, V, peaks[i], th[i])
        assert P[i] == pytest.approx(Po, rel=2e-5)
        for k in range(5):
            if cells[k] == 0:
                continue
            gs = Po / cells[k]
            worst[0] = max(worst[0], abs(P[i] - Po) / Po)
            worst[1] = max(worst[1], abs(g[i, k] - go[k]) / (abs(go[k]) + gs))
            assert abs(g[i, k] - go[k]) <= 2e-4 * (abs(go[k]) + gs), (i, k, g[i, k], go[k])
            assert abs(H[i, k] - Ho[k]) <= 2e-3 * (abs(Ho[k]) + gs / cells[k]), (i, k, H[i, k], Ho[k])
        assert abs(H[i, 5] - Ho[5]) <= 2e-3 * (abs(Ho[5]) + Po / (cells[3] * cells[4]))
    note(f"worst P rel {worst[0]:.2e}, worst gradient rel {worst[1]:.2e}")


def test_gradient_matches_central_differences(noisy):
    """dP/dtheta of the backward kernel against central differences with
    h = 1e-3 grid cell, taken on the FP64 oracle's P (rel err <= 1e-3, with
    a floor of 1e-2 P per cell for near-zero components) and on the device's
    own float32 P with h = 1e-2 cell."""
    wl, V, s, peaks = noisy
    th0 = s.refine_begin(peaks)
    cells, _ = s.refine_cells()
    rng = np.random.default_rng(11)
    th = th0 + rng.uniform(-0.3, 0.3, th0.shape) * np.where(cells > 0, cells, 0.0)
    tt = torch.tensor(th, dtype=torch.float64, device="cuda")
    g = s.refine_backward(tt, torch.ones(len(peaks), dtype=torch.float32, device="cuda")).cpu().numpy()
    P = s.refine_forward(tt).cpu().numpy()
    rel = []
    for i in range(0, len(peaks), 6):
        for k in range(5):
            if cells[k] == 0:
                continue
            h = 1e-3 * cells[k]
            e = np.zeros(5)
            e[k] = h
            fd = (_oracle_eval(wl, V, peaks[i], th[i] + e)[0] - _oracle_eval(wl, V, peaks[i], th[i] - e)[0]) / (2 * h)
            r = abs(g[i, k] - fd) / max(abs(fd), 1e-2 * P[i] / cells[k])
            rel.append(r)
            assert r <= 1e-3, (i, k, g[i, k], fd)
    # the device's own forward, float32 sums: a coarser step
    for k in range(5):
        if cells[k] == 0:
            continue
        e = torch.zeros_like(tt)
        e[:, k] = 1e-2 * cells[k]
        fd = ((s.refine_forward(tt + e) - s.refine_forward(tt - e)).double() / (2e-2 * cells[k])).cpu().numpy()
        err = np.abs(g[:, k] - fd) / np.maximum(np.abs(fd), 1e-1 * P / cells[k])
        assert np.all(err <= 1e-2), (k, err.max())
    note(f"gradient vs FP64 central differences: worst rel {max(rel):.2e}")


def test_autograd_function_drives_a_torch_optimiser(noisy):
    """P(theta) as a torch.autograd.Function (forward and backward kernels):
    autograd's gradient of P.sum() is the backward kernel's, and plain
    gradient-ascent steps in grid-cell units taken by a torch optimiser
    raise every peak's power; the library's own ascent (step kernel) never
    ends below its start."""
    from paper_1801_02391_amd.frbx import refine_power
    wl, V, s, peaks = noisy
    sub = peaks[:16]
    note("native ascent")
    th0, th_nat, P_nat = s.refine(sub, steps=20)
    P0 = s.refine_forward(torch.tensor(th0, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.all(P_nat >= P0 * (1 - 1e-6))
    note("autograd")
    s.refine_begin(sub)
    cells, _ = s.refine_cells()
    scale = torch.tensor(np.where(cells > 0, cells, 0.0), dtype=torch.float64, device="cuda")
    z = torch.zeros((len(sub), 5), dtype=torch.float64, device="cuda", requires_grad=True)
    base = torch.tensor(th0, dtype=torch.float64, device="cuda")
    P = refine_power(base + z * scale, s)
    P.sum().backward()
    g_ref = s.refine_backward(base.contiguous(), torch.ones(len(sub), dtype=torch.float32, device="cuda"))
    assert torch.allclose(z.grad, g_ref * scale, rtol=1e-12, atol=0.0)
    # a few small normalised gradient-ascent steps (0.02 cell at most)
    opt = torch.optim.SGD([z], lr=1.0)
    first = P.detach().clone()
    for _ in range(3):
        opt.zero_grad()
        P = refine_power(base + z * scale, s)
        (-P.sum()).backward()
        with torch.no_grad():
            gmax = z.grad.abs().amax(dim=1, keepdim=True).clamp_min(1e-30)
            z.grad.mul_(0.02 / gmax)
        opt.step()
    last = s.refine_forward((base + z.detach() * scale).contiguous())
    assert torch.all(last >= first * (1 - 1e-3)), (last - first).min().item()
    assert torch.mean((last > first).float()).item() > 0.5


@pytest.mark.parametrize("seed", [0, 1, 4])
def test_refinement_recovers_noise_free_pulse_within_0p05_cell(seed):
    rng = np.random.default_rng(100 + seed)
    dm, w = float(rng.uniform(200, 800)), int(rng.integers(2, 7))
    tau, t0 = float(rng.uniform(-0.4, 0.4)), float(rng.uniform(30, 60))
    step = 15.625
    lo = max(0, int(dm / step) - 2)
    wl = W.custom_workload(if_freq_mhz=F0_8, n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=260,
                           config_id=140 + seed,
                           search=dict(dm_lo=lo * step, dm_step=step, n_dm=5, sbd_pad=4, n_mbd=256,
                                       n_rate=3, windows=[w], threshold=0.5, n_win_min=1, n_bl_min=1),
                           signal=dict(noise=False, pulses=dict(kind="fixed", list=[
                               dict(t0_ms=t0, dm=dm, width_ms=float(w), snr=30.0, delay_us=tau)])))
    V, _ = W.generate(wl)
    note(f"seed {seed}: search")
    s = _search(wl, V)
    P, I = s.power_cube()
    d, q = np.unravel_index(int(np.argmax(P[0])), P[0].shape)
    R, PJ, M = 3, 4 * 32, 256
    idx = int(I[0, d, q])
    peak = dict(baseline=0, dm_index=int(d), window_len=w, k0=int(q) * max(1, w // 2),
                rate_idx=idx // (PJ * M), sbd_idx=(idx // M) % PJ, mbd_idx=idx % M)
    note(f"seed {seed}: refine")
    th0, th, Pf = s.refine([peak], steps=20)
    cells, _ = s.refine_cells()
    T = O.build_grids(wl["layout"], wl["search"])["t_amb"]
    err = (th[0] - np.array([tau, tau, 0.0, dm, t0 - peak["k0"]])) / cells
    err[1] = ((th[0, 1] - tau + T / 2) % T - T / 2) / cells[1]
    note(f"seed {seed}: errors in cells {np.round(err, 4)}")
    assert np.all(np.abs(err) < 0.05), err
    # the oracle's ascent from the same start lands on the same point
    lay, srch = wl["layout"], wl["search"]
    cal = np.ones((8, 32), complex)
    fn = lambda t: O.relaxed_power_grad(*O.relaxed_fringe(V[0].astype(np.complex128), lay, srch, cal,
                                                          peak["k0"], w, t))
    tho, _ = O.newton_ascent(fn, th0[0], O.refine_cells(lay, srch), O.mean_dm_shift(lay), steps=20)
    assert np.all(np.abs(th[0] - tho) / cells < 0.01)


def test_refinement_on_complex32_input_matches_the_oracle_on_the_stored_values(noisy):
    wl, V, _, peaks = noisy
    V16 = W.from_complex32(W.to_complex32(V))
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.load(torch.from_numpy(W.to_complex32(V)).cuda())
    th0 = s.refine_begin(peaks[:8])
    tt = torch.tensor(th0, dtype=torch.float64, device="cuda")
    P = s.refine_forward(tt).cpu().numpy()
    for i in range(8):
        Po = _oracle_eval(wl, V16, peaks[i], th0[i])[0]
        assert P[i] == pytest.approx(Po, rel=2e-5)


def test_refine_state_errors():
    wl = _noisy_workload()
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    with pytest.raises(frbx.FrbxError):
        s.refine_begin([dict(baseline=0, dm_index=0, window_len=2, k0=0, rate_idx=0, sbd_idx=0, mbd_idx=0)])
    V, _ = W.generate(wl)
    s.load(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    with pytest.raises(frbx.FrbxError):
        s.refine_begin([dict(baseline=7, dm_index=0, window_len=2, k0=0, rate_idx=0, sbd_idx=0, mbd_idx=0)])
    with pytest.raises(frbx.FrbxError):
        s.refine_begin([dict(baseline=0, dm_index=0, window_len=2, k0=0, rate_idx=0, sbd_idx=999, mbd_idx=0)])
    th0, th, P = s.refine([], steps=5)
    assert th.shape[0] == 0


def test_refinement_applies_the_calibration():
    """With per-IF channel delays and initial phases set, the refinement's
    |G| and gradient equal the oracle's with the same Eq. 5 calibration."""
    wl = _noisy_workload()
    V, _ = W.generate(wl)
    lay = wl["layout"]
    B, N, J = lay["n_baselines"], lay["n_if"], lay["n_chan"]
    rng = np.random.default_rng(21)
    tau0 = rng.uniform(-0.02, 0.02, (B, N))
    phi0 = rng.uniform(-np.pi, np.pi, (B, N))
    s = frbx.Search(lay)
    s.configure(wl["search"], tau0, phi0)
    s.load(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    s.run()
    peaks = s.top_peaks(12)
    th0 = s.refine_begin(peaks)
    cells, _ = s.refine_cells()
    th = th0 + 0.2 * np.where(cells > 0, cells, 0.0)
    tt = torch.tensor(th, dtype=torch.float64, device="cuda")
    P = s.refine_forward(tt).cpu().numpy()
    g = s.refine_backward(tt, torch.ones(len(peaks), dtype=torch.float32, device="cuda")).cpu().numpy()
    for i, p in enumerate(peaks):
        cal = O.calibration_phasor(J, lay["chan_bw_mhz"], tau0[p["baseline"]], phi0[p["baseline"]])
        Po, go, _ = _oracle_eval(wl, V, p, th[i], cal)
        assert P[i] == pytest.approx(Po, rel=2e-5)
        for k in range(5):
            if cells[k] > 0:
                assert abs(g[i, k] - go[k]) <= 2e-4 * (abs(go[k]) + Po / cells[k])
