"""GPU parity of the HIP search against the FP64 oracle, through the C ABI.

Element-wise: the |G|^2 grid of single segments.  End-to-end: power cube,
peak indices, Eq. 6 statistics, crossings and the grouped detections, on
seeded synthetic inputs small enough for the oracle, with several DM tiles,
ragged channel / AP tails and every transform size the workloads use."""
import os

import numpy as np
import pytest

from oracle import frb_oracle as O
from paper_1801_02391_amd import workloads as W

from gpu_helpers import (POWER_RTOL, compare_crossings, compare_powers, note, oracle_cube,
                         run_gpu)

pytestmark = pytest.mark.gpu


def _tiny(J, M, N=3, R=3, P=4, K=260, windows=(1, 2, 4, 8), n_dm=3, dm_step=120.0, B=None,
          n_stations=3, pulses=None, seed_id=50, if_step=16.0):
    # IF offsets 0, 1, 3, 6, 10, ... times if_step: distinct lattice points
    f0 = [2000.0 + if_step * n * (n + 1) / 2 for n in range(N)]
    sig = dict(noise=True, rfi_frac=0.0, rfi_amp=0.0,
               pulses=pulses or dict(kind="fixed", list=[dict(t0_ms=120.0, dm=dm_step, width_ms=3.0,
                                                                snr=25.0, delay_us=0.01)]))
    return W.custom_workload(if_freq_mhz=f0, n_chan=J, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=K,
                             n_stations=n_stations, config_id=seed_id,
                             search=dict(dm_lo=0.0, dm_step=dm_step, n_dm=n_dm, sbd_pad=P, n_mbd=M,
                                         n_rate=R, windows=list(windows), threshold=3.0,
                                         n_win_min=2, n_bl_min=2),
                             signal=sig)


SHAPES = [  # (J, M, N, R, P)
    (8, 16, 2, 1, 4),
    (16, 64, 3, 3, 4),
    (32, 256, 8, 1, 4),
    (64, 256, 4, 2, 4),
    (64, 64, 5, 1, 2),
    (128, 32, 3, 1, 1),
    (256, 16, 2, 2, 1),
]


@pytest.mark.parametrize("J,M,N,R,P", SHAPES)
def test_segment_grid_elementwise(J, M, N, R, P):
    """Every (rate, SBD, MBD) cell of |G|^2 for two segments, against the
    oracle's Eq. 5 grid (the GPU grid differs from the oracle's only by the
    f_ref,fit phase, which |G| does not see)."""
    wl = _tiny(J, M, N=N, R=R, P=P, K=120, windows=(3, 8), n_dm=2, n_stations=2, seed_id=60 + J)
    V, _ = W.generate(wl)
    g = O.build_grids(wl["layout"], wl["search"])
    out = run_gpu(wl, V)
    s = out["search"]
    cal = np.ones((N, J))
    for (d, wi, q) in [(0, 0, 0), (1, 1, g["segs"][1][2] - 1)]:
        note(f"dump J={J} M={M} d={d} wi={wi} q={q}")
        grid = s.dump_segment(0, d, wi, q)
        l, h, _ = g["segs"][wi]
        rph = O.rate_phasor(g["rates"], g["f0"], l, g["t_ap"])
        Y = O.segment_sums(V[0], g["dk"][d], [q * h], l, rph, cal)
        G = np.abs(O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])[0]) ** 2
        assert grid.shape == G.shape
        err = np.abs(grid - G).max() / G.max()
        assert err < 2e-5, f"grid error {err:.3g}"


@pytest.mark.parametrize("J,M,N,R,P", SHAPES[:5])
def test_search_matches_oracle_end_to_end(J, M, N, R, P, monkeypatch):
    """Full search on 3 baselines x 3 DM trials x 4 windows (ragged segment
    counts) with DM tiles of one trial each (small W budget): power cube,
    indices, statistics, crossings and the grouped detections."""
    monkeypatch.setenv("FRBX_W_BUDGET_MB", "1")
    wl = _tiny(J, M, N=N, R=R, P=P, seed_id=70 + J + M)
    V, _ = W.generate(wl)
    gpu = run_gpu(wl, V)
    note("oracle")
    ora = O.search(V, wl["layout"], wl["search"])
    segs = ora["grids"]["segs"]
    assert gpu["seg"]["n_seg"] == [q for (_, _, q) in segs]
    assert gpu["seg"]["dk_max"] == ora["grids"]["dk_max"]
    B, D = wl["layout"]["n_baselines"], wl["search"]["n_dm"]
    Po, Io, S2o = oracle_cube(ora, B, D, segs)
    n_idx = compare_powers(gpu["P"], gpu["I"], Po, Io, S2o, "cube")
    assert n_idx > 0.1 * Po.size   # broad MBD peaks with few IFs leave many small margins
    # Eq. 6 statistics per (b, d, window)
    nw = len(segs)
    for (b, d, wi), (mu, sd) in ora["stats"].items():
        row = (b * D + d) * nw + wi
        assert gpu["mean"][row] == pytest.approx(mu, rel=2e-5)
        assert gpu["sd"][row] == pytest.approx(sd, rel=2e-3, abs=1e-6 * mu)
    compare_crossings(gpu["crossings"], ora["crossings"], wl["search"]["threshold"])
    # grouping: library output equals the oracle's grouping of the same crossings
    from paper_1801_02391_amd import frbx
    oc = [dict(b=c["baseline"], d=c["dm_index"], l=c["window_len"], k0=c["k0"],
               p_norm=c["power_norm"], mbd_us=c["mbd_us"]) for c in gpu["crossings"]]
    odets, ogroups, _ = O.detect(oc, ora["grids"]["t_amb"], wl["search"]["n_win_min"],
                                 wl["search"]["n_bl_min"])
    assert [(d["baseline"], d["dm_index"], d["k0"], d["window_len"]) for d in gpu["candidates"]] == \
           [(d["b"], d["d"], d["k0"], d["l"]) for d in odets]
    assert [g["n_baselines"] for g in gpu["groups"]] == [g["n_baselines"] for g in ogroups]


def test_dedispersion_tiles_full_and_ragged():
    """Every kind of dedispersion tile: 24 channels (one full and one partial
    16-channel tile) over 700 APs (two full 256-AP tiles and a partial one),
    the three DM trials staged as one group: power cube, indices and Eq. 6
    statistics against the oracle."""
    wl = _tiny(8, 16, N=3, R=1, P=4, K=700, n_dm=3, dm_step=60.0, seed_id=91)
    V, _ = W.generate(wl)
    gpu = run_gpu(wl, V)
    note("oracle")
    ora = O.search(V, wl["layout"], wl["search"])
    dk_max = ora["grids"]["dk_max"]
    assert gpu["seg"]["dk_max"] == dk_max and 700 - dk_max > 512
    segs = ora["grids"]["segs"]
    B, D = wl["layout"]["n_baselines"], wl["search"]["n_dm"]
    Po, Io, S2o = oracle_cube(ora, B, D, segs)
    compare_powers(gpu["P"], gpu["I"], Po, Io, S2o, "cube")
    nw = len(segs)
    for (b, d, wi), (mu, sd) in ora["stats"].items():
        row = (b * D + d) * nw + wi
        assert gpu["mean"][row] == pytest.approx(mu, rel=2e-5)


def test_zero_input_and_degenerate_single_if():
    """All-zero spectra: every power is 0 with the lowest packed index 0 and
    no crossings; one IF: the MBD axis is flat and the lowest MBD bin wins."""
    wl = _tiny(32, 64, N=1, R=2, P=4, K=100, windows=(2, 5), n_dm=2, n_stations=2, seed_id=80)
    V = np.zeros((1, 1, 32, 100), dtype=np.complex64)
    gpu = run_gpu(wl, V)
    assert np.all(gpu["P"] == 0) and np.all(gpu["I"] == 0)
    assert gpu["crossings"] == [] and gpu["candidates"] == []
    V2, _ = W.generate(wl)
    gpu2 = run_gpu(wl, V2)
    ora = O.search(V2, wl["layout"], wl["search"])
    Po, Io, S2o = oracle_cube(ora, 1, 2, ora["grids"]["segs"])
    rel = np.abs(gpu2["P"] - Po) / Po
    assert rel.max() <= POWER_RTOL
    assert np.all(Io % 64 == 0)                # exact ties: the oracle takes m = 0
    # the device's flat MBD axis is equal only up to float32 rounding, so its
    # index may be any cell of the maximal (r, s) column: check that it is one
    g = ora["grids"]
    segs = g["segs"]
    off = np.cumsum([0] + [q for (_, _, q) in segs])
    cal = np.ones((1, 32))
    for d in range(2):
        for wi, (l, h, Q) in enumerate(segs):
            rph = O.rate_phasor(g["rates"], g["f0"], l, g["t_ap"])
            Y = O.segment_sums(V2[0], g["dk"][d], np.arange(Q) * h, l, rph, cal)
            A = np.abs(O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])).reshape(Q, -1)
            gi = gpu2["I"][0, d, off[wi]:off[wi + 1]]
            picked = A[np.arange(Q), gi]
            assert np.all(picked >= A.max(axis=1) * (1 - POWER_RTOL))


def test_window_longer_than_data_and_dm_zero_identity():
    """A window longer than the data after dedispersion has no segments; a
    single DM = 0 trial sums plain AP windows (checked through the grid
    dump against a direct slice sum)."""
    wl = _tiny(16, 16, N=2, R=1, P=2, K=40, windows=(2, 64), n_dm=1, dm_step=0.0, n_stations=2,
               seed_id=81)
    V, _ = W.generate(wl)
    gpu = run_gpu(wl, V)
    assert gpu["seg"]["n_seg"][1] == 0 and gpu["seg"]["n_seg"][0] == 39
    ora = O.search(V, wl["layout"], wl["search"])
    Po, Io, S2o = oracle_cube(ora, 1, 1, ora["grids"]["segs"])
    compare_powers(gpu["P"], gpu["I"], Po, Io, S2o, "dm0")
    g = ora["grids"]
    grid = gpu["search"].dump_segment(0, 0, 0, 5)
    Y = V[0][:, :, 5:7].astype(np.complex128).sum(axis=2)[None, None]
    Y[..., 0] = 0
    G = np.abs(O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])[0, 0]) ** 2
    assert np.abs(grid[0] - G).max() / G.max() < 2e-5


def test_calibration_applied_on_device():
    """Eq. 5 calibration: with per-(baseline, IF) channel delays and initial
    phases the device result matches the oracle's calibrated search."""
    wl = _tiny(32, 64, N=4, R=1, P=4, K=150, windows=(2, 4), n_dm=2, n_stations=3, seed_id=82)
    V, _ = W.generate(wl)
    rng = np.random.default_rng(5)
    B, N = wl["layout"]["n_baselines"], 4
    tau0 = rng.uniform(-0.05, 0.05, (B, N))
    phi0 = rng.uniform(-3, 3, (B, N))
    gpu = run_gpu(wl, V, tau0, phi0)
    ora = O.search(V, wl["layout"], wl["search"], tau0_us=tau0, phi0_rad=phi0)
    Po, Io, S2o = oracle_cube(ora, B, 2, ora["grids"]["segs"])
    compare_powers(gpu["P"], gpu["I"], Po, Io, S2o, "calibrated")


def test_repeat_runs_are_bit_identical():
    wl = _tiny(64, 256, N=4, R=2, P=4, K=200, windows=(2, 4), n_dm=2, n_stations=2, seed_id=83)
    V, _ = W.generate(wl)
    a = run_gpu(wl, V)
    s = a["search"]
    s.run()
    P2, I2 = s.power_cube()
    assert np.array_equal(a["P"].view(np.uint32), P2.view(np.uint32))
    assert np.array_equal(a["I"], I2)


def test_single_baseline_workload():
    """The single-baseline workload (8 IFs x 32 x 1 MHz, 1000 APs, 64 DM
    trials, 4x zero padding, M = 256): full device search; the oracle on the
    DM trials around the injected DM 500 and at the grid ends; the injected
    pulse is the strongest detection, at DM trial 32 with its MBD."""
    wl = W.get_workload("single-1bl-8x32-1000")
    V, truth = W.generate(wl)
    gpu = run_gpu(wl, V)
    dsel = [0, 31, 32, 33, 63]
    note("oracle on DM subset")
    ora = O.search(V, wl["layout"], wl["search"], dm_indices=dsel)
    segs = ora["grids"]["segs"]
    Po, Io, S2o = oracle_cube(ora, 1, 64, segs)
    compare_powers(gpu["P"][:, dsel], gpu["I"][:, dsel], Po[:, dsel], Io[:, dsel], S2o[:, dsel],
                   "single")
    best = max(gpu["candidates"], key=lambda c: c["power_norm"])
    assert best["dm_index"] == 32 and abs(best["k0"] - 400) <= 2
    assert O.wrapped_diff(best["mbd_us"], 0.020, ora["grids"]["t_amb"]) == pytest.approx(0, abs=2e-3)


LATTICES = {  # (IF sky frequencies in MHz on a 16 MHz lattice, M); J = 32
    # first-pass rows: 16 positions at M = 256, 8 at M = 128
    "compact-wrapped": ([3000.0, 2984.0, 3016.0, 2968.0, 3032.0, 2952.0], 256),  # q = 0, -1, 1, -2, 2, -3
    "compact-edge": ([3000.0, 3240.0, 3016.0], 256),                               # q = 0, 15, 1
    "general-edge": ([3000.0, 3256.0, 3016.0], 256),                               # q = 0, 16, 1
    "general-spread": ([3000.0, 3016.0, 3512.0, 3048.0], 256),                     # q = 0, 1, 32, 3
    "compact-edge-m128": ([3000.0, 3016.0, 3112.0], 128),                          # q = 0, 1, 7
    "general-edge-m128": ([3000.0, 3016.0, 3128.0], 128),                          # q = 0, 1, 8
}


@pytest.mark.parametrize("name", list(LATTICES))
def test_compact_and_general_mbd_lattices(name):
    """The MBD transform takes a one-pass form when every IF's lattice
    position fits in one row of the first pass after a common shift (the
    shift is a phase factor on G); both forms against the oracle: power cube
    and indices, and the full |G|^2 grid of one segment."""
    f0, M = LATTICES[name]
    J = 32
    rows = 16 if M == 256 else 8
    wl = W.custom_workload(if_freq_mhz=f0, n_chan=J, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=200,
                           n_stations=2, config_id=90 + len(f0),
                           search=dict(dm_lo=0.0, dm_step=80.0, n_dm=2, sbd_pad=4, n_mbd=M, n_rate=2,
                                       windows=[2, 5], threshold=3.0, n_win_min=2, n_bl_min=1),
                           signal=dict(pulses=dict(kind="fixed", list=[
                               dict(t0_ms=90.0, dm=80.0, width_ms=4.0, snr=20.0, delay_us=0.03)])))
    V, _ = W.generate(wl)
    gpu = run_gpu(wl, V)
    ora = O.search(V, wl["layout"], wl["search"])
    lat = gpu["search"].lattice()
    t_amb = ora["grids"]["t_amb"]
    assert lat["mbd_step_us"] == pytest.approx(t_amb / M, rel=1e-12)
    q = [round((f - f0[0]) * t_amb) % M for f in f0]
    assert lat["q"] == q
    if name.startswith("compact"):
        assert lat["compact_shift"] in q and max((x - lat["compact_shift"]) % M for x in q) < rows
    else:
        assert lat["compact_shift"] == -1
    segs = ora["grids"]["segs"]
    Po, Io, S2o = oracle_cube(ora, 1, 2, segs)
    # (few IFs on a narrow lattice give broad MBD peaks: most margins are
    # small, so the dumped segment's peak cell is checked against the grid)
    compare_powers(gpu["P"], gpu["I"], Po, Io, S2o, name)
    g = ora["grids"]
    l, h, Q = g["segs"][1]
    q = Q // 2
    note(f"dump {name} q={q}")
    grid = gpu["search"].dump_segment(0, 1, 1, q)
    rph = O.rate_phasor(g["rates"], g["f0"], l, g["t_ap"])
    Y = O.segment_sums(V[0], g["dk"][1], [q * h], l, rph, np.ones((len(f0), J)))
    G = np.abs(O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])[0]) ** 2
    assert grid.shape == G.shape
    assert np.abs(grid - G).max() / G.max() < 2e-5
    idx = int(gpu["I"][0, 1, g["segs"][0][2] + q])
    assert G.ravel()[idx] >= G.max() * (1 - 2e-4)
