"""GPU parity of the matrix-core forms of the fringe transform.

f16x3 (three float16 products of a high/low split, float32 accumulation;
with 17-32 IFs each complex product built from three real ones) is held to
the float32 bar: powers within 1e-4 of the FP64 oracle, indices
exact where the oracle's margin exceeds 1e-3.  f16 (one float16 product) is
the low-precision form: powers within 1e-3, indices exact where the margin
exceeds 4e-3, and it is run on complex32 (float16) stored inputs, against
the oracle on the same stored values."""
import numpy as np
import pytest

from oracle import frb_oracle as O
from paper_1801_02391_amd import workloads as W

from gpu_helpers import compare_crossings, note, oracle_cube, run_gpu

pytestmark = pytest.mark.gpu


def _wl(J, N, R, K=220, windows=(2, 4, 8), n_dm=3, seed_id=90, precision="f16x3"):
    f0 = [3000.0 + 32.0 * n * (n + 1) / 2 for n in range(N)]
    return W.custom_workload(
        if_freq_mhz=f0, n_chan=J, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=K, n_stations=3,
        config_id=seed_id,
        search=dict(dm_lo=0.0, dm_step=150.0, n_dm=n_dm, sbd_pad=4, n_mbd=256, n_rate=R,
                    windows=list(windows), threshold=3.0, n_win_min=2, n_bl_min=2,
                    precision=precision),
        signal=dict(pulses=dict(kind="fixed", list=[
            dict(t0_ms=100.0, dm=150.0, width_ms=4.0, snr=30.0, delay_us=0.011)])))


def _check(gpu, ora, B, D, rtol, margin):
    segs = ora["grids"]["segs"]
    Po, Io, S2o = oracle_cube(ora, B, D, segs)
    Pg = gpu["P"].astype(np.float64)
    rel = np.abs(Pg - Po) / Po
    assert rel.max() <= rtol, f"power rel err {rel.max():.3g}"
    sel = (Po - S2o) / Po > margin
    assert sel.sum() > 0.05 * sel.size
    assert np.all(gpu["I"][sel] == Io[sel]), f"{np.sum(gpu['I'][sel] != Io[sel])} index mismatches"
    return rel.max()


@pytest.mark.parametrize("J,N,R", [(32, 8, 1), (64, 32, 2), (16, 12, 3), (128, 20, 1), (32, 17, 2)])
def test_f16x3_matches_oracle_at_float32_bar(J, N, R):
    wl = _wl(J, N, R, seed_id=91 + J + N)
    V, _ = W.generate(wl)
    gpu = run_gpu(wl, V)
    ora = O.search(V, wl["layout"], wl["search"])
    err = _check(gpu, ora, wl["layout"]["n_baselines"], wl["search"]["n_dm"], 1e-4, 1e-3)
    note(f"f16x3 J={J} N={N}: max power rel err {err:.2e}")
    compare_crossings(gpu["crossings"], ora["crossings"], 3.0)


@pytest.mark.parametrize("J,N,R,sbd_mfma", [(64, 32, 2, False), (64, 32, 2, True), (32, 8, 1, False),
                                            (32, 8, 1, True), (16, 12, 3, True), (128, 20, 1, False)])
def test_f16_storage_and_products_within_1e3(J, N, R, sbd_mfma):
    """The f16 form with its SBD transform in float32 (default) and on the
    matrix cores (frbx_set_sbd_matrix_cores) against the oracle."""
    wl = _wl(J, N, R, seed_id=95 + J, precision="f16")
    wl["search"]["sbd_mfma"] = sbd_mfma
    V, _ = W.generate(wl)
    H = W.to_complex32(V)
    Vq = W.from_complex32(H)          # the stored values, exactly
    import torch
    from paper_1801_02391_amd import frbx
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.load(torch.from_numpy(H).to("cuda:0"))
    s.run()
    P, I = s.power_cube()
    ora = O.search(Vq, wl["layout"], wl["search"])
    err = _check(dict(P=P, I=I), ora, wl["layout"]["n_baselines"], wl["search"]["n_dm"], 1e-3, 4e-3)
    note(f"f16 J={J} N={N} sbd on matrix cores {sbd_mfma}: max power rel err {err:.2e}")


def test_mfma_grid_dump_elementwise():
    """Every cell of one segment's |G|^2 from the f16x3 form against the
    oracle's grid (relative to the grid maximum)."""
    wl = _wl(64, 32, 2, K=120, windows=(3, 8), n_dm=2, seed_id=99)
    V, _ = W.generate(wl)
    g = O.build_grids(wl["layout"], wl["search"])
    out = run_gpu(wl, V)
    s = out["search"]
    cal = np.ones((32, 64))
    for (d, wi, q) in [(0, 0, 0), (1, 1, g["segs"][1][2] - 1)]:
        grid = s.dump_segment(0, d, wi, q)
        l, h, _ = g["segs"][wi]
        rph = O.rate_phasor(g["rates"], g["f0"], l, g["t_ap"])
        Y = O.segment_sums(V[0], g["dk"][d], [q * h], l, rph, cal)
        G = np.abs(O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])[0]) ** 2
        assert np.abs(grid - G).max() / G.max() < 2e-5


def test_f16x3_detections_equal_f32_path():
    """The matrix-core f16x3 form and the float32 vector form give the same
    detections and groups on the short VGOS workload."""
    wl = W.get_workload("vgos-6bl-32x64-2000")
    V, _ = W.generate(wl)
    a = run_gpu(wl, V)
    wl2 = W.get_workload("vgos-6bl-32x64-2000", search=dict(precision="f16x3"))
    b = run_gpu(wl2, V)
    rel = np.abs(a["P"].astype(np.float64) - b["P"]) / a["P"]
    assert rel.max() < 1e-4
    key = lambda d: (d["baseline"], d["dm_index"], d["k0"], d["window_len"])
    assert [key(d) for d in a["candidates"]] == [key(d) for d in b["candidates"]]


@pytest.mark.parametrize("J,N,sbd_mfma", [(64, 32, True), (16, 12, True), (64, 32, False)])
def test_f16_grid_dump_elementwise(J, N, sbd_mfma):
    """Every cell of one segment's |G|^2 from the f16 form (the MBD transform,
    and with sbd_mfma the SBD transform too, on the matrix cores) against the
    oracle's grid on the same stored complex32 values, relative to the grid
    maximum."""
    import torch
    from paper_1801_02391_amd import frbx
    wl = _wl(J, N, 2, K=120, windows=(3, 8), n_dm=2, seed_id=97 + J, precision="f16")
    wl["search"]["sbd_mfma"] = sbd_mfma
    V, _ = W.generate(wl)
    H = W.to_complex32(V)
    Vq = W.from_complex32(H)
    g = O.build_grids(wl["layout"], wl["search"])
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.load(torch.from_numpy(H).to("cuda:0"))
    cal = np.ones((N, J))
    worst = 0.0
    for (d, wi, q) in [(0, 0, 0), (1, 1, g["segs"][1][2] - 1)]:
        grid = s.dump_segment(0, d, wi, q)
        l, h, _ = g["segs"][wi]
        rph = O.rate_phasor(g["rates"], g["f0"], l, g["t_ap"])
        Y = O.segment_sums(Vq[0], g["dk"][d], [q * h], l, rph, cal)
        G = np.abs(O.fringe_matrix(Y, g["e_sbd"], g["e_mbd"])[0]) ** 2
        err = np.abs(grid - G).max() / G.max()
        worst = max(worst, err)
        assert err < 2e-3
    note(f"f16 grid dump J={J} N={N}: max |G|^2 error / max {worst:.2e}")
