"""The float32 fringe kernel compiled at run time for the IF lattice (hipRTC:
only the rows of its first MBD pass that hold an IF are read and
transformed) against the statically built kernel on the same data.  The
two are separate compilations of one source, so the compiler may fuse a
multiply and an add differently: the powers agree to float32 rounding
(4e-6 relative), the peak cells, Eq. 6 statistics (to 1e-6), crossings
(apart from marginal ones) and detections are the same.  Lattices: the VGOS
band set (32 IFs on 5 of 16 rows), three IFs spread over two rows at M =
256 and at M = 64, and two lattices for which the static kernel stays in use
(every row holds an IF; compact), where the results are identical."""
import numpy as np
import pytest
import torch

from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

from gpu_helpers import MARGINAL, note

pytestmark = pytest.mark.gpu

# rows of the first MBD pass per lattice size (the kernel's radix split)
ROWS_A = {16: 4, 32: 8, 64: 8, 128: 16, 256: 16}


def expected_rows(q, M):
    mb = M // ROWS_A[M]
    rows = 0
    for x in q:
        rows |= 1 << (int(x) // mb)
    full = (1 << ROWS_A[M]) - 1
    return 0 if rows == full else rows


def _custom(f0, M, n_chan=32, n_frames=600, config_id=81):
    return W.custom_workload(
        if_freq_mhz=f0, n_chan=n_chan, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=n_frames,
        n_stations=3, config_id=config_id,
        search=dict(dm_lo=0.0, dm_step=100.0, n_dm=4, sbd_pad=4, n_mbd=M, n_rate=3,
                    windows=[2, 4, 8], threshold=3.0, n_win_min=2, n_bl_min=2),
        signal=dict(pulses=dict(kind="fixed", list=[
            dict(t0_ms=300.0, dm=200.0, width_ms=4.0, snr=20.0, delay_us=0.004)])))


def _vgos():
    return W.get_workload("vgos-6bl-32x64-2000")


CASES = {
    "vgos-32if-5rows": (_vgos, True),
    "3if-2rows-m256": (lambda: _custom([3000.0, 3032.0, 5240.0], 256), True),
    "3if-2rows-m64": (lambda: _custom([3000.0, 3032.0, 4120.0], 64, config_id=82), True),
    "4if-all-rows-m16": (lambda: _custom([3000.0, 3128.0, 3288.0, 3448.0], 16, config_id=83), False),
    "8if-compact": (lambda: _custom([3000.0 + 32.0 * n for n in range(8)], 256, config_id=84), False),
}


def _run(wl, Vt, spec):
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.set_specialisation(spec)
    s.load(Vt)
    s.run()
    P, I = s.power_cube()
    mean, sd, cnt = s.stats()
    return s, dict(P=P, I=I, mean=mean, sd=sd, cnt=cnt, cross=s.crossings(), cand=s.candidates())


@pytest.mark.parametrize("case", list(CASES))
def test_specialised_kernel_matches_the_static_kernel(case):
    make, specialised = CASES[case]
    wl = make()
    V, _ = W.generate(wl)
    Vt = torch.from_numpy(V).to("cuda:0")
    s1, a = _run(wl, Vt, True)
    s0, b = _run(wl, Vt, False)
    lat = s1.lattice()
    rows, why = s1.specialisation()
    want = expected_rows(lat["q"], wl["search"]["n_mbd"]) if lat["compact_shift"] < 0 else 0
    note(f"{case}: lattice q {lat['q'][:8]}.. compact shift {lat['compact_shift']}, rows {rows:#x} ({why!r})")
    assert why == ""
    assert rows == want and (rows != 0) == specialised
    assert s0.specialisation() == (0, "")
    d = np.abs(a["P"].astype(np.float64) - b["P"]) / np.maximum(b["P"], 1e-30)
    n_idx = int(np.sum(a["I"] != b["I"]))
    note(f"{case}: {int(np.sum(a['P'] != b['P']))} of {a['P'].size} powers differ, max rel {d.max():.3g}; "
         f"{n_idx} indices differ")
    if not specialised:
        for k in ("P", "I", "mean", "sd", "cnt"):
            assert np.array_equal(a[k], b[k]), k
    assert d.max() <= 4e-6
    assert n_idx <= 1e-4 * a["I"].size
    assert np.array_equal(a["cnt"], b["cnt"])
    assert np.allclose(a["mean"], b["mean"], rtol=1e-6) and np.allclose(a["sd"], b["sd"], rtol=1e-6)
    key = lambda c: (c["baseline"], c["dm_index"], c["window_index"], c["segment"])
    ca, cb = {key(c): c for c in a["cross"]}, {key(c): c for c in b["cross"]}
    thr = wl["search"]["threshold"]
    for k in set(ca) ^ set(cb):
        c = ca.get(k) or cb.get(k)
        assert abs(c["power_norm"] - thr) <= MARGINAL * max(1.0, thr), k
    same = [k for k in ca if k in cb]
    assert all((ca[k]["rate_idx"], ca[k]["sbd_idx"], ca[k]["mbd_idx"]) ==
               (cb[k]["rate_idx"], cb[k]["sbd_idx"], cb[k]["mbd_idx"]) for k in same)
    ck = lambda c: (c["baseline"], c["dm_index"], c["window_len"], c["k0"], c["n_windows"])
    assert sorted(map(ck, a["cand"])) == sorted(map(ck, b["cand"]))
    assert len(a["cross"]) > 0


def test_specialisation_follows_the_precision():
    """The matrix-core forms keep their own kernels (row set 0); switching
    back to float32 on the same context builds the specialised one again."""
    wl = _vgos()
    wl["layout"]["n_baselines"] = 1
    wl["layout"]["stations"] = wl["layout"]["stations"][:1]
    V, _ = W.generate(wl, baselines=[0])
    Vt = torch.from_numpy(V).to("cuda:0")
    s = frbx.Search(wl["layout"])
    s.configure(dict(wl["search"], precision="f16x3"))
    s.load(Vt)
    s.run()
    assert s.specialisation()[0] == 0
    s.configure(dict(wl["search"], precision="f32"))
    s.load(Vt)
    s.run()
    assert s.specialisation()[0] == expected_rows(s.lattice()["q"], 256) != 0
