"""GPU parity at the benchmark's full size: the VGOS workload (6 baselines,
32 IFs x 64 channels, 20000 APs, 256 DM trials, 8 rates, 256 x 256 delay
cells) searched exactly as bench.py times it, checked on sampled outputs
that the FP64 oracle computes segment by segment: powers and peak indices
of sampled cube entries (random ones and the strongest crossings) in all
three forms, the Eq. 6 statistics against the device's own cube, the f16
form with float32 re-evaluation against the f32 detections, and the
refinement of the top 1024 peaks against the oracle's gradient and central
differences."""
import numpy as np
import pytest
import torch

from oracle import frb_oracle as O
from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

from gpu_helpers import MARGIN, POWER_RTOL, note

pytestmark = pytest.mark.gpu

NAME = "vgos-6bl-32x64-20000"


@pytest.fixture(scope="module")
def vgos():
    wl = W.get_workload(NAME)
    note("generating the full VGOS workload")
    V, truth = W.generate(wl)
    return wl, V


def _run(wl, V, prec, band=0.0):
    s = frbx.Search(wl["layout"])
    s.configure(dict(wl["search"], precision=prec, recheck_band=band))
    s.load(torch.from_numpy(W.to_complex32(V) if prec == "f16" else V).cuda())
    note(f"full search, {prec}, recheck band {band}")
    s.run()
    return s


@pytest.fixture(scope="module")
def f32_search(vgos):
    wl, V = vgos
    return _run(wl, V, "f32")


def _samples(s, wl, n_random=40, n_top=16, seed=3):
    seg = s.segments()
    B, D = wl["layout"]["n_baselines"], wl["search"]["n_dm"]
    off = np.cumsum([0] + seg["n_seg"])
    rng = np.random.default_rng(seed)
    out = set()
    for _ in range(n_random):
        b, d, w = int(rng.integers(B)), int(rng.integers(D)), int(rng.integers(len(seg["n_seg"])))
        out.add((b, d, w, int(rng.integers(seg["n_seg"][w]))))
    for p in s.top_peaks(n_top):
        out.add((p["baseline"], p["dm_index"], p["window_index"], p["segment"]))
    return sorted(out), off


def _oracle_entries(wl, V, entries):
    g = O.build_grids(wl["layout"], wl["search"])
    N, J = wl["layout"]["n_if"], wl["layout"]["n_chan"]
    cal = np.ones((N, J))
    res = {}
    for (b, d, w, q) in entries:
        P, I, S2 = O.search_row(V[b].astype(np.complex128), g, cal, d, w, q_list=[q])
        res[(b, d, w, q)] = (P[0], I[0], S2[0])
    return res


def _check(P, I, off, ora, rtol, margin):
    worst, n_idx = 0.0, 0
    for (b, d, w, q), (po, io, s2) in ora.items():
        pg, ig = float(P[b, d, off[w] + q]), int(I[b, d, off[w] + q])
        rel = abs(pg - po) / po
        worst = max(worst, rel)
        assert rel <= rtol, ((b, d, w, q), pg, po)
        if (po - s2) / po > margin:
            n_idx += 1
            assert ig == io, ((b, d, w, q), ig, io)
    return worst, n_idx


def test_full_size_f32_sampled_against_the_oracle(vgos, f32_search):
    wl, V = vgos
    s = f32_search
    entries, off = _samples(s, wl)
    ora = _oracle_entries(wl, V, entries)
    P, I = s.power_cube()
    worst, n_idx = _check(P, I, off, ora, POWER_RTOL, MARGIN)
    note(f"f32: {len(entries)} sampled segments, worst power rel err {worst:.2e}, {n_idx} index checks")
    assert n_idx >= len(entries) // 2
    # Eq. 6 statistics of sampled rows = FP64 normalisation of the device's own cube rows
    mean, sd, cnt = s.stats()
    nw = len(off) - 1
    D = wl["search"]["n_dm"]
    for (b, d, w, q) in entries[:20]:
        row = P[b, d, off[w]:off[w + 1]]
        _, mu, sdv = O.normalise(row)
        r = (b * D + d) * nw + w
        assert mean[r] == pytest.approx(mu, rel=1e-9) and sd[r] == pytest.approx(sdv, rel=1e-7)
        assert cnt[r] == off[w + 1] - off[w]


@pytest.mark.parametrize("prec", ["f16x3", "f16"])
def test_full_size_matrix_core_forms_sampled(vgos, prec):
    wl, V = vgos
    s = _run(wl, V, prec)
    entries, off = _samples(s, wl, n_random=24, n_top=8, seed=5)
    Vo = W.from_complex32(W.to_complex32(V)) if prec == "f16" else V
    ora = _oracle_entries(wl, Vo, entries)
    P, I = s.power_cube()
    rtol, margin = (POWER_RTOL, MARGIN) if prec == "f16x3" else (1e-3, 4e-3)
    worst, n_idx = _check(P, I, off, ora, rtol, margin)
    note(f"{prec}: {len(entries)} sampled segments, worst power rel err {worst:.2e}, {n_idx} index checks")


def test_full_size_f16_with_recheck_detects_as_float32(vgos, f32_search):
    """f16 with every segment above threshold - 0.05 re-evaluated in f32:
    the detections equal the f32 search's, and every crossing that differs
    lies within 1e-3 x threshold of it."""
    wl, V = vgos
    s = _run(wl, V, "f16", band=0.05)
    band, n = s.recheck()
    note(f"f16 + recheck: {n} segments re-evaluated")
    assert band == 0.05 and n > 0

    def det(cands):
        return [(c["baseline"], c["dm_index"], c["window_len"], c["k0"]) for c in cands]
    assert det(s.candidates()) == det(f32_search.candidates())
    thr = wl["search"]["threshold"]
    key = lambda c: (c["baseline"], c["dm_index"], c["window_index"], c["segment"])
    a = {key(c): c["power_norm"] for c in s.crossings()}
    b = {key(c): c["power_norm"] for c in f32_search.crossings()}
    for k in set(a) ^ set(b):
        assert abs(a.get(k, b.get(k)) - thr) <= 1e-3 * thr


def test_full_size_refinement_of_the_top_1024_peaks(vgos, f32_search):
    wl, V = vgos
    s = f32_search
    peaks = s.top_peaks(1024)
    assert len(peaks) == 1024
    th0 = s.refine_begin(peaks)
    cells, _ = s.refine_cells()
    tt = torch.tensor(th0, dtype=torch.float64, device="cuda")
    P = s.refine_forward(tt).cpu().numpy()
    g = s.refine_backward(tt, torch.ones(1024, dtype=torch.float32, device="cuda")).cpu().numpy()
    lay, srch = wl["layout"], wl["search"]
    N, J = lay["n_if"], lay["n_chan"]
    cal = np.ones((N, J), complex)
    worst_p = worst_g = worst_fd = 0.0
    for i in range(0, 1024, 64):
        p = peaks[i]
        Vb = V[p["baseline"]].astype(np.complex128)
        f = lambda th: O.relaxed_power_grad(*O.relaxed_fringe(Vb, lay, srch, cal, p["k0"], p["window_len"], th)[:2])
        Po, go = f(th0[i])
        worst_p = max(worst_p, abs(P[i] - Po) / Po)
        assert P[i] == pytest.approx(Po, rel=2e-5)
        for k in range(5):
            if cells[k] == 0:
                continue
            gs = Po / cells[k]
            worst_g = max(worst_g, abs(g[i, k] - go[k]) / (abs(go[k]) + gs))
            assert abs(g[i, k] - go[k]) <= 2e-4 * (abs(go[k]) + gs)
            h = 1e-3 * cells[k]
            e = np.zeros(5)
            e[k] = h
            fd = (f(th0[i] + e)[0] - f(th0[i] - e)[0]) / (2 * h)
            r = abs(g[i, k] - fd) / max(abs(fd), 1e-2 * gs)
            worst_fd = max(worst_fd, r)
            assert r <= 1e-3
    note(f"refinement: P rel {worst_p:.1e}, gradient vs oracle {worst_g:.1e}, vs FD {worst_fd:.1e}")
    th0b, th, Pf = s.refine(peaks, steps=20)
    gain = Pf / P
    note(f"refinement power gain: median {np.median(gain):.4f}, min {gain.min():.4f}, "
         f"share not below the start {np.mean(gain >= 1 - 1e-6):.3f}")
    assert np.median(gain) > 1.0 and np.mean(gain >= 1 - 1e-6) >= 0.99 and gain.min() > 0.9
