"""CPU tests of the C-ABI library: it loads, exports every entry point the
header declares, and its host-only logic (Eq. 2 table, the Sec. 2.4.1 /
Sec. 5.3 grouping, argument validation) agrees with the oracle.  No device
compute is called here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import frb_oracle as O
from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_names():
    src = open(os.path.join(ROOT, "include", "frbx.h")).read()
    return sorted(set(re.findall(r"\b(frbx_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = frbx.lib()
    names = _header_names()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(frbx.exported_names())
    assert frbx.version().startswith("frbx")


@pytest.mark.parametrize("name", ["single-1bl-8x32-1000", "vgos-6bl-32x64-20000",
                                  "paper-3bl-6x32-19531"])
def test_ap_offset_table_matches_oracle(name):
    wl = W.get_workload(name)
    lay, s = wl["layout"], wl["search"]
    lib_tab = frbx.ap_offsets(lay, s["dm_lo"], s["dm_step"], s["n_dm"], s["k_dm"])
    ora = O.ap_offsets(O.dm_trials(s["dm_lo"], s["dm_step"], s["n_dm"]), lay["if_freq_mhz"],
                       lay["n_chan"], lay["chan_bw_mhz"], lay["t_ap_ms"], s["k_dm"])
    assert np.array_equal(lib_tab, ora)


def test_ap_offset_table_k_dm_variant():
    """k_dm = 4.15e6 (the constant printed in Eq. 1) is selectable."""
    lay = W.get_workload("single-1bl-8x32-1000")["layout"]
    a = frbx.ap_offsets(lay, 0.0, 40.0, 8, 4.15e6)
    b = O.ap_offsets(O.dm_trials(0.0, 40.0, 8), lay["if_freq_mhz"], 32, 1.0, 1.0, 4.15e6)
    assert np.array_equal(a, b)


def _random_crossings(rng, n_b, n_d, windows, n, t_amb):
    out = []
    for _ in range(n):
        wi = int(rng.integers(len(windows)))
        l = windows[wi]
        h = max(1, l // 2)
        q = int(rng.integers(0, 60))
        out.append(dict(baseline=int(rng.integers(n_b)), dm_index=int(rng.integers(n_d)),
                        window_index=wi, window_len=l, segment=q, k0=q * h,
                        power_norm=float(rng.uniform(3.0, 9.0)),
                        mbd_us=float(rng.uniform(-t_amb / 2, t_amb / 2)) * (0.3 if rng.random() < 0.7 else 1.0)))
    return out


def _oracle_detect(cross, t_amb, n_win_min, n_bl_min):
    oc = [dict(b=c["baseline"], d=c["dm_index"], l=c["window_len"], k0=c["k0"],
               p_norm=c["power_norm"], mbd_us=c["mbd_us"], key=i) for i, c in enumerate(cross)]
    dets, groups, assign = O.detect(oc, t_amb, n_win_min, n_bl_min)
    return dets, groups, assign


@pytest.mark.parametrize("seed", range(12))
def test_grouping_matches_oracle_on_random_tables(seed):
    """Steps b-d, best-DM merge and cross matching: the library's host code
    and the oracle agree record for record on random crossing tables."""
    rng = np.random.default_rng(seed)
    t_amb = 0.03125
    windows = [2, 4, 8, 16]
    cross = _random_crossings(rng, 3, 4, windows, int(rng.integers(5, 120)), t_amb)
    for k, c in enumerate(cross):
        c["key"] = k
    n_win_min, n_bl_min = int(rng.integers(1, 4)), int(rng.integers(1, 3))
    dets, groups = frbx.detect(cross, t_amb, n_win_min, n_bl_min)
    odets, ogroups, oassign = _oracle_detect(cross, t_amb, n_win_min, n_bl_min)
    assert len(dets) == len(odets)
    for d, o in zip(dets, odets):
        assert (d["baseline"], d["dm_index"], d["k0"], d["window_len"]) == (o["b"], o["d"], o["k0"], o["l"])
        assert d["power_norm"] == o["p_norm"]
        assert d["n_windows"] == o["n_windows"]
    assert len(groups) == len(ogroups)
    for g, o in zip(groups, ogroups):
        assert g["n_baselines"] == o["n_baselines"]
        assert (g["k_start"], g["k_end"]) == (o["k_start"], o["k_end"])
        assert g["best"] == o["best"]
        assert bool(g["reported"]) == o["reported"]
    assert [d["group_id"] for d in dets] == oassign


def test_grouping_hand_built_wrap_and_outlier():
    """The library reproduces the hand-derived P14 cases: MBD wrap across the
    ambiguity edge keeps all windows; an outlier is removed by step c."""
    mk = lambda l, k0, p, m: dict(baseline=0, dm_index=0, window_len=l, k0=k0, power_norm=p, mbd_us=m)
    dets, _ = frbx.detect([mk(8, 10, 4.0, 0.48), mk(4, 12, 5.0, -0.49), mk(2, 13, 3.5, 0.45)], 1.0, 3, 1)
    assert len(dets) == 1 and dets[0]["n_windows"] == 3 and dets[0]["power_norm"] == 5.0
    dets, _ = frbx.detect([mk(8, 10, 4.0, 0.0), mk(4, 12, 4.5, 0.02), mk(2, 13, 9.0, 0.45),
                           mk(2, 14, 3.2, -0.01)], 1.0, 3, 1)
    assert len(dets) == 1 and dets[0]["power_norm"] == 4.5 and dets[0]["window_len"] == 4
    # power-summation form: step c skipped, the outlier is the best member
    dets, _ = frbx.detect([mk(8, 10, 4.0, 0.0), mk(4, 12, 4.5, 0.02), mk(2, 13, 9.0, 0.45)],
                          1.0, 3, 1, use_mbd=False)
    assert len(dets) == 1 and dets[0]["power_norm"] == 9.0


def test_invalid_arguments_are_rejected_without_a_device():
    L = frbx.lib()
    f0 = np.array([3000.0, 3032.0])
    bad = frbx.Layout(1, 2, 48, 100, 1.0, 1.0, f0.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    assert L.frbx_create(C.byref(bad), 0, None, C.byref(h)) == frbx.E_INVAL  # J = 48
    bad2 = frbx.Layout(1, 2, 32, 100, -1.0, 1.0, f0.ctypes.data_as(C.POINTER(C.c_double)))
    assert L.frbx_create(C.byref(bad2), 0, None, C.byref(h)) == frbx.E_INVAL
    assert L.frbx_create(None, 0, None, C.byref(h)) == frbx.E_INVAL
    out = np.zeros(10, dtype=np.int32)
    assert L.frbx_ap_offsets(C.byref(bad), 0.0, 1.0, 1, 0.0, out.ctypes.data_as(C.c_void_p)) == frbx.E_INVAL
    # the getters refuse a NULL context
    n = C.c_int64(0)
    assert L.frbx_get_candidates(None, None, 0, C.byref(n)) == frbx.E_INVAL
    assert L.frbx_run(None) == frbx.E_INVAL
    assert L.frbx_get_lattice(None, None, None, None) == frbx.E_INVAL
    assert L.frbx_set_recheck(None, 0.05) == frbx.E_INVAL
    assert L.frbx_get_recheck(None, None, None) == frbx.E_INVAL
    # the refinement entry points refuse a NULL context
    assert L.frbx_top_peaks(None, 5, None, 0, C.byref(n)) == frbx.E_INVAL
    assert L.frbx_refine_begin(None, None, 0, None) == frbx.E_INVAL
    assert L.frbx_refine_run(None, 3) == frbx.E_INVAL
    assert L.frbx_refine_forward(None, None, None) == frbx.E_INVAL
    assert L.frbx_refine_backward(None, None, None, None) == frbx.E_INVAL
    assert L.frbx_refine_curvature(None, None, None) == frbx.E_INVAL
    assert L.frbx_refine_results(None, None, None, 0, C.byref(n)) == frbx.E_INVAL
    # detect validates its arguments
    assert L.frbx_detect(None, 3, 1.0, 1, 1, 1, None, 0, None, None, 0, None) == frbx.E_INVAL
    assert L.frbx_detect(None, 0, -1.0, 1, 1, 1, None, 0, None, None, 0, None) == frbx.E_INVAL


def test_detect_capacity_protocol():
    """cap = 0 is a size query: E_RANGE with the size needed."""
    L = frbx.lib()
    arr = (frbx.Candidate * 2)()
    for i in range(2):
        arr[i].baseline = i
        arr[i].window_len = 4
        arr[i].k0 = 10
        arr[i].power_norm = 5.0
    nd, ng = C.c_int64(-1), C.c_int64(-1)
    s = L.frbx_detect(arr, 2, 1.0, 1, 2, 1, None, 0, C.byref(nd), None, 0, C.byref(ng))
    assert s == frbx.E_RANGE and nd.value == 2 and ng.value == 1


def _lattice_rule(f0, n_mbd, t_amb):
    """Independent statement of the lattice and of the compact-form rule:
    q_n = (f_n - f_0) T mod M; the one-pass form applies when a shift by one
    IF's position brings every position below the first pass's row count
    (4, 4, 8, 8, 16 rows for M = 16 ... 256), the first such IF (in IF
    order) giving the shift."""
    q = [int(round((f - f0[0]) * t_amb)) % n_mbd for f in f0]
    rows = {16: 4, 32: 4, 64: 8, 128: 8, 256: 16}[n_mbd]
    shift = next((s for s in q if max((x - s) % n_mbd for x in q) < rows), -1)
    return q, shift


@pytest.mark.parametrize("name", W.workload_names())
def test_mbd_lattice_of_the_workloads(name):
    wl = W.get_workload(name)
    lay, srch = wl["layout"], wl["search"]
    t_amb = O.build_grids(lay, srch)["t_amb"]
    got = frbx.mbd_lattice(lay, srch["n_mbd"])
    q, shift = _lattice_rule(lay["if_freq_mhz"], srch["n_mbd"], t_amb)
    assert got["q"] == q and got["compact_shift"] == shift
    assert got["mbd_step_us"] == pytest.approx(t_amb / srch["n_mbd"], rel=1e-12)


def test_mbd_lattice_random_sets_and_edges():
    rng = np.random.default_rng(11)
    for trial in range(200):
        M = int(rng.choice([16, 32, 64, 128, 256]))
        span = int(rng.choice([4, 8, 16, 17, M]))
        N = int(rng.integers(1, min(M, 12, 2 * span) + 1))
        pts = rng.choice(np.arange(-span, span), size=N, replace=False)
        pts = pts - pts[0]                        # IF 0 at offset 0
        if len(set(int(p) % M for p in pts)) < N:
            continue
        f0 = [8000.0 + 16.0 * int(p) for p in pts]   # offsets >= -2M x 16 MHz stay positive
        lay = dict(n_baselines=1, if_freq_mhz=f0, n_chan=16, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=64)
        got = frbx.mbd_lattice(lay, M)
        nz = [int(p) for p in pts if p != 0]
        g_mhz = float(np.gcd.reduce(np.abs(nz))) * 16.0 if nz else None
        t_amb = 1.0 / g_mhz if g_mhz else 1.0 / (16 * 1.0)
        q, shift = _lattice_rule(f0, M, t_amb)
        assert got["q"] == q and got["compact_shift"] == shift, (M, f0)
    # refused: two IFs on one lattice point (offsets 0 and 16 x 16 MHz at M = 16),
    # and an unsupported number of MBD points
    lay = dict(n_baselines=1, if_freq_mhz=[3000.0, 3016.0, 3256.0], n_chan=16, chan_bw_mhz=1.0,
               t_ap_ms=1.0, n_frames=64)
    with pytest.raises(frbx.FrbxError):
        frbx.mbd_lattice(lay, 16)
    assert frbx.mbd_lattice(lay, 32)["compact_shift"] == -1     # q = 0, 1, 16: span 16 > 4 rows
    with pytest.raises(frbx.FrbxError):
        frbx.mbd_lattice(lay, 100)
