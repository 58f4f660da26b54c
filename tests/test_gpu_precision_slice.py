"""The precision workload's shape on a reduced slice: one baseline (the
third, whose pulse near AP 33392 the float32 search reports at DM trial 14
and the matrix-core forms at another trial of equal power), 4096 APs around
that pulse and the first 32 DM trials (step 6.25), 32 IFs x 128 channels, 8
rates, PJ = 512, M = 256.  f16x3 on the complex64 data and f16 with float32
re-evaluation on its complex32 form against the float32 search: crossings
the same apart from marginal ones; single-pulse detections the same outside
the marginal regions of either side (Sec. 2.4.1 / 5.3 decisions within
1e-3 x threshold of going the other way)."""
import numpy as np
import pytest
import torch

from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

from gpu_helpers import MARGINAL, compare_detections, marginal_regions, note

pytestmark = pytest.mark.gpu

K0, K = 31300, 4096


def _as_oracle_keys(cross):
    return [dict(b=c["baseline"], d=c["dm_index"], l=c["window_len"], k0=c["k0"],
                 p_norm=c["power_norm"], mbd_us=c["mbd_us"]) for c in cross]


@pytest.fixture(scope="module")
def runs():
    wl = W.get_workload("precision-21bl-32x128-40000")
    V, _ = W.generate(wl, baselines=[2])
    V = np.ascontiguousarray(V[..., K0:K0 + K])
    lay = dict(wl["layout"], n_baselines=1, stations=[wl["layout"]["stations"][2]], n_frames=K)
    srch = dict(wl["search"], n_dm=32)
    out = {}
    for form, prec, band in (("f32", "f32", 0.0), ("f16x3", "f16x3", 0.0), ("f16-recheck", "f16", 0.05)):
        data = W.to_complex32(V) if prec == "f16" else V
        s = frbx.Search(lay)
        s.configure(dict(srch, precision=prec, recheck_band=band))
        s.load(torch.from_numpy(data).to("cuda:0"))
        s.run()
        out[form] = dict(cross=s.crossings(), cand=s.candidates(), P=s.power_cube()[0],
                         t_amb=s.lattice()["mbd_step_us"] * srch["n_mbd"])
        note(f"slice {form}: {len(out[form]['cross'])} crossings, {len(out[form]['cand'])} detections")
    return srch, out


@pytest.mark.parametrize("form", ["f16x3", "f16-recheck"])
def test_slice_candidates_equal_outside_marginal_decisions(runs, form):
    srch, out = runs
    thr = srch["threshold"]
    a, b = out["f32"], out[form]
    key = lambda c: (c["baseline"], c["dm_index"], c["window_index"], c["segment"])
    ca, cb = {key(c): c for c in a["cross"]}, {key(c): c for c in b["cross"]}
    tol = MARGINAL * max(1.0, thr)
    for k in set(ca) ^ set(cb):
        c = ca.get(k) or cb.get(k)
        assert abs(c["power_norm"] - thr) <= tol, f"non-marginal crossing in one form only: {k}"
    diffs = [abs(ca[k]["power_norm"] - cb[k]["power_norm"]) for k in ca if k in cb]
    assert max(diffs) <= (1e-4 if form == "f16x3" else 5e-3)
    regions = {}
    for side in (a, b):
        for bb, iv in marginal_regions(_as_oracle_keys(side["cross"]), a["t_amb"], thr,
                                       srch["n_win_min"]).items():
            regions.setdefault(bb, []).extend(iv)
    da = [dict(b=c["baseline"], d=c["dm_index"], l=c["window_len"], k0=c["k0"]) for c in a["cand"]]
    db = [dict(b=c["baseline"], d=c["dm_index"], l=c["window_len"], k0=c["k0"]) for c in b["cand"]]
    n_aside = compare_detections(da, db, regions)
    note(f"slice {form}: {len(set(ca) ^ set(cb))} marginal crossings, max |dP_norm| {max(diffs):.2e}; "
         f"{len(da)} / {len(db)} detections, {n_aside} in marginal regions")
    assert len(da) > 0 and n_aside < len(da) + len(db)
