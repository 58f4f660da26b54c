"""What the reduced-precision storage forms do to the search itself, measured
with the FP64 oracle against the unquantised cross spectra (the GPU searches
the stored values exactly; its parity with the oracle on those values is
tested elsewhere).  FP8 e4m3 keeps 3 mantissa bits, so each stored component
is off by up to 2^-4 of itself and the data by a few per cent rms; the segment
powers are coherent sums over l x N x (J - 1) samples whose quantisation
errors are incoherent, so they move by far less, and the detections stay."""
import numpy as np
import pytest

from oracle import frb_oracle as O
from paper_1801_02391_amd import workloads as W


@pytest.fixture(scope="module")
def searched():
    f0 = [3000.0 + 32.0 * n * (n + 1) / 2 for n in range(6)]
    wl = W.custom_workload(if_freq_mhz=f0, n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=600,
                           n_stations=3, config_id=170,
                           search=dict(dm_lo=0.0, dm_step=100.0, n_dm=2, sbd_pad=4, n_mbd=64, n_rate=1,
                                       windows=[4, 8, 16], threshold=3.0, n_win_min=2, n_bl_min=2),
                           signal=dict(rfi_frac=0.05, rfi_amp=3.0, pulses=dict(kind="fixed", list=[
                               dict(t0_ms=150.0, dm=100.0, width_ms=8.0, snr=6.0, delay_us=0.02),
                               dict(t0_ms=400.0, dm=100.0, width_ms=4.0, snr=8.0, delay_us=-0.05)])))
    V, _ = W.generate(wl)
    c8, sc = W.to_e4m3(V)
    forms = {"c64": V, "e4m3": W.from_e4m3(c8, sc), "c32": W.from_complex32(W.to_complex32(V))}
    return V, forms, {k: O.search(v, wl["layout"], wl["search"]) for k, v in forms.items()}


def _power_rel_err(ref, got):
    return np.concatenate([np.abs(got["cube"][key][0] - P) / P for key, (P, _, _) in ref["cube"].items()])


def _data_rel_rms(V, Vq):
    return float(np.sqrt(np.mean(np.abs(Vq - V) ** 2) / np.mean(np.abs(V) ** 2)))


@pytest.mark.parametrize("form,data_rms,p_median,p_max", [
    ("e4m3", (0.015, 0.04), 0.01, 0.05),
    ("c32", (5e-5, 5e-4), 1e-4, 5e-4),
])
def test_storage_error_in_the_data_and_in_the_powers(searched, form, data_rms, p_median, p_max):
    V, forms, res = searched
    e = _data_rel_rms(V, forms[form])
    assert data_rms[0] < e < data_rms[1]
    rel = _power_rel_err(res["c64"], res[form])
    assert np.median(rel) < p_median and rel.max() < p_max
    # incoherent errors: the powers move by less than the data
    assert np.median(rel) < e / 2


@pytest.mark.parametrize("form", ["e4m3", "c32"])
def test_detections_and_groups_survive_the_storage_form(searched, form):
    _, _, res = searched
    key = lambda d: (d["b"], d["d"], d["l"], d["k0"])
    ref, got = res["c64"]["detections"], res[form]["detections"]
    assert [key(d) for d in got] == [key(d) for d in ref] and len(ref) >= 6
    # the peak cell may move to a neighbour where two cells nearly tie
    M = len(res["c64"]["grids"]["tau_m"])
    for a, b in zip(ref, got):
        assert abs(a["s"] - b["s"]) <= 1 and min((a["m"] - b["m"]) % M, (b["m"] - a["m"]) % M) <= 1
    assert [(g["k_start"], g["k_end"], g["n_baselines"]) for g in res[form]["groups"]] == \
        [(g["k_start"], g["k_end"], g["n_baselines"]) for g in res["c64"]["groups"]]
    # crossings that differ lie near the threshold
    a = {(c["b"], c["d"], c["wi"], c["q"]): c["p_norm"] for c in res["c64"]["crossings"]}
    b = {(c["b"], c["d"], c["wi"], c["q"]): c["p_norm"] for c in res[form]["crossings"]}
    for k in set(a) ^ set(b):
        assert abs(a.get(k, b.get(k)) - 3.0) < 0.1
