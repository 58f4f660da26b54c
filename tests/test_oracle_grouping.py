"""P14: hand-built crossing tables with outcomes derived by hand from
Sec. 2.4.1 (steps b-d, cross matching), Sec. 2.4.2 and Sec. 5.3."""
import numpy as np
import pytest

from oracle import frb_oracle as O


def C(l, k0, p, mbd, **kw):
    d = dict(l=l, k0=k0, p_norm=p, mbd_us=mbd)
    d.update(kw)
    return d


def test_mbd_average_wraps_around_the_ambiguity():
    """Step c: MBDs 0.48, -0.49, 0.45 (period 1) sit together across the
    +-T/2 edge; the circular mean keeps all three windows."""
    cands = [C(8, 10, 4.0, 0.48), C(4, 12, 5.0, -0.49), C(2, 13, 3.5, 0.45)]
    out = O.group_windows(cands, 1.0, 3)
    assert len(out) == 1
    det, members = out[0]
    assert det["n_windows"] == 3 and det["p_norm"] == 5.0 and len(members) == 3


def test_mbd_outlier_removed_and_best_survivor_kept():
    """Step c removes the 0.45 outlier (circular mean 0.0287, |0.421| >= 1/4);
    step d counts windows {8, 4, 2} among survivors and keeps the highest
    normalised power among them (the removed outlier had the highest)."""
    cands = [C(8, 10, 4.0, 0.0), C(4, 12, 4.5, 0.02), C(2, 13, 9.0, 0.45), C(2, 14, 3.2, -0.01)]
    m = O.circular_mean([0.0, 0.02, 0.45, -0.01], 1.0)
    assert m == pytest.approx(0.0287, abs=5e-4)
    out = O.group_windows(cands, 1.0, 3)
    assert len(out) == 1
    det, _ = out[0]
    assert det["n_windows"] == 3
    assert det["p_norm"] == 4.5 and det["l"] == 4


def test_n_win_min_boundary():
    """Step d: exactly N_win,min windows is a detection, one fewer is not."""
    cands = [C(8, 0, 4.0, 0.0), C(4, 2, 4.0, 0.0)]
    assert len(O.group_windows(cands, 1.0, 2)) == 1
    assert len(O.group_windows(cands, 1.0, 3)) == 0


def test_candidate_overlapping_two_groups_joins_the_first():
    """Step b: largest window first; a candidate overlapping members of two
    groups joins the lower-numbered one; groups are never merged."""
    cands = [C(8, 0, 4.0, 0.0),     # group 0: [0, 7]
             C(8, 10, 4.1, 0.0),    # group 1: [10, 17]
             C(4, 6, 4.2, 0.0),     # [6, 9]  -> group 0
             C(4, 8, 4.3, 0.0)]     # [8, 11] overlaps [6, 9] (g0) and [10, 17] (g1) -> g0
    out = O.group_windows(cands, 1.0, 1)
    assert len(out) == 2
    (d0, m0), (d1, m1) = out
    assert sorted(m0) == [0, 2, 3] and m1 == [1]
    assert d0["p_norm"] == 4.3 and d1["p_norm"] == 4.1


def test_insertion_order_is_window_descending():
    """Step b starts with the largest window: a small-window candidate listed
    first still lands in the group the large window opened."""
    cands = [C(2, 5, 3.5, 0.0), C(16, 0, 3.4, 0.0)]
    out = O.group_windows(cands, 1.0, 2)
    assert len(out) == 1
    det, members = out[0]
    assert members == [1, 0] and det["l"] == 2


def test_best_dm_bin_is_kept():
    """Sec. 5.3 coarse search: a pulse seen in several DM bins keeps the bin
    with the highest power; a separate pulse stays separate."""
    dets = [dict(d=3, k0=100, l=4, p_norm=5.0), dict(d=5, k0=101, l=4, p_norm=7.0),
            dict(d=4, k0=300, l=2, p_norm=4.0), dict(d=6, k0=98, l=4, p_norm=6.0)]
    out = O.merge_dm(dets)
    assert len(out) == 2
    assert out[0]["d"] == 5 and out[0]["p_norm"] == 7.0
    assert out[1]["d"] == 4


def test_cross_matching_counts_baselines():
    """Cross matching: overlapping single pulses from two baselines form a
    group with 2 baselines (reported for N_bl,min = 2); a lone pulse on a third
    baseline forms a group that is not reported; two detections of the same
    baseline count once."""
    dets = [dict(b=0, k0=50, l=4, p_norm=5.0), dict(b=1, k0=52, l=2, p_norm=6.0),
            dict(b=0, k0=53, l=2, p_norm=4.0), dict(b=2, k0=400, l=4, p_norm=8.0)]
    groups, assign = O.cross_match(dets, 2)
    assert len(groups) == 2
    assert groups[0]["n_baselines"] == 2 and groups[0]["reported"]
    assert groups[0]["k_start"] == 50 and groups[0]["k_end"] == 54   # [53, 54]
    assert groups[0]["best"] == 1
    assert groups[1]["n_baselines"] == 1 and not groups[1]["reported"]
    assert assign == [0, 0, 0, 1]


def test_power_summation_skips_mbd_filter():
    """Sec. 2.4.2: powers of the baselines are summed per segment, then Eq. 6,
    the threshold and steps b and d; MBD plays no role (step c skipped)."""
    rng = np.random.default_rng(0)
    segs = [(8, 4, 40), (4, 2, 80)]
    rows = []
    for (l, h, Q) in segs:
        per_b = [rng.uniform(1.0, 1.1, Q) for _ in range(2)]
        # a pulse near frame 100 in both windows, split over the two baselines
        per_b[0][100 // h] += 2.0
        per_b[1][100 // h] += 2.0
        rows.append(per_b)
    out = O.power_sum_detect(rows, segs, 1.0, 3.0, 2)
    assert len(out) == 1
    assert out[0]["n_windows"] == 2 and out[0]["k0"] == 100


def test_normalise_and_threshold_strict():
    """Eq. 6 with the population deviation and a strict '>' threshold; a
    constant row (deviation 0) gives no crossings."""
    P = np.array([1.0, 1.0, 1.0, 5.0])
    pn, mu, sd = O.normalise(P)
    assert mu == 2.0 and sd == pytest.approx(np.sqrt(3.0))
    assert list(O.crossings(pn, pn[3] - 1e-12)) == [3]
    assert list(O.crossings(pn, pn[3])) == []
    pn0, _, sd0 = O.normalise(np.ones(5))
    assert pn0 is None and sd0 == 0.0 and len(O.crossings(pn0, 3.0)) == 0
