"""Shared helpers of the GPU parity tests: run the HIP search through the C
ABI and the FP64 oracle on the same seeded inputs, and compare them to the
bar of the search (powers within 1e-4 relative, peak indices exact where the
oracle's peak margin exceeds 1e-3, identical crossings apart from marginal
ones, identical grouping)."""
import sys

import numpy as np

from oracle import frb_oracle as O

POWER_RTOL = 1e-4     # FP32 path vs FP64 oracle, relative, on |G|
MARGIN = 1e-3         # index parity required where (best - second)/best > MARGIN
MARGINAL = 1e-3       # a crossing is marginal if |P_norm - thr| <= MARGINAL * max(1, thr)


def note(msg):
    sys.stderr.write(f"[gpu-test] {msg}\n")
    sys.stderr.flush()


def run_gpu(wl, V, tau0=None, phi0=None, device=0):
    import torch
    from paper_1801_02391_amd import frbx
    lay = wl["layout"]
    s = frbx.Search(lay, device=device)
    s.configure(wl["search"], tau0, phi0)
    Vt = torch.from_numpy(np.ascontiguousarray(V)).to(f"cuda:{device}")
    s.load(Vt)
    note(f"run {wl.get('name')} B={lay['n_baselines']} N={lay['n_if']} J={lay['n_chan']} "
         f"K={lay['n_frames']} D={wl['search']['n_dm']} R={wl['search']['n_rate']} "
         f"M={wl['search']['n_mbd']} P={wl['search']['sbd_pad']} W={wl['search']['windows']}")
    s.run()
    P, I = s.power_cube()
    mean, sd, cnt = s.stats()
    out = dict(search=s, P=P, I=I, mean=mean, sd=sd, cnt=cnt, seg=s.segments(),
               crossings=s.crossings(), candidates=s.candidates(), groups=s.groups(), V=Vt)
    return out


def oracle_cube(res, B, D, segs):
    S = sum(q for (_, _, q) in segs)
    P = np.zeros((B, D, S))
    I = np.zeros((B, D, S), dtype=np.int64)
    S2 = np.zeros((B, D, S))
    off = np.cumsum([0] + [q for (_, _, q) in segs])
    for (b, d, wi), (p, i, s2) in res["cube"].items():
        P[b, d, off[wi]:off[wi + 1]] = p
        I[b, d, off[wi]:off[wi + 1]] = i
        S2[b, d, off[wi]:off[wi + 1]] = s2
    return P, I, S2


def compare_powers(Pg, Ig, Po, Io, S2o, where=""):
    """Powers within POWER_RTOL; indices equal where the margin is large.
    Returns the number of index comparisons made."""
    Pg = np.asarray(Pg, dtype=np.float64)
    rel = np.abs(Pg - Po) / np.maximum(np.abs(Po), 1e-30)
    worst = np.unravel_index(np.argmax(rel), rel.shape) if rel.size else None
    assert rel.size == 0 or rel.max() <= POWER_RTOL, f"{where}: power rel err {rel.max():.3g} at {worst}"
    margin = (Po - S2o) / np.maximum(Po, 1e-30)
    sel = margin > MARGIN
    bad = np.nonzero(sel & (Ig != Io))
    assert len(bad[0]) == 0, f"{where}: {len(bad[0])} index mismatches, first at {[x[0] for x in bad]}"
    return int(sel.sum())


def compare_crossings(gpu_cross, ora_cross, thr):
    """Same crossings except marginal ones (|P_norm - thr| small on either
    side); the normalised powers of common ones agree to 1e-3."""
    def key(c, b="baseline", d="dm_index", w="window_index", q="segment"):
        return (c[b], c[d], c[w], c[q])
    g = {key(c): c for c in gpu_cross}
    o = {(c["b"], c["d"], c["wi"], c["q"]): c for c in ora_cross}
    tol = MARGINAL * max(1.0, thr)
    n_marg = 0
    for k in set(g) ^ set(o):
        pn = g[k]["power_norm"] if k in g else o[k]["p_norm"]
        assert abs(pn - thr) <= tol, f"non-marginal crossing only on one side: {k} pnorm {pn}"
        n_marg += 1
    for k in set(g) & set(o):
        assert abs(g[k]["power_norm"] - o[k]["p_norm"]) <= 1e-3, k
    return n_marg
