"""Benchmark of the cross-spectrum FRB search on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step is one full search (frbx_run): dedispersion over every DM trial,
fringe search of every segment of every window and rate bin, Eq. 6
statistics and threshold, multi-window filter, best-DM merge and
cross-baseline matching, with the cross spectra already resident in HBM.
Prints one JSON line.  The metric is search cells per second, a cell being
one evaluated |G| at (baseline, DM trial, window, segment, rate, SBD, MBD).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

T_START = time.perf_counter()   # the wall-clock budget counts from here

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (packed), published
# without packed FP32 (kept out of every device code object): 256 CU x 4 SIMD
# x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_FP16_MFMA_TFLOPS = 2500.0  # MI355X dense FP16 matrix, published
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, published
# channel counts for which the f16 form runs its SBD transform on the matrix
# cores as well (the library's fringe_gemm_kernel)
SBD_GEMM_CHANNELS = (16, 32, 64)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_vgos_6bl_20000.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1801_02391_amd", "csrc", f)
                  for f in ("frbx_kernels.hip", "frbx_fringe.h")]


def kernel_code_sha256():
    """SHA-256 of the kernel sources without their // comments and blank
    lines: a change of code (not of commentary) invalidates measured
    counters."""
    import hashlib
    lines = []
    for path in KERNEL_SOURCES:
        for line in open(path):
            code = line.split("//", 1)[0].rstrip()
            if code:
                lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def measured_traffic(key, workload):
    """HBM bytes per launch of a kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary in profiles/ (calibrated against a plain copy), or None
    when there is none for this workload or the kernel source has changed
    since the counters were taken."""
    import hashlib
    if workload != "vgos-6bl-32x64-20000" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = (x.strip() for x in line.split("=", 1))
            vals[k] = v
    sha = kernel_code_sha256()
    if vals.get("kernels_sha256") != sha or key not in vals:
        return None
    return float(vals[key])


def mbd_one_pass_rows(s, M):
    """Rows of the one-pass MBD form when the float32 search runs it (compact
    IF lattice), else 0 (the general two-pass form)."""
    if s.lattice()["compact_shift"] < 0:
        return 0
    return {16: 4, 32: 4, 64: 8, 128: 8, 256: 16}[M]


def mbd_form(rows, s=None):
    if not rows:
        spec = s.specialisation()[0] if s is not None else 0
        if spec:
            return {"mbd_form": f"two-pass, first pass on {bin(spec).count('1')} rows "
                                f"(row set {spec:#x}, kernel compiled for the IF lattice)"}
        return {"mbd_form": "two-pass"}
    return {"mbd_form": f"one-pass (compact IF lattice, {rows} rows)",
            "note": "achieved counts the work of the one-pass form (the first MBD pass is skipped)"}


def log(msg):
    sys.stderr.write(f"[bench {time.perf_counter() - T_START:6.1f} s] {msg}\n")
    sys.stderr.flush()


# A step longer than this gets one untimed warm-up only.
LONG_STEP_S = 5.0
# Planning guesses of a form's step time as a fraction of the f32 step on the
# same workload (measured on MI355X; each form's own warm-up step replaces
# the guess once it has run).
FORM_COST = {"f32": 1.0, "f16x3": 0.9, "f16": 0.5, "f16-recheck": 0.55}
# Time reserved for the refinement leg (library ascent, FP64 oracle
# gradient check) and for loading a form's input onto the device.
REFINE_RESERVE_S = 30.0
LOAD_RESERVE_S = 8.0


class Budget:
    """Wall-clock budget of the whole run, counted from process start: the
    timed steps of every form are sized so that the run prints its line
    before the deadline (full steps only; the count actually timed is
    reported)."""

    def __init__(self, seconds):
        self.deadline = T_START + seconds

    def left(self):
        return self.deadline - time.perf_counter()


# rows of the first MBD pass of the float32 kernel per lattice size
MBD_PASS1_ROWS = {16: 4, 32: 8, 64: 8, 128: 16, 256: 16}


def pruned_dft_flops(n, mask):
    """Work of an n-point radix-2 decimation-in-frequency DFT whose inputs
    outside `mask` (bit i: input i may be non-zero) are zero, counted as the
    kernel does it: a butterfly with two non-zero inputs 10 flops (the
    5 n log2 n convention), with one non-zero input 6 (its twiddle product
    only), with none 0."""
    flops, span = 0, n // 2
    while span >= 1:
        out = 0
        for b in range(n // 2):
            i0 = (b // span) * 2 * span + b % span
            i1 = i0 + span
            nz = ((mask >> i0) & 1) + ((mask >> i1) & 1)
            flops += (0, 6, 10)[nz]
            if nz:
                out |= (1 << i0) | (1 << i1)
        mask, span = out, span // 2
    return flops


def fringe_flops_per_cell(N, J, P, M, one_pass_rows=0, first_pass_rows=0):
    """Algorithmic FP32 work per evaluated cell of the FFT-form search: per
    (segment, rate) an SBD transform per IF (N * 5 PJ log2 PJ), an MBD
    transform per SBD bin (PJ * 5 M log2 M), |G|^2 and compare (4 PJ M) and
    the rotated segment sum (8 N J), divided by the PJ * M cells.

    one_pass_rows = MB > 0 counts the one-pass MBD form of a compact IF
    lattice instead, the work that form does: per SBD bin, M / MB lanes
    each twiddle MB - 1 rows (6 flops each) and run one MB-point transform
    (5 MB log2 MB).  first_pass_rows (a row set, bit i1) counts the
    two-pass form whose first pass transforms only those rows: the MBD
    term scaled by the pruned pass's share of the two passes' butterflies."""
    PJ = P * J
    if one_pass_rows:
        MB = one_pass_rows
        mbd = PJ * (M // MB) * (6 * (MB - 1) + 5 * MB * math.log2(MB))
    else:
        mbd = PJ * 5 * M * math.log2(M)
        if first_pass_rows:
            MA = MBD_PASS1_ROWS[M]
            MB = M // MA
            dense1 = MB * pruned_dft_flops(MA, (1 << MA) - 1)
            pass2 = MA * pruned_dft_flops(MB, (1 << MB) - 1)
            mbd *= (MB * pruned_dft_flops(MA, first_pass_rows) + pass2) / (dense1 + pass2)
    per = N * 5 * PJ * math.log2(PJ) + mbd + 4 * PJ * M + 8 * N * J
    return per / (PJ * M)


def three_real_products(form, N, J):
    """Whether the matrix-core MBD GEMM of this form forms each complex
    product from three real ones (the library's rule: f16x3 with 17-32 IFs
    and at most 64 channels)."""
    return form == "f16x3" and 16 < N <= 32 and J <= 64


def cpu_baseline(wl, V, target_s=15.0):
    """The FP64 oracle timed on a bounded sample of the same workload: whole
    segments (every rate, SBD and MBD cell) of baseline 0 at the middle DM
    trial, smallest window first, until about target_s of CPU work."""
    import numpy as np
    from oracle import frb_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    lay, srch = wl["layout"], wl["search"]
    g = O.build_grids(lay, srch)
    cal = O.calibration_phasor(lay["n_chan"], lay["chan_bw_mhz"], np.zeros(lay["n_if"]),
                               np.zeros(lay["n_if"]))
    d = srch["n_dm"] // 2
    PJ, M, R = len(g["tau_s"]), len(g["tau_m"]), len(g["rates"])
    O.search_row(V[0], g, cal, d, 0, q_list=[0], chunk=1)       # warm caches / BLAS
    Q = g["segs"][0][2]
    n, el = 0, 0.0
    t0 = time.perf_counter()
    while el < target_s and n < Q:
        k = min(8, Q - n)
        O.search_row(V[0], g, cal, d, 0, q_list=list(range(n, n + k)), chunk=8)
        n += k
        el = time.perf_counter() - t0
    cells = n * R * PJ * M
    return {"value": cells / el, "unit": "cells/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} segments (window {g['segs'][0][0]} APs, baseline 0, DM trial {d}) "
                      f"x {R} rates x {PJ} SBD x {M} MBD cells, float64 numpy oracle, "
                      f"{el:.1f} s",
            **host_cpu()}


def host_cpu():
    """The host's CPU model and logical core count."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "host_logical_cores": os.cpu_count()}


def cpu_full(wl, V, gpu_candidates):
    """The FP64 oracle over the whole workload (every baseline, DM trial,
    window and segment), timed, and its single-pulse detections against the
    f32 search's (baseline, DM trial, window, first AP) on the same data."""
    from oracle import frb_oracle as O
    lay, srch = wl["layout"], wl["search"]
    g = O.build_grids(lay, srch)
    # per baseline (the detection lists of steps b-d and the DM merge are per
    # baseline; cross-baseline matching only groups them)
    ora = set()
    t0 = time.perf_counter()
    for b in range(lay["n_baselines"]):
        res = O.search(V, lay, srch, baselines=[b])
        ora |= {(d["b"], d["d"], d["l"], d["k0"]) for d in res["detections"]}
        log(f"oracle baseline {b + 1}/{lay['n_baselines']}: {time.perf_counter() - t0:.1f} s")
    el = time.perf_counter() - t0
    cells = lay["n_baselines"] * srch["n_dm"] * sum(q for (_, _, q) in g["segs"]) * \
        len(g["rates"]) * len(g["tau_s"]) * len(g["tau_m"])
    gpu = {c[:4] for c in gpu_candidates}
    return {"value": cells / el, "unit": "cells/s", "seconds": round(el, 2), "cells": cells,
            "kind": "oracle, whole workload", "detections_oracle": len(ora),
            "detections_identical": ora == gpu, "only_oracle": len(ora - gpu),
            "only_gpu": len(gpu - ora), **host_cpu()}


def oracle_fd_check(wl, V, cells, peaks, theta, g_dev, n_check, budget_s):
    """The backward kernel's gradient against central differences of the
    FP64 oracle's relaxed |G| (h = 1e-3 grid cell in every parameter) on
    n_check peaks spread over the list.  Error of each component relative to
    max(|fd|, 1e-2 P / cell); stops early when budget_s runs out."""
    import numpy as np
    from oracle import frb_oracle as O
    lay, srch = wl["layout"], wl["search"]
    N, J, K = lay["n_if"], lay["n_chan"], lay["n_frames"]
    f0 = np.asarray(lay["if_freq_mhz"], dtype=np.float64)
    kdm = srch.get("k_dm", O.K_DM_DEFAULT) or O.K_DM_DEFAULT
    _, dxd = O.relaxed_offsets(1.0, f0, J, lay["chan_bw_mhz"], lay["t_ap_ms"], kdm)
    cal = np.ones((N, J), complex)
    errs, done, outliers = [], 0, []
    t0 = time.perf_counter()
    for i in np.unique(np.linspace(0, len(peaks) - 1, n_check).astype(int)):
        if time.perf_counter() - t0 > budget_s:
            break
        p = peaks[i]
        th = np.asarray(theta[i], dtype=np.float64)
        l = p["window_len"]
        # the frames the interpolation can touch, cast to float64 once
        x_hi = (abs(th[3]) + cells[3]) * float(dxd.max())
        lo = max(0, int(p["k0"]) - 16)
        hi = min(K, int(p["k0"]) + l + int(math.ceil(x_hi)) + 16 + int(abs(th[4])))
        Vb = np.asarray(V[p["baseline"], :, :, lo:hi], dtype=np.complex128)
        k0 = int(p["k0"]) - lo

        def P_of(t):
            return abs(O.relaxed_fringe(Vb, lay, srch, cal, k0, l, t, kdm)[0])
        P0 = P_of(th)
        for k in range(5):
            if cells[k] == 0:
                continue
            h = 1e-3 * cells[k]
            e = np.zeros(5)
            e[k] = h
            fd = (P_of(th + e) - P_of(th - e)) / (2 * h)
            scale = max(abs(fd), 1e-2 * P0 / cells[k])
            err = abs(g_dev[i, k] - fd) / scale
            errs.append(err)
            if err > 1e-3:
                # the difference quotient's own error: Richardson extrapolation
                # with h / 2 removes its h^2 term
                fd2 = (P_of(th + e / 2) - P_of(th - e / 2)) / h
                rich = (4 * fd2 - fd) / 3
                outliers.append({"peak": int(i), "param": ("sbd", "mbd", "rate", "dm", "t")[k],
                                 "err": float(err), "err_vs_extrapolated": float(abs(g_dev[i, k] - rich) / scale),
                                 "fd_truncation": float(abs(rich - fd) / scale)})
        done += 1
    errs = np.asarray(errs)
    if errs.size == 0:
        return {"peaks_checked": 0}
    return {"vs": "central differences of the FP64 oracle (h = 1e-3 cell), error relative to "
                  "max(|fd|, 1e-2 P/cell)",
            "peaks_checked": done, "components": int(errs.size),
            "median": float(np.median(errs)), "p99": float(np.percentile(errs, 99)),
            "max": float(errs.max()), "share_within_1e-3": float(np.mean(errs <= 1e-3)),
            "above_1e-3": outliers[:8], "seconds": round(time.perf_counter() - t0, 1)}


def refine_leg(args, wl, V, s, truth, budget):
    """Refinement of the top coarse peaks (by normalised power) after the
    search: the library's ascent timed with HIP events, the gradient of the
    backward kernel against central differences of the FP64 oracle, and the
    distance of the refined parameters from the injected truth for the peaks
    that belong to an injected pulse."""
    import numpy as np
    import torch
    lay, srch = wl["layout"], wl["search"]
    peaks = s.top_peaks(args.refine_peaks)
    n = len(peaks)
    if n == 0:
        return {"peaks": 0}
    s.refine(peaks, steps=args.refine_steps)       # warm-up (allocations, code load)
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th0, th, P = s.refine(peaks, steps=args.refine_steps)
    el = time.perf_counter() - t0
    tim = s.timing()
    cells, _ = s.refine_cells()
    # gradient check at a generic point a quarter cell off the grid
    th_chk = th0 + 0.25 * np.where(cells > 0, cells, 0.0)
    tt = torch.tensor(th_chk, dtype=torch.float64, device="cuda")
    g = s.refine_backward(tt, torch.ones(n, dtype=torch.float32, device="cuda")).cpu().numpy()
    fd = oracle_fd_check(wl, V, cells, peaks, th_chk, g, args.refine_fd_peaks,
                         max(5.0, min(60.0, budget.left() - args.cpu_seconds - 20.0)))
    log(f"refinement gradient vs FP64 central differences: {fd}")
    # truth: pulse-associated peaks (baseline, time overlap at f_ref, DM within 2 cells)
    t_ap = lay["t_ap_ms"]
    t_amb = cells[1] * srch["n_mbd"]
    errs, dm_errs = [], []
    for i, p in enumerate(peaks):
        for pu in truth.get("pulses", []):
            a0 = pu["t0_ms"] / t_ap
            w = pu["width_ms"] / t_ap
            if not (p["k0"] < a0 + w and a0 < p["k0"] + p["window_len"]):
                continue
            if abs(p["dm"] - pu["dm"]) > 2 * cells[3]:
                continue
            tau = pu["baseline_delay_us"][p["baseline"]]
            e = np.zeros(4)
            e[0] = (th[i, 0] - tau) / cells[0]
            e[1] = ((th[i, 1] - tau + t_amb / 2) % t_amb - t_amb / 2) / cells[1]
            e[2] = (th[i, 2] - pu.get("rate", 0.0)) / cells[2] if cells[2] > 0 else 0.0
            e[3] = (th[i, 3] - pu["dm"]) / cells[3]
            errs.append(e)
            if p["window_len"] == int(round(w)):
                dm_errs.append(e[3])
            break
    errs = np.abs(np.array(errs)) if errs else np.zeros((0, 4))
    within = {k: round(float(np.mean(errs[:, i] < 0.05)), 3) if len(errs) else None
              for i, k in enumerate(("sbd", "mbd", "rate", "dm"))}
    med = {k: round(float(np.median(errs[:, i])), 4) if len(errs) else None
           for i, k in enumerate(("sbd", "mbd", "rate", "dm"))}
    return {
        "peaks": n, "steps": args.refine_steps, "ms": round(1e3 * el, 3),
        "kernel_ms": round(tim["refine_ms"], 3), "launches": tim["n_refine"],
        "peak_steps_per_s": round(n * args.refine_steps / el, 1),
        "power_gain_median": round(float(np.median(P / np.maximum(
            s.refine_forward(torch.tensor(th0, dtype=torch.float64, device="cuda")).cpu().numpy(), 1e-30))), 5),
        "grad_vs_fp64_central_diff": fd,
        "pulse_peaks": int(len(errs)),
        "within_0.05_cell": within,
        "median_abs_err_cells": med,
        "dm_within_0.05_cell_window_eq_width": (round(float(np.mean(np.abs(dm_errs) < 0.05)), 3)
                                                if dm_errs else None),
        "n_window_eq_width": len(dm_errs),
    }


def run_form(args, wl, V, prec, dev, truth, budget, reserve_after, headline):
    """Full searches in one precision form: untimed warm-up (one when a step
    is long), then as many timed steps as the budget leaves after
    `reserve_after(step_s)` seconds for the legs still to come, at most
    --steps (at most 2 for a form that is not the headline).  Returns the
    JSON record (without the CPU baseline)."""
    import torch
    from paper_1801_02391_amd import frbx
    from paper_1801_02391_amd import workloads as W
    lay = wl["layout"]
    # "f16-recheck": the f16 form with every segment above threshold - band
    # (the crossings and the segments near the threshold) re-evaluated in f32
    base_prec = "f16" if prec == "f16-recheck" else prec
    band = args.recheck_band if prec == "f16-recheck" else 0.0
    srch = dict(wl["search"], precision=base_prec, recheck_band=band)
    if base_prec == "f16":
        Vt = torch.from_numpy(W.to_complex32(V)).to(dev)
    else:
        Vt = torch.from_numpy(V).to(dev)
    torch.cuda.synchronize()
    s = frbx.Search(lay, device=0)
    s.configure(srch)
    s.load(Vt)
    seg = s.segments()
    B, D = lay["n_baselines"], srch["n_dm"]
    N, J, P, M, R = lay["n_if"], lay["n_chan"], srch["sbd_pad"], srch["n_mbd"], srch["n_rate"]
    PJ = P * J
    cells = B * D * seg["total"] * R * PJ * M
    log(f"{prec}: segments/(b,d) {seg['total']}  cells/step {cells:.3e}")

    # warm-up: the first run (allocations, code load) is never timed; more
    # warm-up runs only while a step is short
    want_warm = max(1, args.warmup if headline else 1)
    warm = []
    while len(warm) < want_warm:
        t = time.perf_counter()
        s.run()
        warm.append(time.perf_counter() - t)
        log(f"{prec}: warmup {len(warm)}/{want_warm} {warm[-1]:.2f} s")
        if warm[-1] > LONG_STEP_S or budget.left() - reserve_after(warm[-1]) < 2 * warm[-1]:
            break
    step_s = warm[-1]
    max_steps = args.steps if headline else min(args.steps, 2)
    n_steps = int(max(1, min(max_steps, (budget.left() - reserve_after(step_s)) // step_s)))
    log(f"{prec}: timing {n_steps} step(s) of ~{step_s:.2f} s ({budget.left():.0f} s of budget left)")
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tim = {"fringe_ms": 0.0, "n_fringe": 0, "fringe_units": 0, "dedisperse_ms": 0.0,
           "n_dedisperse": 0, "dedisperse_units": 0, "stats_ms": 0.0, "n_stats": 0,
           "dedisperse_bytes": 0}
    for i in range(n_steps):
        t = time.perf_counter()
        s.run()
        tt = s.timing()
        for k in tim:
            tim[k] += tt[k]
        log(f"{prec}: step {i + 1}/{n_steps} {time.perf_counter() - t:.2f} s "
            f"(fringe {tt['fringe_ms'] / 1e3:.2f} s, dedisperse {tt['dedisperse_ms'] / 1e3:.3f} s)")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: read {n * 4} B, wrote {n * 4} B")
        del src, dst
    cands = s.candidates()
    n_det = len(cands)
    groups = s.groups()
    n_rep = sum(1 for g in groups if g["reported"])
    refine = (refine_leg(args, wl, V, s, truth, budget)
              if (prec == "f32" and args.refine_peaks > 0) else None)

    # dominant kernel: the fringe search
    cells_per_unit = R * PJ * M
    avg_ms = tim["fringe_ms"] / max(1, tim["n_fringe"])
    units_per_launch = tim["fringe_units"] / max(1, tim["n_fringe"])
    rows = mbd_one_pass_rows(s, M) if prec == "f32" else 0
    extra = {}
    if prec == "f32":
        # FFT-form FP32 work on the vector ALUs (the one-pass form's own work
        # when it runs, the pruned first pass's when the kernel is compiled
        # for the lattice's rows)
        spec_rows = s.specialisation()[0] if not rows else 0
        fpc = fringe_flops_per_cell(N, J, P, M, rows, spec_rows)
        bound, peak, kern = "alu", PEAK_FP32_TFLOPS, "fringe_kernel"
    else:
        # the matrix-core work: the real-embedded MBD GEMM, 2 x (2N) x (2M)
        # flops per SBD bin, i.e. 8 N flops per cell, or 6 N where each
        # complex product is formed from three real ones (three GEMMs of
        # K = N); f16x3 issues it three times (high/low split), reported
        # separately.  The f16 form also runs the SBD transform as a
        # real-embedded GEMM where J <= 64: per (segment, rate) P sub-grids
        # of 2 x (2J) x (2J) x N flops over PJ M cells, 8 N J / M flops per
        # cell.
        k3 = three_real_products(base_prec, N, J)
        fpc = (6 if k3 else 8) * N
        extra["mbd_products"] = "three real per complex" if k3 else "four real per complex"
        extra["method_flops_per_cell"] = 8 * N
        kern = "fringe_mfma_kernel"
        if base_prec == "f16" and srch.get("sbd_mfma") and J in SBD_GEMM_CHANNELS:
            fpc += 8 * N * J / M
            extra["method_flops_per_cell"] += 8 * N * J / M
            kern = "fringe_gemm_kernel"
        bound, peak = "mfma", PEAK_FP16_MFMA_TFLOPS
    flops_launch = units_per_launch * cells_per_unit * fpc
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    if prec == "f32":
        extra = {"attainable_peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS,
                 "frac_attainable": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4)}
    elif base_prec == "f16x3":
        extra.update({"issued_products": 3, "achieved_issued": round(3 * achieved, 3),
                      "frac_issued": round(3 * achieved / peak, 4)})
    tkey = kern if prec == "f32" else f"{kern}_{base_prec}"
    traffic = measured_traffic(tkey, args.workload)
    roof = {"bound": bound, "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), **extra,
            "traffic": traffic,
            **({"traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT)} if traffic is not None else {}),
            "kernel": kern, "avg_launch_ms": round(avg_ms, 4),
            "flops_per_cell": round(fpc, 3), "units_per_launch": units_per_launch}
    if prec == "f32":
        roof.update(mbd_form(rows, s))
    # dedispersion kernel against HBM: every dedispersed spectrum written
    # once and every channel's input span read once per group of DM trials
    # (byte count reported by the library per launch)
    d_avg = tim["dedisperse_ms"] / max(1, tim["n_dedisperse"])
    d_bytes = tim["dedisperse_bytes"] / max(1, tim["n_dedisperse"])
    d_gbs = d_bytes / (d_avg * 1e-3) / 1e9 if d_avg > 0 else 0.0
    d_traffic = measured_traffic("dedisperse_kernel_complex32" if base_prec == "f16" else "dedisperse_kernel",
                                 args.workload)
    roof_dd = {"bound": "hbm", "achieved": round(d_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "frac": round(d_gbs / PEAK_HBM_GBS, 4), "kernel": "dedisperse_kernel",
               "avg_launch_ms": round(d_avg, 4), "algorithmic_bytes_per_launch": d_bytes,
               "traffic": d_traffic,
               **({"traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT)} if d_traffic is not None else {})}

    out = {
        "metric": "search cells/s (baseline x DM x window segment x rate x SBD x MBD)",
        "value": cells * n_steps / el,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": len(warm),
        "ms_per_step": 1e3 * el / n_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16x3": "f16x3 (MBD: 3 f16 MFMA products, f32 accumulate)",
                  "f16": "f16 storage + f16 MFMA, f32 accumulate",
                  "f16-recheck": f"f16 storage + f16 MFMA, f32 accumulate; segments above "
                                 f"threshold - {band} re-evaluated in f32"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "baselines": B, "if": N, "chan": J,
                   "frames": lay["n_frames"], "dm_trials": D, "rate_bins": R, "sbd_bins": PJ,
                   "mbd_bins": M, "windows": srch["windows"], "segments_per_bl_dm": seg["total"],
                   "cells_per_step": cells},
        "roofline": roof,
        "roofline_dedisperse": roof_dd,
        **({"recheck": {"band": band, "segments": s.recheck()[1],
                        "fraction_of_segments": s.recheck()[1] / max(1, B * D * seg["total"])}}
           if band > 0 else {}),
        "detections": n_det,
        "reported_groups": n_rep,
        "_candidates": [(c["baseline"], c["dm_index"], c["window_len"], c["k0"], c["power_norm"])
                        for c in cands],
        "_crossings": [(c["baseline"], c["dm_index"], c["window_index"], c["segment"], c["power_norm"])
                       for c in s.crossings()],
    }
    if refine is not None:
        out["refine"] = refine
    del s, Vt
    torch.cuda.empty_cache()
    return out


def run_stream(args):
    """Streaming search (chunks pushed as FP8 e4m3 with per-channel scales,
    DM-overlap carry on the device): the pushes that fill the carry are
    untimed; every later push completes a full chunk of segments and is
    timed.  Reports chunks per second for the baselines searched and the
    fraction of real time that one GPU sustains for the whole array."""
    import numpy as np
    import torch
    from paper_1801_02391_amd import frbx
    from paper_1801_02391_amd import workloads as W
    name = "stream-45bl-16x256-600000"
    base = W.get_workload(name)
    chunk = base["chunk_frames"]
    K = chunk * args.chunks
    nb = args.baselines or 1
    n_pulses = max(1, round(base["signal"]["pulses"]["count"] * K / base["layout"]["n_frames"]))
    wl = W.get_workload(name, layout=dict(n_frames=K),
                        signal=dict(pulses=dict(base["signal"]["pulses"], count=n_pulses)))
    log(f"generating {nb} baseline(s) x {K} APs of {name}")
    t0 = time.perf_counter()
    V, truth = W.generate(wl, baselines=list(range(nb)))
    lay = dict(wl["layout"], n_baselines=nb, stations=wl["layout"]["stations"][:nb])
    srch = dict(wl["search"], precision=args.precision)
    codes, scales, plain = [], [], []
    for i in range(args.chunks):
        ci = np.ascontiguousarray(V[..., i * chunk:(i + 1) * chunk])
        c8, sc = W.to_e4m3(ci)
        codes.append(torch.from_numpy(c8).cuda())
        scales.append(torch.from_numpy(sc).cuda())
        if args.quant_error:
            plain.append(ci)
    del V
    log(f"generated and encoded in {time.perf_counter() - t0:.1f} s")
    s = frbx.Search(lay, device=0)
    s.configure(srch)
    seg = s.segments()
    lmax = max(srch["windows"])
    n_warm = min(args.chunks - 1, -(-(seg["dk_max"] + lmax) // chunk))
    s.stream_begin(chunk)
    N, J, P, M, R, D = lay["n_if"], lay["n_chan"], srch["sbd_pad"], srch["n_mbd"], srch["n_rate"], srch["n_dm"]
    cells_seg = R * P * J * M
    tim = {"fringe_ms": 0.0, "n_fringe": 0, "fringe_units": 0, "dedisperse_ms": 0.0,
           "n_dedisperse": 0, "dedisperse_units": 0, "dedisperse_bytes": 0}
    t_push, cells, cubes = [], 0, []
    for i in range(args.chunks):
        timed = i >= n_warm
        s.set_timing(timed)
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.stream_push(codes[i], "e4m3", scales[i])
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        pos = s.stream_position()
        ns = sum(pos["n_seg"])
        log(f"push {i + 1}/{args.chunks} {'timed' if timed else 'warm-up'}: {el:.2f} s, {ns} segments per (b, d)")
        if args.quant_error:
            cubes.append((s.power_cube()[0], s.crossings()))
        if timed:
            t_push.append(el)
            cells += nb * D * ns * cells_seg
            tt = s.timing()
            for k in tim:
                tim[k] += tt[k]
    el = sum(t_push)
    chunk_s = el / len(t_push)
    t_chunk = chunk * lay["t_ap_ms"] * 1e-3
    full_b = base["layout"]["n_baselines"]
    avg = tim["fringe_ms"] / max(1, tim["n_fringe"])
    units = tim["fringe_units"] / max(1, tim["n_fringe"])
    if args.precision == "f32":
        rows = mbd_one_pass_rows(s, M)
        fpc = fringe_flops_per_cell(N, J, P, M, rows, 0 if rows else s.specialisation()[0])
        bound, peak, kern = "alu", PEAK_FP32_TFLOPS, "fringe_kernel"
    else:
        fpc = (6 if three_real_products(args.precision, N, J) else 8) * N * (3 if args.precision == "f16x3" else 1)
        bound, peak, kern = "mfma", PEAK_FP16_MFMA_TFLOPS, "fringe_mfma_kernel"
        if args.precision == "f16" and srch.get("sbd_mfma") and J in SBD_GEMM_CHANNELS:
            fpc += 8 * N * J / M
            kern = "fringe_gemm_kernel"
    ach = units * cells_seg * fpc / (avg * 1e-3) / 1e12 if avg > 0 else 0.0
    d_avg = tim["dedisperse_ms"] / max(1, tim["n_dedisperse"])
    d_gbs = tim["dedisperse_bytes"] / max(1, tim["n_dedisperse"]) / (d_avg * 1e-3) / 1e9 if d_avg > 0 else 0.0
    n_det = len(s.candidates())
    quant = quantisation_error(s, lay, srch, chunk, plain, codes, scales, cubes, truth) if args.quant_error else None
    return {
        "metric": "search cells/s (baseline x DM x window segment x rate x SBD x MBD)",
        "value": cells / el, "unit": "cells/s", "n_gpus": 1, "steps": len(t_push), "warmup": n_warm,
        "ms_per_step": 1e3 * chunk_s, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f16x3": "f16x3 (MBD: 3 f16 MFMA products, f32 accumulate)",
                  "f16": "f16 MFMA, f32 accumulate"}[args.precision] + ", input fp8 e4m3 + f32 scale",
        "data": "synthetic",
        "config": {"workload": name, "baselines": nb, "of_baselines": full_b, "if": N, "chan": J,
                   "chunk_frames": chunk, "chunk_s": t_chunk, "dm_trials": D, "rate_bins": R,
                   "sbd_bins": P * J, "mbd_bins": M, "windows": srch["windows"], "dk_max": seg["dk_max"]},
        "stream": {"s_per_chunk": chunk_s, "chunks_per_s": 1.0 / chunk_s,
                   "real_time_fraction_one_gpu_all_baselines": t_chunk / (chunk_s * full_b / nb),
                   "dedisperse_gbs": round(d_gbs, 1), "dedisperse_frac_hbm": round(d_gbs / PEAK_HBM_GBS, 4),
                   "detections_so_far": n_det},
        "roofline": {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(ach / peak, 4), "traffic": None, "kernel": kern,
                     "avg_launch_ms": round(avg, 4), "flops_per_cell": round(fpc, 2),
                     "units_per_launch": units, **(mbd_form(mbd_one_pass_rows(s, M), s) if args.precision == "f32" else {})},
        "quantisation": quant,
    }


def quantisation_error(s8, lay, srch, chunk, plain, codes, scales, pushed8, truth):
    """Search the same chunks again unquantised (complex64) and compare with
    the FP8 stream: the storage form's error in the data, in every segment's
    peak power, in the threshold crossings and in the detections (all of
    them, and those that overlap an injected pulse)."""
    import numpy as np
    import torch
    from paper_1801_02391_amd import frbx
    from paper_1801_02391_amd import workloads as W
    num = den = 0.0
    for c, c8, sc in zip(plain, codes, scales):
        q = W.from_e4m3(c8.cpu().numpy(), sc.cpu().numpy())
        num += float(np.sum(np.abs(q - c) ** 2))
        den += float(np.sum(np.abs(c) ** 2))
    s = frbx.Search(lay, device=0)
    s.configure(srch)
    s.stream_begin(chunk)
    rel, x0, x8 = [], {}, {}
    xkey = lambda x: (x["baseline"], x["dm_index"], x["window_index"], x["segment"])
    for c, (P8, cr8) in zip(plain, pushed8):
        s.stream_push(torch.from_numpy(c).cuda())
        P = s.power_cube()[0]
        ok = P > 0
        rel.append((np.abs(P8[ok] - P[ok]) / P[ok]).ravel())
        x0.update({xkey(x): x["power_norm"] for x in s.crossings()})
        x8.update({xkey(x): x["power_norm"] for x in cr8})
    rel = np.concatenate(rel)
    thr = srch["threshold"]
    xdiff = set(x0) ^ set(x8)
    common = set(x0) & set(x8)
    key = lambda d: (d["baseline"], d["dm_index"], d["window_len"], d["k0"])
    d0, d8 = s.candidates(), s8.candidates()
    a, b = {key(d) for d in d0}, {key(d) for d in d8}
    t_ap = lay["t_ap_ms"]

    def pulses_found(dets):
        n = 0
        for pu in truth.get("pulses", []):
            a0, w = pu["t0_ms"] / t_ap, pu["width_ms"] / t_ap
            if any(d["k0"] < a0 + w and a0 < d["k0"] + d["window_len"] for d in dets):
                n += 1
        return n
    log(f"quantisation: {rel.size} segment powers, {len(x0)} / {len(x8)} crossings, "
        f"{len(a)} / {len(b)} detections compared")
    return {"vs": "the same chunks searched as complex64 (unquantised)",
            "data_rel_rms": round(float(np.sqrt(num / den)), 5),
            "power_rel_err_median": float(np.median(rel)), "power_rel_err_p99": float(np.quantile(rel, 0.99)),
            "power_rel_err_max": float(rel.max()), "segments": int(rel.size),
            "crossings_unquantised": len(x0), "crossings_fp8": len(x8), "crossings_differing": len(xdiff),
            "crossings_differing_max_abs_power_norm_minus_threshold":
                round(max((abs(x0.get(k, x8.get(k)) - thr) for k in xdiff), default=0.0), 4),
            "crossings_common_max_abs_power_norm_diff":
                round(max((abs(x0[k] - x8[k]) for k in common), default=0.0), 4),
            "detections_unquantised": len(a), "detections_fp8": len(b),
            "detections_only_unquantised": len(a - b), "detections_only_fp8": len(b - a),
            "pulses_injected": len(truth.get("pulses", [])),
            "pulses_found_unquantised": pulses_found(d0), "pulses_found_fp8": pulses_found(d8)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="vgos-6bl-32x64-20000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-full", action="store_true",
                    help="also run the FP64 oracle over the whole workload (small workloads): "
                         "its cells/s and whether its detections equal the f32 search's")
    ap.add_argument("--precision", default="f32", choices=["f32", "f16x3", "f16"],
                    help="f32: vector-ALU FFT transforms; f16x3: MBD on the matrix cores "
                         "as three float16 products (float32-grade); f16: one float16 "
                         "product with complex32 (float16) stored cross spectra")
    ap.add_argument("--only", action="store_true",
                    help="time only --precision (default: also the other forms, reported "
                         "with their speedup over it)")
    ap.add_argument("--baselines", type=int, default=0,
                    help="search only the first n baselines (one GPU's share of a larger array)")
    ap.add_argument("--stream", action="store_true",
                    help="streaming run of the 45-baseline FP8 workload instead: --baselines "
                         "of its baselines (default 1), --chunks 1 s chunks, the last two timed")
    ap.add_argument("--chunks", type=int, default=6)
    ap.add_argument("--recheck-band", type=float, default=0.05,
                    help="the f16-recheck form re-evaluates in f32 every segment whose "
                         "normalised power exceeds threshold - band")
    ap.add_argument("--quant-error", action="store_true",
                    help="with --stream: search the chunks again unquantised and report the "
                         "FP8 storage error in the data, the powers and the detections")
    ap.add_argument("--refine-peaks", type=int, default=1024,
                    help="after the f32 search, refine this many top peaks (0: skip)")
    ap.add_argument("--refine-steps", type=int, default=20)
    ap.add_argument("--refine-fd-peaks", type=int, default=256,
                    help="peaks whose backward-kernel gradient is checked against central "
                         "differences of the FP64 oracle")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock budget of the whole run from process start: the number of "
                         "timed (full) steps of each form is cut to fit it and reported")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after the timed steps, run one plain device copy (float32 "
                         "multiply by 1) of this many MiB, to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "frbx searches on one GPU only: --gpus must be 1 (across "
                                   "GPUs the search would be split by baseline, which is not built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1801_02391_amd import frbx
    from paper_1801_02391_amd import workloads as W

    if args.stream:
        print(json.dumps(run_stream(args)), flush=True)
        return
    wl = W.get_workload(args.workload)
    lay, srch = wl["layout"], wl["search"]
    log(f"generating {args.workload}")
    t0 = time.perf_counter()
    if args.baselines and args.baselines < lay["n_baselines"]:
        # one GPU's share of the baselines, at the workload's full shape
        V, truth = W.generate(wl, baselines=list(range(args.baselines)))
        wl["layout"]["n_baselines"] = args.baselines
        wl["layout"]["stations"] = wl["layout"]["stations"][:args.baselines]
    else:
        V, truth = W.generate(wl)
    log(f"generated {V.nbytes / 1e9:.2f} GB in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()

    forms = [args.precision] if args.only else [args.precision] + [p for p in ("f16x3", "f16", "f16-recheck")
                                                                   if p != args.precision]
    budget = Budget(args.budget_s)
    cpu_s = 0.0 if args.no_cpu_baseline else args.cpu_seconds + 5.0

    def reserve(rest, base_step):
        """Seconds the legs after the current one need: each remaining form
        loads its input and runs three steps (one warm-up, two timed), the
        f32 refinement leg, the CPU baseline."""
        r = cpu_s
        for f in rest:
            r += LOAD_RESERVE_S + 3.0 * FORM_COST[f] / FORM_COST[args.precision] * base_step
        return r

    results, skipped = {}, {}
    base_step = None
    for i, prec in enumerate(forms):
        rest = forms[i + 1:]
        if i == 0:
            refine_s = REFINE_RESERVE_S if (prec == "f32" and args.refine_peaks > 0) else 0.0
            res = lambda st: reserve(rest, st) + refine_s
        else:
            res = lambda st: reserve(rest, base_step)
            need = LOAD_RESERVE_S + 2.0 * FORM_COST[prec] / FORM_COST[args.precision] * base_step
            if budget.left() - reserve(rest, base_step) < need:
                skipped[prec] = f"not run: {budget.left():.0f} s of the {args.budget_s:.0f} s budget left"
                log(f"{prec}: {skipped[prec]}")
                continue
        results[prec] = run_form(args, wl, V, prec, dev, truth, budget, res, headline=(i == 0))
        if i == 0:
            base_step = results[prec]["ms_per_step"] * 1e-3
    out = results[args.precision]
    out["steps_requested"] = args.steps
    out["warmup_requested"] = args.warmup
    out["budget_s"] = args.budget_s
    base_c = {c[:4]: c[4] for c in out["_candidates"]}
    thr = srch["threshold"]

    base_x = {c[:4]: c[4] for c in out["_crossings"]}

    def compare(r):
        other = {c[:4]: c[4] for c in r["_candidates"]}
        diff = sorted(set(base_c) ^ set(other))
        pn = [base_c.get(k, other.get(k)) for k in diff]
        ox = {c[:4]: c[4] for c in r["_crossings"]}
        xdiff = sorted(set(base_x) ^ set(ox))
        xpn = [base_x.get(k, ox.get(k)) for k in xdiff]
        common = set(base_x) & set(ox)
        return {"identical": not diff, "only_" + args.precision: sum(1 for k in diff if k in base_c),
                "only_this_form": sum(1 for k in diff if k in other),
                "differing_power_norm_minus_threshold": [round(v - thr, 5) for v in pn[:8]],
                "crossings_differing": len(xdiff),
                "crossings_differing_max_abs_power_norm_minus_threshold":
                    round(max((abs(v - thr) for v in xpn), default=0.0), 5),
                "crossings_common_max_abs_power_norm_diff":
                    round(max((abs(base_x[k] - ox[k]) for k in common), default=0.0), 6)}
    if len(forms) > 1:
        base = out["value"]
        out["precision_forms"] = {
            p: {"value": r["value"], "ms_per_step": r["ms_per_step"], "dtype": r["dtype"],
                "speedup_vs_" + args.precision: r["value"] / base, "roofline": r["roofline"],
                "detections": r["detections"], "reported_groups": r["reported_groups"],
                **({"recheck": r["recheck"]} if "recheck" in r else {}),
                "candidates_vs_" + args.precision: compare(r)}
            for p, r in results.items() if p != args.precision}
        out["precision_forms"].update({p: {"skipped": why} for p, why in skipped.items()})
    if args.cpu_full and args.precision == "f32":
        log("timing the oracle on the whole workload")
        out["cpu_full"] = cpu_full(wl, V, out["_candidates"])
    for r in results.values():
        r.pop("_candidates", None)
        r.pop("_crossings", None)
    if not args.no_cpu_baseline:
        log("timing the oracle on a CPU sample")
        out["cpu_baseline"] = cpu_baseline(wl, V[:1], max(3.0, min(args.cpu_seconds, budget.left() - 5.0)))
    out["wall_s"] = round(time.perf_counter() - T_START, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
