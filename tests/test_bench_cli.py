"""CPU checks of the benchmark's command line and the workload catalogue
(no device needed)."""
import json
import os
import subprocess
import sys

import numpy as np

from paper_1801_02391_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_workload_catalogue_shapes():
    """The benchmark workloads carry the shapes they are quoted on."""
    wl = W.get_workload("vgos-6bl-32x64-20000")
    lay, s = wl["layout"], wl["search"]
    assert (lay["n_baselines"], lay["n_if"], lay["n_chan"], lay["n_frames"]) == (6, 32, 64, 20000)
    assert (s["n_dm"], s["n_rate"], s["sbd_pad"], s["n_mbd"]) == (256, 8, 4, 256)
    wl = W.get_workload("precision-21bl-32x128-40000")
    assert (wl["layout"]["n_baselines"], wl["layout"]["n_chan"], wl["layout"]["chan_bw_mhz"]) == (21, 128, 0.25)
    wl = W.get_workload("stream-45bl-16x256-600000")
    lay, s = wl["layout"], wl["search"]
    assert (lay["n_baselines"], lay["n_if"], lay["n_chan"], lay["n_frames"]) == (45, 16, 256, 600000)
    assert s["n_dm"] == 2048 and abs(s["dm_step"] * s["n_dm"] - 3000.0) < 1e-9 and wl["chunk_frames"] == 10000
    # the IF lattice of every benchmark layout has distinct positions below M
    for name in ("vgos-6bl-32x64-20000", "precision-21bl-32x128-40000", "stream-45bl-16x256-600000"):
        f0 = np.asarray(W.get_workload(name)["layout"]["if_freq_mhz"])
        d = f0 - f0[0]
        g = np.gcd.reduce(np.round(d[1:] * 1000).astype(np.int64))
        q = np.round(d * 1000 / g).astype(np.int64)
        assert len(set(q)) == len(q) and q.max() < 256


def test_short_stream_workload_generates_one_baseline():
    wl = W.get_workload("stream-45bl-16x256-600000", layout=dict(n_frames=40000),
                        signal=dict(pulses=dict(W.get_workload("stream-45bl-16x256-600000")["signal"]["pulses"],
                                                count=3)))
    V, truth = W.generate(wl, baselines=[0])
    assert V.shape == (1, 16, 256, 40000) and V.dtype == np.complex64
    assert len(truth["pulses"]) == 3


def test_algorithmic_flops_per_cell_of_the_roofline():
    """FFT-form work per cell behind the f32 roofline, against the count
    written out by hand: per (segment, rate) N 5 PJ log2 PJ (SBD) +
    PJ 5 M log2 M (MBD) + 4 PJ M (|G|^2 and compare) + 8 N J (rotated
    segment sum), over PJ M cells."""
    sys.path.insert(0, ROOT)
    import bench
    # VGOS: N = 32, J = 64, PJ = 256, M = 256:
    # (327680 + 2621440 + 262144 + 16384) / 65536
    assert bench.fringe_flops_per_cell(32, 64, 4, 256) == 3227648 / 65536 == 49.25
    # streaming: N = 16, J = 256, PJ = 1024, M = 256:
    # (819200 + 10485760 + 1048576 + 32768) / 262144
    assert bench.fringe_flops_per_cell(16, 256, 4, 256) == 12386304 / 262144 == 47.25


def test_algorithmic_flops_per_cell_of_the_one_pass_form():
    """The one-pass MBD form (compact IF lattice) is credited with the work it
    does: per SBD bin, M / MB lanes each twiddle MB - 1 rows (6 flops) and
    run one MB-point transform (5 MB log2 MB), instead of 5 M log2 M.
    Single-baseline shape, N = 8, J = 32, PJ = 128, M = 256, MB = 16:
    (35840 + 128 x 16 x (90 + 320) + 131072 + 2048) / 32768."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.fringe_flops_per_cell(8, 32, 4, 256, 16) == 1008640 / 32768 == 30.78125
    # below the two-pass count of the same shape
    assert bench.fringe_flops_per_cell(8, 32, 4, 256) > 30.78125


def test_work_of_the_pruned_first_pass():
    """Hand count for the VGOS row set {0, 4, 6, 7, 14} of a 16-point
    decimation-in-frequency transform: stage 1 (span 8) has three butterflies
    with one non-zero input and one with two (3 x 6 + 10 = 28), stage 2
    four with two and four with one (44), stage 3 four and four (64), stage
    4 eight full butterflies (80): 216 of the dense 5 x 16 x 4 = 320."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.pruned_dft_flops(16, 0xFFFF) == 320
    assert bench.pruned_dft_flops(16, 0x40D1) == 28 + 44 + 64 + 80
    assert bench.pruned_dft_flops(16, 0x0001) == 6 * (8 + 4 + 2 + 1) - 6 * 0
    # two-pass VGOS cell: 16 lanes x (216 instead of 320) in the first pass,
    # 16 x 320 in the second, of 5 x 256 x 8 = 10240 FFT-form flops
    full = bench.fringe_flops_per_cell(32, 64, 4, 256)
    pruned = bench.fringe_flops_per_cell(32, 64, 4, 256, 0, 0x40D1)
    assert abs((full - pruned) * 65536 - 256 * 10240 * (1 - (16 * 216 + 16 * 320) / (32 * 320))) < 1e-6


def test_measured_traffic_is_keyed_to_the_kernel_code(tmp_path, monkeypatch):
    """The bench reports counter-measured HBM bytes only for the workload they
    were taken on and only while the kernel code hashes as it did then; the
    hash ignores comments and blank lines."""
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.hip"
    src.write_text("int x;  // a note\n\nint y;\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    sha = bench.kernel_code_sha256()
    src.write_text("// another note\nint x;\nint y;   // changed commentary\n")
    assert bench.kernel_code_sha256() == sha
    traffic = tmp_path / "traffic.txt"
    traffic.write_text(f"# comment = ignored\nkernels_sha256 = {sha}\nfringe_kernel = 12345\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    assert bench.measured_traffic("fringe_kernel", "vgos-6bl-32x64-20000") == 12345.0
    assert bench.measured_traffic("fringe_kernel", "single-1bl-8x32-1000") is None
    assert bench.measured_traffic("dedisperse_kernel", "vgos-6bl-32x64-20000") is None
    src.write_text("int x;\nint y = 1;\n")
    assert bench.measured_traffic("fringe_kernel", "vgos-6bl-32x64-20000") is None
