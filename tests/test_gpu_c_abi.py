"""A whole search from plain C through the C ABI (tests/c_search_check.c:
host-pointer load, default stream, no Python on the device path) gives the
same power cube, bit for bit, as the Python binding on the same data."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from paper_1801_02391_amd import frbx
from paper_1801_02391_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1801_02391_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_search_from_c_equals_the_binding(tmp_path):
    f0 = [3000.0 + 32.0 * n * (n + 1) / 2 for n in range(5)]
    wl = W.custom_workload(if_freq_mhz=f0, n_chan=32, chan_bw_mhz=1.0, t_ap_ms=1.0, n_frames=300,
                           n_stations=3, config_id=160,
                           search=dict(dm_lo=0.0, dm_step=100.0, n_dm=3, sbd_pad=4, n_mbd=64, n_rate=2,
                                       windows=[2, 4, 8], threshold=3.0, n_win_min=2, n_bl_min=1),
                           signal=dict(pulses=dict(kind="fixed", list=[
                               dict(t0_ms=120.0, dm=100.0, width_ms=4.0, snr=25.0, delay_us=0.01)])))
    V, _ = W.generate(wl)
    inp, out = tmp_path / "v.bin", tmp_path / "cube.bin"
    np.ascontiguousarray(V).tofile(inp)
    exe = tmp_path / "c_search_check"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_search_check.c"), "-L", LIBDIR, "-lfrbx",
                    f"-Wl,-rpath,{LIBDIR}", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe), str(inp), str(out), "3", "5", "32", "300", "3", "100", "2", "64",
                        *[repr(x) for x in f0]], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    n = int(r.stdout.split()[1])
    raw = np.fromfile(out, dtype=np.uint8)
    Pc = raw[:4 * n].view(np.float32)
    Ic = raw[4 * n:].view(np.int32)
    s = frbx.Search(wl["layout"])
    s.configure(wl["search"])
    s.load(torch.from_numpy(np.ascontiguousarray(V)).cuda())
    s.run()
    P, I = s.power_cube()
    assert np.array_equal(P.ravel().view(np.uint32), Pc.view(np.uint32)) and np.array_equal(I.ravel(), Ic)
    assert int(r.stdout.split()[3]) == len(s.candidates())
    # the MBD lattice seen from C equals the binding's
    lat = s.lattice()
    line = r.stdout.splitlines()[1].split()
    assert line[0] == "lattice" and int(line[1]) == lat["compact_shift"]
    assert float(line[2]) == lat["mbd_step_us"] and [int(x) for x in line[3:]] == lat["q"]
