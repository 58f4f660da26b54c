"""The C ABI from plain C: tests/c_abi_check.c is compiled with gcc as C11
against include/frbx.h, linked with libfrbx.so and run on the CPU; its
AP-offset table must equal the oracle's and its grouping the hand-derived
result."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import frb_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1801_02391_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_program_uses_the_abi(tmp_path):
    exe = tmp_path / "c_abi_check"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_check.c"), "-L", LIBDIR, "-lfrbx",
                    f"-Wl,-rpath,{LIBDIR}", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = {ln.split()[0]: ln.split()[1:] for ln in r.stdout.splitlines()}
    assert lines["version"][0] == "frbx"
    dk = np.array(list(map(int, lines["dk"]))).reshape(3, 4, 16)
    ora = O.ap_offsets(O.dm_trials(0.0, 150.0, 3), [3000.0, 3032.0, 3096.0, 3192.0], 16, 1.0, 1.0, 4.149e6)
    assert np.array_equal(dk, ora)
    # positions 0, 1, 3, 6 of a 32 MHz lattice (T = 1/32 us): the one-pass form, shift 0
    assert lines["lattice"][0] == "0" and float(lines["lattice"][1]) == 1.0 / 32 / 256
    assert lines["lattice"][2:] == ["0", "1", "3", "6"]
    # baseline 0 has two overlapping windows -> one detection (the 8-AP window
    # is inserted first, the higher normalised power survives); baseline 1 one;
    # they overlap in time -> one group of 2 baselines, reported
    assert lines["detections"] == ["2", "groups", "1", "reported", "1"]
    dets = [ln.split()[1:] for ln in r.stdout.splitlines() if ln.startswith("det ")]
    assert dets == [["0", "102", "8", "5.000"], ["1", "104", "4", "6.000"]]
    assert lines["null"] == ["null", "context"]
