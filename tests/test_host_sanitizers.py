"""The host side of libfrbx under AddressSanitizer and UndefinedBehavior-
Sanitizer, on the CPU: the library is rebuilt with both sanitizers on its
host code (device code is never instrumented), the plain C programs that use
the C ABI are built with them too, and they run with any report fatal.
The instrumented build is cached under _build/san, keyed by the sources."""
import hashlib
import os
import shutil
import subprocess

import pytest

from paper_1801_02391_amd.build import write_rtc_source

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1801_02391_amd", "csrc")
INC = os.path.join(ROOT, "include")
SAN = os.path.join(ROOT, "_build", "san")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                                reason="ROCm hipcc / clang not available")


def _digest():
    h = hashlib.sha256()
    for name in ("frbx_host.cpp", "frbx_kernels.hip", "frbx_internal.h", "frbx_fringe.h", "frbx_jit.cpp"):
        h.update(open(os.path.join(CSRC, name), "rb").read())
    h.update(open(os.path.join(INC, "frbx.h"), "rb").read())
    h.update(" ".join(SAN_HOST).encode())
    return h.hexdigest()[:16]


@pytest.fixture(scope="module")
def san_lib():
    out = os.path.join(SAN, _digest())
    lib = os.path.join(out, "libfrbx.so")
    if not os.path.exists(lib):
        os.makedirs(out, exist_ok=True)
        flags = ["-std=c++17", "-fPIC", "-g", "-O1", f"--offload-arch=gfx950",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        k = os.path.join(out, "k.o")
        h = os.path.join(out, "h.o")
        j = os.path.join(out, "j.o")
        write_rtc_source()
        subprocess.run([HIPCC, "-c", *flags, *SAN_HOST, os.path.join(CSRC, "frbx_jit.cpp"), "-o", j],
                       check=True, capture_output=True)
        subprocess.run([HIPCC, "-c", *flags, *SAN_HOST, os.path.join(CSRC, "frbx_kernels.hip"), "-o", k],
                       check=True, capture_output=True)
        subprocess.run([HIPCC, "-c", *flags, "-ffp-contract=off", *SAN_HOST,
                        os.path.join(CSRC, "frbx_host.cpp"), "-o", h], check=True, capture_output=True)
        tmp = lib + ".tmp"
        subprocess.run([HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", k, h, j, "-lhiprtc", "-o", tmp],
                       check=True, capture_output=True)
        os.replace(tmp, lib)
    return out


def _run_c(san_lib, src, tmp_path):
    exe = tmp_path / os.path.basename(src).replace(".c", "")
    subprocess.run([CLANG, "-std=c11", "-g", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", INC, src,
                    "-L", san_lib, "-lfrbx", f"-Wl,-rpath,{san_lib}", "-lm", "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=ENV)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    return r.stdout


def test_c_abi_program_is_clean_under_asan_and_ubsan(san_lib, tmp_path):
    out = _run_c(san_lib, os.path.join(ROOT, "tests", "c_abi_check.c"), tmp_path)
    lines = {ln.split()[0]: ln.split()[1:] for ln in out.splitlines()}
    assert lines["detections"] == ["2", "groups", "1", "reported", "1"]


def test_randomised_host_calls_are_clean_under_asan_and_ubsan(san_lib, tmp_path):
    out = _run_c(san_lib, os.path.join(ROOT, "tests", "c_host_fuzz.c"), tmp_path)
    assert out.startswith("fuzz ok")
