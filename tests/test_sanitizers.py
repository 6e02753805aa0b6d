"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code.

Two executables, built here with gcc / g++ (host code only, no GPU code):

* the FP64 oracle (``oracle/lbm_oracle.c``) under ``tests/sanitize/oracle_driver.c``:
  every exported routine on small cases that reach every boundary rule, every
  collision model and every inflow kind, the cylinder mantle included;
* the library's host code: the collocation rules and gPC basis
  (``csrc/quadrature.cpp``) and the kernels' link rules, flags, slot maps and
  in-place adjoint map evaluated on the host (``csrc/hostcheck.hip`` compiled
  as plain C++), under ``tests/sanitize/host_driver.cpp``.

Each must exit 0 with no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2508_18202_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-4000:]
    return report


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-std=c99", "-D_GNU_SOURCE", *SAN, os.path.join(HERE, "oracle_driver.c"),
                           "-lm", "-o", exe])
    assert "oracle sanitizer driver: ok" in _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the ROCm headers not available")
def test_host_code_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_asan")
    # the host checker is plain host C++: a copy under a .cpp name keeps this
    # host-only build apart from the HIP sources
    hc = str(tmp_path / "hostcheck_host.cpp")
    shutil.copyfile(os.path.join(CSRC, "hostcheck" + ".hip"), hc)
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{CSRC}",
                           os.path.join(HERE, "host_driver.cpp"), os.path.join(CSRC, "quadrature.cpp"), hc,
                           "-o", exe])
    assert "host sanitizer driver: ok" in _run(exe)
