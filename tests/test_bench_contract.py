"""Host-side checks of the measurement contract and of the product path's
refusal to run without the HIP library (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_profile_matches_the_kernel_sources():
    """The committed HBM-counter summary was taken on the current step-kernel
    sources, so the bench line reports its traffic (it reports null after
    any change to them until the counters are taken again)."""
    alg = 152 * 13 * 1942272
    t, launch = bench.load_traffic(alg)
    assert t is not None
    assert 1.0 < t / alg < 1.5
    assert set(launch) == {"block", "cells_per_thread", "nontemporal", "xcd_order"}


def test_binding_fails_loudly_without_the_library(tmp_path):
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2508_18202_amd import lbmsc as L\n"
        "L.LIB_PATH = %r\n"
        "try:\n"
        "    L.lib()\n"
        "except RuntimeError as e:\n"
        "    print('refused:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(1)\n" % (ROOT, str(tmp_path / "missing.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "no fallback" in r.stdout
