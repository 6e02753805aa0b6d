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


def _counter_db(path, counter, per_step, copy_kib, n_steps=40):
    """A stand-in rocprofv3 database: the step dispatches of the Smagorinsky
    model alternate even/odd, then the 1 GiB calibration copy."""
    import sqlite3
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    d = 1
    for n in range(n_steps):
        par = n % 2
        name = f"void lbmsc::(anonymous namespace)::k_step<128, 1, {'true' if par == 0 else 'false'}, 1, {par}>" \
               "(lbmsc::Geo const*, int const*, int, lbmsc::StepArgs, int*)"
        con.execute("insert into counters_collection values (?, ?, ?, ?)", (d, name, counter, per_step[par]))
        d += 1
        # another model's step and an unrelated kernel in between are ignored
        con.execute("insert into counters_collection values (?, ?, ?, ?)",
                    (d, "void lbmsc::(anonymous namespace)::k_step<128, 1, true, 0, 0>(x)", counter, 1.0))
        d += 1
    con.execute("insert into counters_collection values (?, ?, ?, ?)", (d, "__amd_rocclr_copyBuffer", counter, copy_kib))
    con.commit()
    con.close()


def test_traffic_summary_scales_by_the_calibration_copy(tmp_path):
    """HBM bytes per launch = mean over parities of (fetch + write), each
    counter scaled so that the 1 GiB copy reads 1 GiB."""
    f, w = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    _counter_db(f, "FETCH_SIZE", (1000.0, 1100.0), 524288.0)      # FETCH_SIZE reads half the copy
    _counter_db(w, "WRITE_SIZE", (2000.0, 2300.0), 1048576.0)
    t = bench.summarize_traffic(f, w, first=4, count=20)
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    assert t["per_parity_bytes"]["even"] == [1000 * 2 * 1024, 2000 * 1024]
    assert t["per_parity_bytes"]["odd"] == [1100 * 2 * 1024, 2300 * 1024]
    assert t["hbm_bytes_per_launch"] == round(0.5 * 1024 * (2000 + 2000 + 2200 + 2300))
    assert t["launch_partial"] == {"block": 128, "cells_per_thread": 1}
    assert t["steps"] == [4, 23]
