#!/usr/bin/env python
"""Benchmark of the SC-LBM hot path on one MI355X.

One benchmark step is one full stochastic-collocation pass of the urban LES
ensemble workload: 13 Smolyak Clenshaw-Curtis nodes (level 2) of a
256x128x64 box with a seeded 6x4 building array, D3Q19 Smagorinsky
(Cs = 0.1) with a log-law inflow, 20000 time steps of all 13 nodes batched in
one plan (graph replay of step pairs), time averages of u and |u| over the
last 5000 states, then the FP64 quadrature mean and variance fields.
Inputs are synthetic and seeded; everything is resident in HBM.

Prints one JSON line: aggregate MLUPS over fluid cells (value), the
roofline of the collide-and-stream kernel (algorithmic 152 B per fluid cell
update against 8 TB/s), and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "aggregate MLUPS (batched vs one-at-a-time) + %HBM roofline; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_UPDATE = 152          # 19 FP32 populations read + written
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_collide_stream_urban_les.json")
# every source that shapes the step kernels' code: a change to any of them
# invalidates the committed counter summary
KERNEL_SRCS = [os.path.join(ROOT, "paper_2508_18202_amd", *p) for p in
               (("csrc", "device.h"), ("csrc", "steps.hip"), ("csrc", "kernels.h"), ("csrc", "rules.h"),
                ("csrc", "d3q19.h"), ("build.py",))]


def summarize_traffic(fetch_csv: str, write_csv: str, first: int, count: int) -> dict:
    """HBM bytes per collide-and-stream launch of the headline workload from
    two rocprofv3 --pmc runs of `bench.py ... --profile-calib` (FETCH_SIZE,
    then WRITE_SIZE; KiB per dispatch; the runs' results.db or counter CSV
    files): the step dispatches of the
    Smagorinsky model in dispatch order are the time steps of the headline
    pass (one dispatch per step), the medians over steps first ..
    first+count-1 per parity are scaled by what each counter reads for the
    1 GiB calibration copy at the end of the run."""
    import csv
    import re
    import statistics

    def load(path, counter):
        rows = {}
        if path.endswith(".db"):                  # rocprofv3's default (rocpd SQLite) output
            import sqlite3
            con = sqlite3.connect(path)
            q = "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?"
            for d, name, v in con.execute(q, (counter,)):
                rows[int(d)] = (name, float(v))
            con.close()
        else:                                     # --output-format csv
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter:
                        rows[int(r["Dispatch_Id"])] = (r["Kernel_Name"], float(r["Counter_Value"]))
        return [rows[k] for k in sorted(rows)]

    def steps_of(seq):
        out = []
        for name, v in seq:
            m = re.search(r"k_step<(\d+), (\d+), (true|false), (\d+), (\d+)>", name)
            if m and m.group(4) == "1":
                out.append((int(m.group(5)), v, {"block": int(m.group(1)), "cells_per_thread": int(m.group(2))}))
        return out

    res = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        seq = load(path, counter)
        copies = [v for name, v in seq if "copyBuffer" in name]
        factor = (1 << 20) / copies[-1]           # the 1 GiB calibration copy, in KiB
        all_steps = steps_of(seq)
        if len(all_steps) < first + count:
            raise SystemExit(f"{path}: {len(all_steps)} step dispatches, fewer than {first + count}")
        st = all_steps[first:first + count]
        res[key] = {par: statistics.median(v for p_, v, _ in st if p_ == par) * 1024 * factor for par in (0, 1)}
        res[key + "_factor"] = round(factor, 3)
        res[key + "_copy_kib"] = copies[-1]
        res["launch"] = st[0][2]
    hbm = 0.5 * (res["fetch"][0] + res["write"][0] + res["fetch"][1] + res["write"][1])
    return {"kernel_sha": kernel_sha(), "hbm_bytes_per_launch": int(round(hbm)),
            "fetch_factor": res["fetch_factor"], "write_factor": res["write_factor"],
            "calibration_copy_kib": {"fetch": res["fetch_copy_kib"], "write": res["write_copy_kib"]},
            "per_parity_bytes": {"even": [int(res["fetch"][0]), int(res["write"][0])],
                                 "odd": [int(res["fetch"][1]), int(res["write"][1])]},
            "steps": [first, first + count - 1], "launch_partial": res["launch"],
            "summary": "collide_stream_urban_les_hbm_traffic.md"}


def progress(msg: str):
    """One line per finished pass, leg or run on stderr (the JSON line alone
    goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed SC passes")
    ap.add_argument("--warmup", type=int, default=1, help="untimed SC passes")
    ap.add_argument("--lbm-steps", type=int, default=20000, help="time steps per pass")
    ap.add_argument("--avg-len", type=int, default=5000, help="QoI averaging window")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0: autotuned shape)")
    ap.add_argument("--cache-block", type=int, default=-1,
                    help="MiB per instance block of plain stretches (-1: the library default, 0: off)")
    ap.add_argument("--cells-per-thread", type=int, default=1)
    ap.add_argument("--model", default="smagorinsky", help=argparse.SUPPRESS)
    ap.add_argument("--nontemporal", type=int, default=1, help="mask: 1 even steps, 2 odd steps")
    ap.add_argument("--xcd-order", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward cost leg")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="run length of the adjoint/forward cost legs (objective over the last quarter)")
    ap.add_argument("--no-rr3", action="store_true",
                    help="skip the regularised-collision, series-inflow and Gauss-Hermite/gPC legs")
    ap.add_argument("--no-uneven", action="store_true", help="skip the batched vs one-at-a-time leg")
    ap.add_argument("--no-cylinder", action="store_true", help="skip the paper-size cylinder leg")
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="time budget of the urban LES samples of the CPU baseline")
    ap.add_argument("--assimilation-iters", type=int, default=0,
                    help="also run the data-assimilation configuration at its size for this many "
                         "gradient-descent iterations (about 100 s each; 0 = skip)")
    ap.add_argument("--only-assimilation", action="store_true",
                    help="skip the headline pass and every other leg (with --assimilation-iters)")
    ap.add_argument("--no-small", action="store_true", help="skip the small block-case leg")
    ap.add_argument("--ramp", type=int, default=None,
                    help="inflow ramp length of the headline pass (profiling runs; default: the workload's 1000)")
    ap.add_argument("--box", type=int, nargs=3, metavar=("NX", "NY", "NZ"), help=argparse.SUPPRESS)
    ap.add_argument("--faces", nargs=6, help=argparse.SUPPRESS)
    ap.add_argument("--no-buildings", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary of two rocprofv3 counter runs and exit (no GPU)")
    ap.add_argument("--profile-calib", action="store_true",
                    help="also run a plain copy of known size (HBM counter calibration)")
    return ap.parse_args()


def kernel_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(launch_bytes_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary and
    the launch shape the counters were taken in, if they were taken on the
    current kernel source; else (None, None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("kernel_sha") != kernel_sha():
        return None, None
    return t.get("hbm_bytes_per_launch"), t.get("launch")


def _host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, solid, theta, seconds: float):
    """The FP64 oracle as it stands, timed on the host on bounded samples of
    the workloads: the headline urban LES case (one node; on every thread the
    process may use and on one thread), the small block case in full, one
    instance of each uneven box size, one node of the data-assimilation box,
    and one node of the adjoint case forward and backward.  MLUPS count fluid
    cells."""
    from oracle import oracle as orc
    from paper_2508_18202_amd import inputs
    visible = len(os.sched_getaffinity(0))
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    threads = omp if omp > 0 else visible
    orc.set_threads(threads)
    used = orc.set_threads(0)

    def rate(case, n_fluid, step0, budget, max_steps, f=None):
        f = case.init() if f is None else f
        n = 0
        t0 = time.perf_counter()
        while True:
            f = case.step(step0 + n, f)
            n += 1
            dt = time.perf_counter() - t0
            if dt >= budget or n >= max_steps:
                break
        return n_fluid * n / dt / 1e6, n, dt

    fluid = int((solid == 0).sum())
    case = orc.Case.from_workload(w, solid, theta)
    v_all, n_all, t_all = rate(case, fluid, 1000, 0.5 * seconds, 400)
    orc.set_threads(1)
    v_one, n_one, t_one = rate(case, fluid, 1000, 0.25 * seconds, 100)
    orc.set_threads(threads)
    legs = {"urban_les_one_thread": {"value": round(v_one, 2), "unit": "MLUPS", "threads": 1,
                                     "sample": f"1 of 13 nodes, {n_one} steps past the ramp, {t_one:.1f} s"}}
    # small block case in full: 5 Gauss-Legendre nodes x 1000 steps
    sb = inputs.small_block()
    sbs = inputs.solid_mask(sb)
    xs, _ = orc.collocation(sb)
    t0 = time.perf_counter()
    for xi in xs:
        orc.run(orc.Case.from_workload(sb, sbs, orc.node_params(sb, xi)), sb.steps)
    dt = time.perf_counter() - t0
    legs["small_block_full"] = {"value": round(len(xs) * int((sbs == 0).sum()) * sb.steps / dt / 1e6, 2),
                                "unit": "MLUPS", "threads": used,
                                "sample": f"all 5 nodes x 1000 steps (the whole case), {dt:.2f} s"}
    # one instance per uneven box size
    tot, tt = 0, 0.0
    seen = set()
    for uw in inputs.uneven_cases():
        if (uw.nx, uw.ny, uw.nz) in seen:
            continue
        seen.add((uw.nx, uw.ny, uw.nz))
        us = inputs.solid_mask(uw)
        xu, _ = orc.collocation(uw)
        r, n, dt = rate(orc.Case.from_workload(uw, us, orc.node_params(uw, xu[0])), int((us == 0).sum()), 1000,
                        0.05 * seconds, 20)
        tot += int((us == 0).sum()) * n
        tt += dt
    legs["uneven_one_per_size"] = {"value": round(tot / tt / 1e6, 2), "unit": "MLUPS", "threads": used,
                                   "sample": "1 instance of each of 128x64x32, 192x96x48, 256x128x64, "
                                             f"up to 20 steps each, {tt:.1f} s"}
    # data-assimilation box: one node, a few steps
    aw = inputs.assimilation_case()
    asol = inputs.solid_mask(aw)
    xa, _ = orc.collocation(aw)
    r, n, dt = rate(orc.Case.from_workload(aw, asol, orc.node_params(aw, xa[0])), int((asol == 0).sum()), 1000,
                    0.1 * seconds, 5)
    legs["assimilation_one_node"] = {"value": round(r, 2), "unit": "MLUPS", "threads": used,
                                     "sample": f"1 of 13 nodes of 512x256x128, {n} steps, {dt:.1f} s"}
    # adjoint case: one node, forward with snapshots and the checkpointed adjoint
    dw = inputs.adjoint_case(steps=20, avg_len=5)
    dsol = inputs.solid_mask(dw)
    probes = inputs.probe_cells(dw, dsol)
    xd, _ = orc.collocation(dw)
    dcase = orc.Case.from_workload(dw, dsol, orc.node_params(dw, xd[0]))
    dfl = int((dsol == 0).sum())
    t0 = time.perf_counter()
    orc.run(dcase, dw.steps, avg_start=dw.avg_start, probes=probes)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    orc.adjoint(dcase, dw.steps, dw.avg_start, probes, np.full(len(probes), 1.0 / len(probes)), ckpt=dw.steps)
    t_adj = time.perf_counter() - t0
    legs["adjoint_case_one_node"] = {"forward_mlups": round(dfl * dw.steps / t_fwd / 1e6, 2),
                                     "adjoint_mlups": round(dfl * dw.steps / t_adj / 1e6, 2),
                                     "adjoint_vs_forward": round(t_adj / t_fwd, 2), "threads": used,
                                     "sample": f"1 of 13 nodes of 128x64x48, {dw.steps} steps forward, then the "
                                               f"adjoint (forward re-run from the snapshot included), "
                                               f"{t_fwd:.1f} s + {t_adj:.1f} s"}
    return {"value": round(v_all, 2), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"FP64 oracle (gcc -O2, OpenMP, {used} threads: the CPU share this process may use), "
                      f"1 of 13 nodes of the 256x128x64 urban LES case, {n_all} time steps past the inflow ramp, "
                      f"{t_all:.1f} s",
            "host": {"cpu": _host_cpu(), "logical_cpus_visible": visible, "logical_cpus_total": os.cpu_count()},
            "configs": legs}


def copy_ceiling(nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Read + write rate of a plain device-to-device copy on this GPU (GB/s)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del src, dst
    return 2 * nbytes / best / 1e9


def _after_ramp_rate(w, variant, steps: int, label: str):
    """Step-pair launch time of the 13 nodes of workload w, timed with events
    over `steps` steps after the inflow ramp."""
    import torch
    from paper_2508_18202_amd import sc
    from paper_2508_18202_amd import inputs
    solid = inputs.solid_mask(w)
    n_fluid = int((solid == 0).sum())
    x, a, th = sc.collocation(w)
    cg = sc.make_geometry(w, solid)
    ens = sc.Ensemble([cg], [th], use_graph=True, variant=variant)
    try:
        ens.advance(w.ramp)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ens.advance(steps)
        e1.record()
        e1.synchronize()
        if ens.health() >= 0:
            raise RuntimeError(f"{label} leg went unstable")
        t = e0.elapsed_time(e1) / 1e3 / steps
        launch_bytes = BYTES_PER_CELL_UPDATE * len(ens) * n_fluid
        return {"avg_launch_us": round(t * 1e6, 2), "kernel_mlups": round(len(ens) * n_fluid / t / 1e6, 1),
                "achieved_gbs": round(launch_bytes / t / 1e9, 1),
                "frac": round(launch_bytes / t / 1e9 / HBM_PEAK_GBS, 4)}
    finally:
        ens.close()


def rr3_leg(variant, steps: int = 1000):
    """The regularised third-order collision (with the Smagorinsky tau_eff) on
    the same 13-node urban batch."""
    from paper_2508_18202_amd import inputs
    w = inputs.scaled(inputs.urban_les(), 256, 128, 64, model="rr3")
    out = {"workload": "13 Smolyak nodes x 256x128x64 urban LES, regularised third-order collision, "
                       f"Smagorinsky Cs=0.1, {steps} steps after the ramp"}
    out.update(_after_ramp_rate(w, variant, steps, "regularised"))
    return out


def series_leg(variant, steps: int = 1000):
    """The same batch driven by an hourly wind series (four 250-step hours with
    100-step blends after the ramp): the in-kernel series evaluation."""
    from paper_2508_18202_amd import inputs
    w = inputs.urban_series(hours=4, hour_steps=250, blend_steps=100)
    out = {"workload": "13 Smolyak nodes x 256x128x64 urban LES, Smagorinsky Cs=0.1, hourly-series inflow "
                       f"(hours of 250 steps, blends of 100), {steps} steps after the ramp"}
    out.update(_after_ramp_rate(w, variant, steps, "series"))
    return out


def gauss_hermite_leg(variant, steps: int = 300, avg_len: int = 100):
    """The paper's stochastic set-up at its node count: 121 Gauss-Hermite
    nodes (11 x 11) of a 128x64x48 urban box with the hourly-series inflow,
    stepped in one plan; then the order-5 gPC expansion of the time-averaged
    fields (21 coefficients, variance and 95 % band per value).  Without a
    given launch shape the autotuner picks one on this batch (its 128-cell
    rows put boundary lanes in every wavefront, so its best shape differs
    from the headline box's)."""
    import torch
    from paper_2508_18202_amd import inputs, sc
    from paper_2508_18202_amd import lbmsc as L
    w = inputs.scaled(inputs.urban_gpc(hours=4, hour_steps=100, blend_steps=30), 128, 64, 48, ramp=100,
                      ref_height=48.0)
    solid = inputs.solid_mask(w)
    n_fluid = int((solid == 0).sum())
    x, a, th = sc.collocation(w)
    cg = sc.make_geometry(w, solid)
    total = w.ramp + steps
    if variant is None:
        tune = sc.Ensemble([cg], [th], use_graph=False)
        variant = tuple(L.lbm_plan_autotune(tune.plan, sc.stream_handle()))
        tune.close()
    ens = sc.Ensemble([cg], [th], avg_begin=total - avg_len, avg_end=total, use_graph=True, variant=variant)
    try:
        ens.advance(w.ramp)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ens.advance(steps - avg_len)
        e1.record()
        ens.advance(avg_len)
        if ens.health() >= 0:
            raise RuntimeError("Gauss-Hermite leg went unstable")
        t_step = e0.elapsed_time(e1) / 1e3 / (steps - avg_len)
        q = torch.empty(len(ens), cg.ncells, 4, dtype=torch.float32, device="cuda")
        for j in range(len(ens)):
            ens.averages_into(j, q[j])
        sc.gpc(q, x, a, 5)                             # warm-up
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record()
        r = sc.gpc(q, x, a, 5)
        g1.record()
        g1.synchronize()
        t_gpc = g0.elapsed_time(g1) / 1e3
        n_el = q[0].numel()
        P = r["coef"].shape[0]
        gpc_bytes = n_el * (len(ens) * 4 + P * 8 + 8 + 16)
        launch_bytes = BYTES_PER_CELL_UPDATE * len(ens) * n_fluid
        return {"workload": "121 Gauss-Hermite nodes (11 x 11) x 128x64x48 urban LES, hourly-series inflow, "
                            f"{steps - avg_len} timed steps; order-5 gPC of the time-averaged fields",
                "instances": len(ens),
                "launch": dict(zip(("block", "cells_per_thread", "nontemporal", "xcd_order"), map(int, variant))),
                "step_us": round(t_step * 1e6, 2),
                "kernel_mlups": round(len(ens) * n_fluid / t_step / 1e6, 1),
                "frac": round(launch_bytes / t_step / 1e9 / HBM_PEAK_GBS, 4),
                "gpc_terms": P, "gpc_elements": n_el, "gpc_ms": round(t_gpc * 1e3, 3),
                "gpc_gbs": round(gpc_bytes / t_gpc / 1e9, 1),
                "gpc_fp64_gflops": round(2.0 * n_el * len(ens) * P / t_gpc / 1e9, 1)}
    finally:
        ens.close()


def cylinder_leg(variant, steps: int = 40, warm: int = 6, max_nodes: int = 121):
    """The paper's domain class at its size: a cylinder of radius 270 and
    height 40 cells (1 m cells; box 544 x 544 x 40, 9.04 M fluid cells) whose
    mantle carries an hourly-series wind, two central blocks, Smagorinsky LES;
    the 121 Gauss-Hermite nodes (11 x 11) in one plan when HBM holds them
    (about 0.9 GB each), else as many as fit; probe-line sums accumulated over
    the timed steps.  Without a given launch shape the autotuner picks one on
    four nodes of the same geometry."""
    import torch
    from paper_2508_18202_amd import inputs, sc
    from paper_2508_18202_amd import lbmsc as L
    w = inputs.cylinder_gpc()
    solid = inputs.solid_mask(w)
    n_fluid = int((solid == 0).sum())
    x, a, th = sc.collocation(w)
    probes = inputs.probe_cells(w, solid)
    cg = sc.make_geometry(w, solid, probes)
    per_inst = 19 * cg.qs * 4 + 16 * len(probes)
    free, _ = torch.cuda.mem_get_info()
    k = int(max(1, min(max_nodes, len(th), (free - (16 << 30)) // per_inst)))
    if variant is None:
        # launch shape tuned on four nodes of the same geometry (cached per box size)
        small = sc.Ensemble([cg], [th[:4]], use_graph=False)
        variant = tuple(L.lbm_plan_autotune(small.plan, sc.stream_handle()))
        small.close()
    ens = sc.Ensemble([cg], [th[:k]], avg_begin=warm, avg_end=warm + steps, fields=False,
                      use_graph=True, variant=variant)
    try:
        ens.advance(warm)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ens.advance(steps)
        e1.record()
        e1.synchronize()
        if ens.health() >= 0:
            raise RuntimeError("cylinder leg went unstable")
        t = e0.elapsed_time(e1) / 1e3 / steps
        launch_bytes = BYTES_PER_CELL_UPDATE * k * n_fluid
        # the paper's output: order-5 gPC of the probe-line averages over all
        # nodes (needs the whole rule), mean and 95 % band per probe
        gpc_ms = None
        if k == len(th):
            pq = torch.empty(k, len(probes), dtype=torch.float32, device="cuda")
            for j in range(k):
                ens.averages_into(j, None, pq[j])
            sc.gpc(pq, x, a, 5)
            torch.cuda.synchronize()
            g0 = torch.cuda.Event(enable_timing=True)
            g1 = torch.cuda.Event(enable_timing=True)
            g0.record()
            r = sc.gpc(pq, x, a, 5)
            g1.record()
            g1.synchronize()
            gpc_ms = round(g0.elapsed_time(g1), 3)
            if not bool(torch.isfinite(r["band"]).all()):
                raise RuntimeError("cylinder leg: non-finite gPC band")
        return {"workload": f"{k} of the 121 Gauss-Hermite nodes x cylinder r=270 h=40 (544x544x40 box), "
                            "mantle velocity condition with an hourly-series wind, Smagorinsky Cs=0.1, "
                            f"probe lines, {steps} timed steps; order-5 gPC of the probe-line averages",
                "probes": int(len(probes)), "gpc_ms": gpc_ms,
                "instances": k, "fluid_cells_per_instance": n_fluid,
                "fluid_fraction_of_box": round(n_fluid / cg.ncells, 4),
                "launch": {"block": variant[0], "cells_per_thread": variant[1], "nontemporal": variant[2],
                           "xcd_order": variant[3]},
                "step_ms": round(t * 1e3, 3),
                "kernel_mlups": round(k * n_fluid / t / 1e6, 1),
                "frac": round(launch_bytes / t / 1e9 / HBM_PEAK_GBS, 4),
                "hbm_gib_populations": round(k * 19 * cg.qs * 4 / 2 ** 30, 1)}
    finally:
        ens.close()


def adjoint_leg(variant, steps: int = 2000, avg_len: int = 500, ckpt: int = 100, model: str = "bgk"):
    """Cost of the gradient against a plain forward run on the adjoint
    workload (13 Smolyak nodes of 128x64x48, BGK, Smagorinsky or the
    regularised collision, probe-plane QoI): the adjoint driver's forward
    run (with snapshots, or recording every step when those records fit in
    device memory) and its reverse sweep, timed against the same forward
    run without either; ratio = (driver's forward - plain forward + sweep) /
    plain forward."""
    import torch
    from paper_2508_18202_amd import inputs, sc
    from paper_2508_18202_amd.adjoint import CheckpointedAdjoint
    w = inputs.adjoint_case(steps=steps, avg_len=avg_len)
    if model != "bgk":
        w = inputs.scaled(w, w.nx, w.ny, w.nz, model=model, cs=0.1)
    solid = inputs.solid_mask(w)
    probes = inputs.probe_cells(w, solid)
    x, a, th = sc.collocation(w)
    cg = sc.make_geometry(w, solid, probes)
    ens = sc.Ensemble([cg], [th], avg_begin=w.avg_start, avg_end=w.steps, fields=False,
                      use_graph=True, variant=variant)
    try:
        run = CheckpointedAdjoint(ens, steps, ckpt)
        pw = [torch.full((len(probes),), 1.0 / len(probes), dtype=torch.float64, device="cuda")] * len(ens)
        run.forward()
        run.backward(pw)                       # warm-up
        ens.reset()
        torch.cuda.synchronize()
        tp = time.perf_counter()
        ens.advance(steps)                     # the plain forward run
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - tp
        t0 = time.perf_counter()
        run.forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = run.backward(pw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fluid = int((solid == 0).sum())
        # per-step kernel ratio: the adjoint steps of the first segment (its
        # records are still in place) against plain forward steps
        from paper_2508_18202_amd import lbmsc as L
        s = sc.stream_handle()
        k = len(ens)
        lam_ptr = [[t.data_ptr() for t in run.lam[b][:k]] for b in range(1 if run.inplace else 2)]
        rec_ptr = [t.data_ptr() for t in run.rec[:k]]
        pw_ptr = [p.data_ptr() for p in pw]
        g2 = torch.zeros(k, 3, dtype=torch.float64, device="cuda")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for n in range(ckpt - 1, -1, -1):
            if run.inplace:
                L.lbm_adjoint_step_inplace(ens.plan, n, lam_ptr[0], rec_ptr, run.kind, ckpt, pw_ptr,
                                           g2.data_ptr(), s)
            else:
                L.lbm_adjoint_step(ens.plan, n, lam_ptr[(n + 1) % 2], lam_ptr[n % 2], rec_ptr, run.kind, ckpt,
                                   pw_ptr, g2.data_ptr(), s)
        e1.record()
        e1.synchronize()
        t_adj = e0.elapsed_time(e1) / 1e3 / ckpt
        ens.reset()
        e0.record()
        ens.advance(ckpt)
        e1.record()
        e1.synchronize()
        t_fwd = e0.elapsed_time(e1) / 1e3 / ckpt
        coll = {"bgk": "BGK tau 0.6",
                "smagorinsky": "Smagorinsky Cs=0.1, tau0 0.6",
                "rr3": "regularised third-order collision, Smagorinsky Cs=0.1, tau0 0.6"}[model]
        gcpu = g.cpu().numpy()
        grads = {str(j): [float(v) for v in gcpu[j]] for j in (2, 10)}
        vs_oracle = None
        gold = os.path.join(ROOT, "tests", "golden", "adjoint_case_gradient.json")
        if model == "bgk" and steps == 2000 and ckpt == 100 and os.path.exists(gold):
            with open(gold) as fh:
                ref = json.load(fh)
            idx = [nd["index"] for nd in ref["nodes"]]
            go = np.asarray([nd["grad"] for nd in ref["nodes"]])
            gg = np.asarray([gcpu[j] for j in idx])
            # per parameter k: max_j |g_jk - g_oracle_jk| / max_j |g_oracle_jk|
            vs_oracle = {"nodes": idx,
                         "per_parameter": [float(np.abs(gg[:, k] - go[:, k]).max() / np.abs(go[:, k]).max())
                                           for k in range(3)]}
        mode = ("every step recorded by the forward run" if run.store_all else
                f"the last {run.stored} steps recorded by the forward run, the {run.head} before in "
                f"segments of {ckpt} re-run from snapshots with recording")
        return {"workload": f"13 Smolyak nodes x 128x64x48 {coll}, log-law inflow, probe plane, "
                            f"{steps} steps, objective over the last {avg_len}",
                "sweep": mode,
                "forward_s": round(t_plain, 4), "driver_forward_s": round(t1 - t0, 4),
                "adjoint_s": round(t2 - t1, 4),
                "ratio": round((t1 - t0 - t_plain + t2 - t1) / t_plain, 3),
                "forward_mlups": round(len(ens) * fluid * steps / t_plain / 1e6, 1),
                "adjoint_step_us": round(t_adj * 1e6, 1), "forward_step_us": round(t_fwd * 1e6, 1),
                "kernel_ratio": round(t_adj / t_fwd, 3),
                "lambda_buffers": "one, in place" if run.inplace else "two",
                "record": {1: "(rho, u), 16 B per cell", 2: "populations, 76 B per cell",
                           3: "regularised state, 64 B per cell"}[run.kind],
                "grad_finite": bool(torch.isfinite(g).all()),
                "grad_nodes": grads,
                "grad_rel_err_vs_stored_oracle": vs_oracle}
    finally:
        ens.close()


def small_block_leg():
    """The small SC-LBM case in full: 5 Gauss-Legendre nodes of the 32x16x16
    BGK block case, 1000 steps, final fields and FP64 moments; the stepping
    of the 5 nodes in one plan (graph replay) against one plan per node (one
    launch per node per step).  3 MB of populations: cache-resident, so no
    roofline figure."""
    import torch
    from paper_2508_18202_amd import inputs, sc
    from paper_2508_18202_amd import lbmsc as L
    w = inputs.small_block()
    solid = inputs.solid_mask(w)
    fluid = int((solid == 0).sum())
    x, a, th = sc.collocation(w)
    cg = sc.make_geometry(w, solid)

    def sc_pass():
        x, a, th = sc.collocation(w)
        ens = sc.Ensemble([cg], [th], use_graph=True)
        try:
            ens.advance(w.steps)
            q = torch.stack([ens.fields(j) for j in range(len(ens))])
            mean, var = sc.moments(q, a)
            if ens.health() >= 0:
                raise RuntimeError("small block leg went unstable")
            return mean
        finally:
            ens.close()

    sc_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sc_pass()
    torch.cuda.synchronize()
    t_pass = time.perf_counter() - t0
    ens = sc.Ensemble([cg], [th], use_graph=True)
    try:
        ens.advance(w.steps)
        ens.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.advance(w.steps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        plans = [L.lbm_plan_create([inst], use_graph=True) for inst in ens.instances]
        stream = sc.stream_handle()
        for p_ in plans:
            L.lbm_collide_stream(p_, 2, stream)
            L.lbm_plan_set_step(p_, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p_ in plans:
            L.lbm_collide_stream(p_, w.steps, stream)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        for p_ in plans:
            L.lbm_plan_destroy(p_)
    finally:
        ens.close()
    n = len(th)
    return {"workload": "5 Gauss-Legendre nodes x 32x16x16 D3Q19 BGK tau 0.6, one 6x6x8 block, uniform inflow "
                        "0.05 (1 + 0.1 xi), 1000 steps, final fields and FP64 moments",
            "sc_pass_ms": round(t_pass * 1e3, 2),
            "sc_pass_mlups": round(n * fluid * w.steps / t_pass / 1e6, 1),
            "batched_mlups": round(n * fluid * w.steps / tb / 1e6, 1),
            "one_at_a_time_mlups": round(n * fluid * w.steps / ts / 1e6, 1),
            "speedup": round(ts / tb, 3)}


def uneven_leg(variant, steps: int = 96, warm: int = 32):
    """The 48 uneven cases x 13 nodes (624 instances) advanced in one plan vs
    the same instances advanced one at a time (a plan per instance, each run
    through all of its steps before the next starts), both with graph replay,
    on plain steps (the cases without their inflow ramp: the same kernels,
    and graph replay covers every step)."""
    import torch
    from paper_2508_18202_amd import inputs, sc
    from paper_2508_18202_amd import lbmsc as L
    cases = [inputs.scaled(w, w.nx, w.ny, w.nz, ramp=0) for w in inputs.uneven_cases(steps=steps)]
    cgs, ths, fluid = [], [], 0
    for w in cases:
        s = inputs.solid_mask(w)
        cgs.append(sc.make_geometry(w, s))
        ths.append(sc.collocation(w)[2])
        fluid += 13 * int((s == 0).sum())
    ens = sc.Ensemble(cgs, ths, use_graph=True, variant=variant)
    try:
        ens.advance(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.advance(steps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        # one plan per instance over the batch's own population arrays
        plans = []
        stream = sc.stream_handle()
        for k, inst in enumerate(ens.instances):
            plans.append(L.lbm_plan_create([inst], use_graph=True, block=variant[0],
                                           cells_per_thread=variant[1], nontemporal=variant[2],
                                           xcd_order=variant[3]))
            L.lbm_plan_set_step(plans[-1], ens.step)
            L.lbm_collide_stream(plans[-1], warm, stream)      # graph capture, untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in plans:
            L.lbm_collide_stream(p, steps, stream)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        for p in plans:
            L.lbm_plan_destroy(p)
        return {"workload": "48 cases (16 each of 128x64x32, 192x96x48, 256x128x64) x 13 nodes = "
                            f"{len(ens)} instances, {steps} plain steps after {warm}, graph replay",
                "batched_mlups": round(fluid * steps / tb / 1e6, 1),
                "one_at_a_time_mlups": round(fluid * steps / ts / 1e6, 1),
                "speedup": round(ts / tb, 3)}
    finally:
        ens.close()


def assimilation_leg(iters: int):
    """The data-assimilation configuration at its size: 13 Smolyak nodes of
    the 512x256x128 Smagorinsky box (10x6 buildings, 16.8 M cells each), 64
    probes, 2000 steps per forward run with the objective over the last 500,
    observations from the hidden truth with 5 % noise, then `iters`
    gradient-descent iterations (Armijo backtracking) through the
    checkpointed adjoint, one node per reverse sweep (group_size 1: snapshots
    every 100 steps and 100 recorded population states of one node)."""
    import torch
    from paper_2508_18202_amd import inputs
    from paper_2508_18202_amd.assimilation import Assimilation
    w = inputs.assimilation_case()
    t0 = time.perf_counter()
    da = Assimilation(w, w.steps, w.steps - w.avg_start, ckpt=100, group_size=1)
    t_setup = time.perf_counter() - t0
    try:
        fwd, bwd = [], []
        run_f, run_b = da.runner.forward, da.runner.backward

        def timed_forward():
            t = time.perf_counter()
            r = run_f()
            torch.cuda.synchronize()
            fwd.append(time.perf_counter() - t)
            progress(f"assimilation forward run {len(fwd)}: {fwd[-1]:.1f} s")
            return r

        def timed_backward(pw):
            t = time.perf_counter()
            r = run_b(pw)
            torch.cuda.synchronize()
            bwd.append(time.perf_counter() - t)
            progress(f"assimilation reverse sweep {len(bwd)}: {bwd[-1]:.1f} s")
            return r

        da.runner.forward, da.runner.backward = timed_forward, timed_backward
        n_probes = len(da.ens.cases[0].probes)
        t0 = time.perf_counter()
        da.observe(inputs.da_truth(), inputs.da_noise(2 * n_probes))
        t_obs = time.perf_counter() - t0
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        hist = da.run(inputs.da_start(), iters)
        t_run = time.perf_counter() - t0
        peak = torch.cuda.max_memory_allocated()
        free, total = torch.cuda.mem_get_info()
        fluid = int((inputs.solid_mask(w) == 0).sum())
        return {"workload": "13 Smolyak nodes x 512x256x128 D3Q19 Smagorinsky Cs=0.1, 10x6 buildings, log-law inflow, "
                            "64 probes, 2000 steps per forward run (objective over the last 500), snapshots every 100, "
                            "one node per reverse sweep",
                "iterations": len(hist), "setup_s": round(t_setup, 1), "observe_s": round(t_obs, 1),
                "run_s": round(t_run, 1), "s_per_iteration": round(t_run / max(1, len(hist)), 1),
                "forward_runs_s": [round(v, 2) for v in fwd], "backward_runs_s": [round(v, 2) for v in bwd],
                "forward_mlups": round(13 * fluid * w.steps / min(fwd) / 1e6, 1) if fwd else None,
                "history": hist,
                "peak_torch_gib": round(peak / 2 ** 30, 1),
                "device_used_gib": round((total - free) / 2 ** 30, 1)}
    finally:
        da.close()


def main():
    args = parse()
    if args.summarize_traffic:
        # the plain stretch of the headline pass the counter runs took,
        # from the same flags: steps after the ramp, before the QoI window
        ramp = 1000 if args.ramp is None else args.ramp
        first = ramp + 16
        count = (args.lbm_steps - min(args.avg_len, args.lbm_steps)) - 16 - first
        t = summarize_traffic(*args.summarize_traffic, first=first, count=count - count % 2)
        t["algorithmic_bytes_per_launch"] = BYTES_PER_CELL_UPDATE * 13 * 1942272
        # the launch shape the counter runs were given
        t["launch"] = {"block": args.block, "cells_per_thread": args.cells_per_thread,
                       "nontemporal": args.nontemporal, "xcd_order": args.xcd_order}
        assert (t["launch"]["block"], t["launch"]["cells_per_thread"]) == \
            (t["launch_partial"]["block"], t["launch_partial"]["cells_per_thread"]), "launch shape mismatch"
        del t["launch_partial"]
        print(json.dumps(t, indent=1))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(instances would shard across GPUs with no communication during stepping).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2508_18202_amd import inputs, sc
    from paper_2508_18202_amd import lbmsc as L

    torch.cuda.set_device(0)
    if args.only_assimilation:
        print(json.dumps({"assimilation": assimilation_leg(max(1, args.assimilation_iters))}), flush=True)
        return
    lbm_steps = args.lbm_steps
    w = inputs.urban_les(steps=lbm_steps, avg_len=min(args.avg_len, lbm_steps))
    if args.model != w.model:        # experiments only: the workload is Smagorinsky
        w = inputs.scaled(w, w.nx, w.ny, w.nz, model=args.model, tau0=0.6, cs=0.0)
    if args.ramp is not None:        # profiling runs: a short ramp before the plain stretch
        w = inputs.scaled(w, w.nx, w.ny, w.nz, ramp=args.ramp)
    # experiments only (traffic studies): another box, other faces, no buildings
    if args.box:
        w = inputs.scaled(w, *args.box)
    if args.faces:
        w = inputs.scaled(w, w.nx, w.ny, w.nz, faces=tuple(args.faces))
    solid = np.zeros((w.nz, w.ny, w.nx), np.uint8) if args.no_buildings else inputs.solid_mask(w)
    n_fluid = int((solid == 0).sum())
    ramp = min(w.ramp, w.avg_start)
    plain = max(0, w.avg_start - ramp)
    plain -= plain % 16
    # launch shape (block, cells per thread, non-temporal) from the project's
    # autotuner, cached per architecture / model / box sizes
    if args.block:
        variant = (args.block, args.cells_per_thread, args.nontemporal, args.xcd_order)
    else:
        x, a, th = sc.collocation(w)
        cg = sc.make_geometry(w, solid)
        ens = sc.Ensemble([cg], [th], use_graph=False)
        variant = L.lbm_plan_autotune(ens.plan, sc.stream_handle())
        ens.close()
        del ens, cg

    checks = {}

    blocks_used = {"n": 0}

    def sc_pass(timing, check=False, phases=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        x, a, th = sc.collocation(w)                       # collocation rule + node parameters
        cg = sc.make_geometry(w, solid)
        ens = sc.Ensemble([cg], [th], avg_begin=w.avg_start, avg_end=w.steps, use_graph=True, variant=variant,
                          cache_block=None if args.cache_block < 0 else args.cache_block << 20)
        blocks_used["n"] = L.lbm_plan_cache_blocks(ens.plan)    # geometry + rest state of all nodes
        try:
            ev[1].record()
            ens.advance(ramp)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            ens.advance(plain)                              # pure collide-and-stream launches
            e1.record()
            ens.advance(w.steps - ramp - plain)             # QoI window
            ev[2].record()
            q = torch.empty(len(ens), cg.ncells, 4, dtype=torch.float32, device="cuda")
            for j in range(len(ens)):
                ens.averages_into(j, q[j])
            ev[3].record()
            mean, var, nneg = sc.moments(q, a, count_negative=True)
            ev[4].record()
            bad = ens.health()
            if bad >= 0:
                raise RuntimeError(f"node {bad} went unstable")
            timing.append((e0, e1))
            if phases is not None:
                phases.append((ev, e0, e1))
            if check:
                last_q.update(q=q, a=a)
            if check:
                # invariants of the full-length run: finite fields and moments,
                # the mean density deviation of every node (sum of f - w over the
                # fluid cells, solid slots being zero), negative Smolyak variances
                drift = [float(ens.populations(j).sum(dtype=torch.float64)) / n_fluid for j in range(len(ens))]
                checks.update({
                    "fields_finite": bool(torch.isfinite(q).all()),
                    "moments_finite": bool(torch.isfinite(mean).all() and torch.isfinite(var).all()),
                    "mean_density_deviation_max": max(abs(d) for d in drift),
                    "negative_variance_count": int(nneg),
                    "negative_variance_fraction": round(int(nneg) / (4 * n_fluid), 6)})
            return mean, var, len(ens)
        finally:
            ens.close()

    for k in range(args.warmup):
        sc_pass([])
        progress(f"warm-up pass {k + 1}/{args.warmup}")
    torch.cuda.synchronize()
    timing = []
    phases = []
    last_q = {}
    t0 = time.perf_counter()
    for k in range(args.steps):
        mean, var, n_inst = sc_pass(timing, check=(k == args.steps - 1), phases=phases)
        progress(f"timed pass {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    updates = n_inst * n_fluid * lbm_steps * args.steps
    mlups = updates / elapsed / 1e6
    launches = plain
    kern_ms = [e0.elapsed_time(e1) / max(1, launches) for (e0, e1) in timing]
    avg_launch_s = float(np.mean(kern_ms)) / 1e3 if launches else float("nan")
    launch_bytes = BYTES_PER_CELL_UPDATE * n_inst * n_fluid
    achieved = launch_bytes / avg_launch_s / 1e9 if launches else float("nan")
    traffic, traffic_launch = load_traffic(launch_bytes)
    copy_gbs = copy_ceiling()
    props = torch.cuda.get_device_properties(0)
    # where a pass's time goes (HIP events on the launch stream, mean over the
    # timed passes): set-up (collocation, geometry, rest state), ramp, plain
    # steps, the QoI window (each step also reads and writes the FP32 partial
    # sums, +32 B per fluid cell, and every 64 states a flush into FP64), the
    # window averages, and the FP64 moments of the 13 x 4 x cells values
    win = w.steps - ramp - plain
    ph = np.mean([[ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(e0), e0.elapsed_time(e1),
                   e1.elapsed_time(ev[2]), ev[2].elapsed_time(ev[3]), ev[3].elapsed_time(ev[4])]
                  for ev, e0, e1 in phases], axis=0) if phases else np.full(6, float("nan"))
    n_el = 4 * int(np.prod(solid.shape))
    breakdown = {
        "setup_ms": round(float(ph[0]), 2), "ramp_ms": round(float(ph[1]), 2),
        "plain_ms": round(float(ph[2]), 2), "window_ms": round(float(ph[3]), 2),
        "averages_ms": round(float(ph[4]), 3), "moments_ms": round(float(ph[5]), 3),
        "window_launch_us": round(float(ph[3]) * 1e3 / max(1, win), 2),
        "window_gbs": round((BYTES_PER_CELL_UPDATE + 32) * n_inst * n_fluid / (float(ph[3]) / max(1, win) / 1e3) / 1e9, 1),
    }
    if last_q:
        # the moments kernel alone on the last pass's window averages (the
        # pass's moments phase also holds the count's copy to the host)
        qq, aa = last_q["q"], np.ascontiguousarray(last_q["a"], dtype=np.float64)
        mean_k = torch.empty(qq.shape[1:], dtype=torch.float64, device="cuda")
        var_k = torch.empty_like(mean_k)
        neg_k = torch.zeros(1, dtype=torch.int64, device="cuda")
        n_q, n_e = qq.shape[0], qq[0].numel()
        for rep_ in range(2):
            k0 = torch.cuda.Event(enable_timing=True)
            k1 = torch.cuda.Event(enable_timing=True)
            k0.record()
            for _ in range(20):
                L.lbm_sc_moments(qq.data_ptr(), aa, n_q, n_e, mean_k.data_ptr(), var_k.data_ptr(),
                                 neg_k.data_ptr(), sc.stream_handle())
            k1.record()
            k1.synchronize()
        t_k = k0.elapsed_time(k1) / 20 / 1e3
        breakdown["moments_kernel_us"] = round(t_k * 1e6, 1)
        breakdown["moments_kernel_gbs"] = round((n_q * 4 + 16) * n_e / t_k / 1e9, 1)
        del last_q["q"]

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "urban LES ensemble: 13 Smolyak CC level-2 nodes x 256x128x64 D3Q19 "
                        "Smagorinsky Cs=0.1, seeded 6x4 buildings, log-law inflow, "
                        f"{lbm_steps} steps, averages over the last {w.steps - w.avg_start}, FP64 moments",
            "lbm_steps": lbm_steps,
            "instances": n_inst,
            "fluid_cells_per_instance": n_fluid,
            "launch": {"block": variant[0], "cells_per_thread": variant[1], "nontemporal": variant[2],
                       "xcd_order": variant[3]},
            "cache_blocks": blocks_used["n"],
            "parallelism": "batched instances, 1 GPU",
            "device": {"name": props.name, "arch": getattr(props, "gcnArchName", ""),
                       "compute_units": props.multi_processor_count,
                       "hbm_gib": round(props.total_memory / 2 ** 30, 1)},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "collide_stream (even/odd in-place pair, Smagorinsky); a launch is one time step of the "
                      "batch (one dispatch per instance block when the plan uses cache blocks)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_launch": traffic_launch,
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "dispatches_per_launch": max(1, blocks_used["n"]),
            "algorithmic_bytes_per_launch": launch_bytes,
            "copy_ceiling": {"value": round(copy_gbs, 1), "unit": "GB/s",
                             "kernel": "hipMemcpyAsync device to device, 2 GiB, best of 5",
                             "frac": round(achieved / copy_gbs, 4)},
        },
        "kernel_mlups": round(n_inst * n_fluid / avg_launch_s / 1e6, 1),
        "pass_breakdown": breakdown,
        "invariants": checks,
    }

    def leg(name, fn, *a, **kw):
        t0 = time.perf_counter()
        r = fn(*a, **kw)
        r["wall_s"] = round(time.perf_counter() - t0, 1)
        out[name] = r
        progress(f"{name}: {r['wall_s']} s")
    if not args.no_small:
        leg("small_block", small_block_leg)
    if not args.no_rr3:
        leg("regularised_collision", rr3_leg, variant)
        leg("series_inflow", series_leg, variant)
        leg("gauss_hermite_gpc", gauss_hermite_leg, None if not args.block else variant)
    if not args.no_cylinder:
        leg("cylinder", cylinder_leg, None if not args.block else variant)
    if not args.no_adjoint:
        n_adj = args.adjoint_steps
        if n_adj < 200 or n_adj % 100:
            raise SystemExit("--adjoint-steps must be a multiple of 100, at least 200")
        leg("adjoint_vs_forward", adjoint_leg, variant, steps=n_adj, avg_len=n_adj // 4)
        leg("adjoint_vs_forward_smagorinsky", adjoint_leg, variant, steps=n_adj, avg_len=n_adj // 4,
            model="smagorinsky")
        leg("adjoint_vs_forward_regularised", adjoint_leg, variant, steps=n_adj, avg_len=n_adj // 4, model="rr3")
    if not args.no_uneven:
        leg("batched_vs_one_at_a_time", uneven_leg, variant)
    if args.assimilation_iters > 0:
        leg("assimilation", assimilation_leg, args.assimilation_iters)
    if not args.no_cpu:
        x, a, th = sc.collocation(w)
        leg("cpu_baseline", cpu_baseline, w, solid, th[0], args.cpu_seconds)
    if args.profile_calib:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * 4 * n
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
