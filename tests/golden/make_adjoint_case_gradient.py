"""Writes adjoint_case_gradient.json: the FP64 oracle's inflow-parameter
gradients of the adjoint workload at its own horizon.

Workload (the adjoint configuration): 128x64x48 box with a seeded 4x3
building array, D3Q19 BGK tau 0.6, log-law inflow from rest without a ramp,
2000 steps, objective J = mean over the 32x16 probe plane (x = 96, solid
cells left out) of u_x averaged over the states (1500, 2000], snapshots every
100 steps.  For two of the 13 Smolyak nodes (the slowest node with the
direction +5 degrees and the fastest with -5 degrees), the oracle's discrete
adjoint gives dJ/d(u*, phi, z0) and its forward run the 512 probe averages.
The node parameters are rounded to FP32, the precision the library's
instance table holds them in, so that both sides run the same inflow.

Calls only oracle/ and the seeded input generators.  Takes about 20 min
per node on 8 cores: ``OMP_NUM_THREADS=8 python tests/golden/make_adjoint_case_gradient.py``.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc  # noqa: E402
from paper_2508_18202_amd import inputs  # noqa: E402

NODES = (2, 10)


def main():
    w = inputs.adjoint_case()
    solid = inputs.solid_mask(w)
    probes = inputs.probe_cells(w, solid)
    pw = np.full(len(probes), 1.0 / len(probes))
    x, a = orc.collocation(w)
    out = {"workload": w.name, "steps": w.steps, "avg_start": w.avg_start, "ckpt": w.ckpt_every,
           "probe_count": int(len(probes)), "probe_weights": "uniform 1/probe_count",
           "mask_sha256": inputs.mask_hash(solid), "nodes": []}
    for j in NODES:
        theta = np.asarray(orc.node_params(w, x[j]), dtype=np.float32).astype(np.float64)
        case = orc.Case.from_workload(w, solid, theta)
        t0 = time.time()
        g, _ = orc.adjoint(case, w.steps, w.avg_start, probes, pw, ckpt=w.ckpt_every)
        r = orc.run(case, w.steps, avg_start=w.avg_start, probes=probes)
        print(f"node {j}: grad {g}, J {float(np.dot(pw, r['probe'])):.9e}, {time.time() - t0:.0f} s", flush=True)
        out["nodes"].append({"index": j, "xi": [float(v) for v in x[j]], "theta": [float(v) for v in theta],
                             "grad": [float(v) for v in g], "J": float(np.dot(pw, r["probe"])),
                             "probe_avg": [float(v) for v in r["probe"]]})
    with open(os.path.join(HERE, "adjoint_case_gradient.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
