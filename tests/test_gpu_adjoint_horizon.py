"""The adjoint configuration at its own horizon against the FP64 oracle.

13 Smolyak nodes of the 128x64x48 BGK case with the 4x3 building array and
the log-law inflow, 2000 steps from rest, objective J = mean of u_x over the
probe plane and the states (1500, 2000], snapshots every 100 steps: the
checkpointed GPU adjoint (both lambda layouts) in the bench's launch shape,
against the oracle's discrete adjoint of two nodes stored by
tests/golden/make_adjoint_case_gradient.py (the oracle alone takes about 20
minutes per node on 8 cores).

Tolerances at this horizon follow from the measured drift of the FP32
state: on this machine the velocity fields leave the FP64 ones by 5e-6 (250
steps), 1.1e-5 (500), 3.2e-5 (1000) relative, and the objective, a mean of
u_x over a plane where the flow changes sign, is a small difference of
values about twenty times larger, which amplifies that drift (probe
averages 3.3e-4 relative L2 at 2000 steps).  Gradients per parameter k,
max_j |g_jk - g^oracle_jk| / max_j |g^oracle_jk| <= 2e-4 over the stored
nodes (measured 0.85e-4, 0.90e-4 and 1.16e-4 for u*, phi and z0); probe
averages <= 5e-4 relative L2.  The two lambda layouts agree with each
other to 1e-9.  The 1e-4 gradient bar is held at 30 steps on this machine in
test_gpu_adjoint.py.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2508_18202_amd import inputs, sc
from paper_2508_18202_amd.adjoint import CheckpointedAdjoint

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_case_gradient.json")


@pytest.mark.parametrize("inplace", [False, True], ids=["two_buffers", "in_place"])
def test_adjoint_case_full_horizon(inplace):
    with open(GOLD) as fh:
        gold = json.load(fh)
    w = inputs.adjoint_case()
    solid = inputs.solid_mask(w)
    assert inputs.mask_hash(solid) == gold["mask_sha256"]
    assert (w.steps, w.avg_start, w.ckpt_every) == (gold["steps"], gold["avg_start"], gold["ckpt"])
    probes = inputs.probe_cells(w, solid)
    assert len(probes) == gold["probe_count"]
    x, a, th = sc.collocation(w)
    cg = sc.make_geometry(w, solid, probes)
    ens = sc.Ensemble([cg], [th], avg_begin=w.avg_start, avg_end=w.steps, fields=False, use_graph=True,
                      variant=(128, 1, 1, 1))
    try:
        run = CheckpointedAdjoint(ens, w.steps, w.ckpt_every, inplace=inplace)
        q = run.forward()
        pw = torch.full((len(probes),), 1.0 / len(probes), dtype=torch.float64, device="cuda")
        g = run.backward([pw] * len(ens)).cpu().numpy()
        run.close()
    finally:
        ens.close()
    idx = [nd["index"] for nd in gold["nodes"]]
    go = np.array([nd["grad"] for nd in gold["nodes"]])
    for nd in gold["nodes"]:
        j = nd["index"]
        # both sides ran the same (FP32-rounded) inflow parameters
        assert np.array_equal(np.asarray(th[j], np.float64), np.asarray(nd["theta"]))
        qa = q[j].cpu().numpy().astype(np.float64)
        qo = np.asarray(nd["probe_avg"])
        qerr = np.linalg.norm(qa - qo) / np.linalg.norm(qo)
        print(f"node {j}: probe averages rel L2 {qerr:.2e}", flush=True)
        assert qerr < 5e-4, (j, qerr)
    for k in range(3):
        err = np.abs(g[idx, k] - go[:, k]).max() / np.abs(go[:, k]).max()
        print(f"parameter {k}: gpu {g[idx, k]}, oracle {go[:, k]}, error {err:.2e}", flush=True)
        assert err < 2e-4, (k, err)
    _GRADS[inplace] = g


_GRADS = {}


def test_adjoint_case_layouts_agree():
    """Both lambda layouts of the full-horizon run give the same gradients
    (same forward state, the same transposed map stored two ways)."""
    if len(_GRADS) < 2:
        pytest.skip("needs both full-horizon runs")
    a, b = _GRADS[False], _GRADS[True]
    for k in range(3):
        assert np.abs(a[:, k] - b[:, k]).max() <= 1e-9 * np.abs(a[:, k]).max(), k
