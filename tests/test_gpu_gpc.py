"""GPU gPC expansion and the 121-node Gauss-Hermite ensemble against the oracle.

* lbm_gpc_coefficients on seeded inputs and on a polynomial QoI: coefficients,
  variance and 95 % band equal the oracle's projection of the same FP32
  values (FP64 sums in both; tolerance 1e-10 relative to the largest term);
* the paper's stochastic set-up (11 x 11 Gauss-Hermite nodes on
  zeta_1 ~ N(1, 0.1^2), zeta_2 ~ N(0, (6 deg)^2), hourly-series inflow) on a
  reduced urban box: the probe-line time averages of all 121 nodes against
  oracle runs (1e-5), and the order-5 gPC of the GPU probe
  averages against the oracle's expansion of the same values; the gPC mean
  equals the quadrature mean.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc
from paper_2508_18202_amd import inputs, sc
from gpu_util import oracle_case

pytestmark = pytest.mark.gpu
COEF_TOL = 1e-10


def _say(msg):
    print(msg, flush=True)


def _check(got, want):
    scale = max(1e-300, np.abs(want).max())
    assert np.abs(got - want).max() <= COEF_TOL * scale, (np.abs(got - want).max(), scale)


@pytest.mark.parametrize("order,n_elems", [(5, 10007), (3, 1), (7, 4096)])
def test_gpc_kernel_matches_oracle(order, n_elems):
    nodes, a = orc.tensor_gauss_hermite(11, 2)
    rng = np.random.default_rng(order)
    q = (0.02 + 0.01 * rng.standard_normal((121, n_elems))).astype(np.float32)
    z1, z2 = nodes[:, 0], nodes[:, 1]
    q[:, 0] = (3 + 2 * z1 - z2 + z1 ** 2 + z1 * z2 + z1 ** 3).astype(np.float32)   # a polynomial QoI
    r = sc.gpc(torch.from_numpy(q).cuda(), nodes, a, order)
    ro = orc.gpc(q.astype(np.float64), nodes, a, order)
    assert np.array_equal(r["alpha"], ro["alpha"])
    _check(r["coef"].cpu().numpy(), ro["coef"])
    _check(r["var"].cpu().numpy(), ro["var"])
    _check(r["band"].cpu().numpy(), ro["band"])


def test_gpc_empty_input():
    nodes, a = orc.tensor_gauss_hermite(3, 2)
    r = sc.gpc(torch.zeros(9, 0, device="cuda"), nodes, a, 2)
    assert r["coef"].shape == (6, 0)


def test_gauss_hermite_ensemble_probe_lines():
    w = inputs.scaled(inputs.urban_gpc(hours=4, hour_steps=30, blend_steps=10), 48, 24, 20, ramp=20,
                      steps=140, avg_start=100, ref_height=20.0)
    solid = inputs.solid_mask(w)
    probes = inputs.probe_cells(w, solid)
    assert len(probes) > 40
    _say("gauss-hermite ensemble: GPU (121 nodes)")
    r = sc.run_sc(w, solid, probes=probes)
    ens = r["ensemble"]
    try:
        pq = r["probe_q"].cpu().numpy()
        nodes, a = r["nodes"], r["weights"]
        xo, ao = orc.collocation(w)
        assert np.abs(nodes - xo).max() < 1e-12 and np.abs(a - ao).max() < 1e-14
        for j in range(len(nodes)):
            if j % 10 == 0:
                _say(f"gauss-hermite ensemble: oracle node {j}")
            th = orc.node_params(w, nodes[j])
            res = orc.run(oracle_case(w, solid, th), w.steps, avg_start=w.avg_start, probes=probes)
            err = np.abs(pq[j] - res["probe"]).max() / np.abs(res["probe"]).max()
            assert err < 1e-5, (j, err)
        g = sc.gpc(r["probe_q"], nodes, a, 5)
        go = orc.gpc(pq.astype(np.float64), nodes, a, 5)
        _check(g["coef"].cpu().numpy(), go["coef"])
        _check(g["band"].cpu().numpy(), go["band"])
        mean_q, _ = sc.moments(r["probe_q"], a)
        assert np.abs(g["mean"].cpu().numpy() - mean_q.cpu().numpy()).max() < 1e-12 * np.abs(go["mean"]).max()
    finally:
        ens.close()
