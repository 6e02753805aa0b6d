"""Pins of the oracle's discrete adjoint.

The gradient of a probe QoI with respect to the inflow parameters is not in
arXiv 2508.18202; it differentiates the paper's deterministic solver
(Sec. 2.2) with respect to the uncertain boundary data of Sec. 3.  The oracle
adjoint is pinned by
* a dot-product test of one step: <dS v, w> (central differences of the
  oracle's own forward step) equals <v, dS^T w> (its adjoint step);
* central finite differences of the whole forward run in float64
  (relative step 1e-4 for u* and z0, absolute 1e-4 rad for the direction).
"""
import numpy as np
import pytest

from oracle import oracle as orc

FACES = ["inlet", "outlet", "periodic", "periodic", "wall", "freeslip"]


def _small_solid(nx=20, ny=10, nz=9):
    s = np.zeros((nz, ny, nx), np.uint8)
    s[0:5, 3:7, 6:10] = 1
    return s


def _state(case, steps=40):
    f = case.init()
    for n in range(steps):
        f = case.step(n, f)
    return f


@pytest.mark.parametrize("model,cs", [("bgk", 0.0), ("smagorinsky", 0.2), ("rr3", 0.15)])
def test_adjoint_step_dot_product(model, cs):
    nx, ny, nz = 20, 10, 9
    case = orc.Case(nx, ny, nz, FACES, _small_solid(nx, ny, nz), model=model, tau0=0.56, cs=cs,
                    inflow="loglaw", theta=(0.01, 0.1, 0.5), ramp=0)
    f = _state(case)
    rng = np.random.default_rng(2)
    fluid = case.solid.reshape(-1) == 0
    v = rng.standard_normal(f.shape) * fluid
    w = rng.standard_normal(f.shape) * fluid
    eps = 1e-6 if model == "bgk" else 1e-8   # truncation vs round-off optimum
    jv = (case.step(40, f + eps * v) - case.step(40, f - eps * v)) / (2 * eps)
    lam, _ = case.adjoint_step(40, f, w)
    lhs = (jv * w).sum()
    rhs = (v * lam).sum()
    assert abs(lhs - rhs) < 1e-9 * abs(lhs)


def _probe_plane(nx, ny, nz, solid):
    xp = (3 * nx) // 4
    cells = [(z * ny + y) * nx + xp for z in range(nz // 2) for y in range(ny)
             if not solid[z, y, xp]]
    return np.asarray(cells, dtype=np.int64)


@pytest.mark.parametrize("model,cs,inflow,theta,ramp", [
    ("bgk", 0.0, "uniform", (0.05, 0.0, 0.0), 0),
    ("bgk", 0.0, "loglaw", (0.012, 0.05, 0.5), 0),
    ("smagorinsky", 0.1, "loglaw", (0.012, -0.07, 0.5), 30),
    ("rr3", 0.1, "loglaw", (0.012, 0.04, 0.5), 30),
    ("rr3", 0.0, "uniform", (0.05, -0.03, 0.0), 0),
])
def test_adjoint_gradient_matches_central_differences(model, cs, inflow, theta, ramp):
    nx, ny, nz = 20, 10, 9
    solid = _small_solid(nx, ny, nz)
    steps, avg_start = 90, 60
    case = orc.Case(nx, ny, nz, FACES, solid, model=model, tau0=0.56, cs=cs,
                    inflow=inflow, theta=theta, ramp=ramp)
    probes = _probe_plane(nx, ny, nz, solid)
    pw = np.full(len(probes), 1.0 / len(probes))
    grad, _ = orc.adjoint(case, steps, avg_start, probes, pw, ckpt=25)
    fd = np.zeros(3)
    for k in range(3):
        if inflow == "uniform" and k == 2:
            continue
        h = 1e-4 * abs(theta[k]) if k != 1 else 1e-4
        tp, tm = list(theta), list(theta)
        tp[k] += h
        tm[k] -= h
        jp = orc.probe_objective(case.with_theta(tp), steps, avg_start, probes, pw)
        jm = orc.probe_objective(case.with_theta(tm), steps, avg_start, probes, pw)
        fd[k] = (jp - jm) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 0
    assert np.abs(grad - fd).max() < 1e-6 * scale, (grad, fd)
    if inflow == "uniform":
        assert grad[2] == 0.0
