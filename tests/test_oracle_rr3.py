"""Pins of the oracle's regularised third-order collision (model "rr3").

Sec. 2.2 of arXiv 2508.18202 expands the equilibrium to third order in
Hermite polynomials that are orthogonal on D3Q19, and replaces the
non-equilibrium part f^(1) = f - f^eq by its expansion to third order with
the Hermite coefficients of Eq. (hermiteCoeff); Eq. (deterministicLBE) relaxes
it with 1 - 1/tau_eff.  The tests pin what the mathematics fixes:

* the basis: mutually orthogonal under sum_i w_i P(c_i) Q(c_i), rank 16 on the
  19 velocities (three ghost directions remain);
* the equilibrium: density, momentum and stress of the Maxwellian exactly,
  and the third-order moments that D3Q19 supports equal the Maxwellian's
  Q_abc = rho (u_a u_b u_c + cs2 (u_a d_bc + u_b d_ac + u_c d_ab));
* at u = 0 the equilibrium is w rho, and it differs from the second-order one
  only by terms cubic in u;
* the collision conserves mass and momentum, relaxes the non-equilibrium
  stress and the supported third-order moments by (1 - 1/tau_eff) (with the
  Smagorinsky tau_eff), leaves its output in the span of the basis, and
  removes a pure ghost perturbation completely;
* Taylor-Green decay gives the viscosity (tau - 1/2) / 3.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc

CS2 = 1.0 / 3.0
# third-order moment combinations D3Q19 supports: (a, a, b) +- (b, c, c)
COMBOS = [((0, 0, 1), (1, 2, 2)), ((0, 2, 2), (0, 1, 1)), ((1, 1, 2), (0, 0, 2))]


def _maxwell_q3(rho, u, a, b, c):
    d = np.eye(3)
    return rho * (u[a] * u[b] * u[c] + CS2 * (u[a] * d[b, c] + u[b] * d[a, c] + u[c] * d[a, b]))


def _q3(f, a, b, c):
    cv, _, _ = orc.lattice()
    return float((cv[:, a] * cv[:, b] * cv[:, c] * f).sum())


def _one_cell(model="rr3", tau0=0.6, cs=0.0):
    return orc.Case(1, 1, 1, ["periodic"] * 6, np.zeros(1, np.uint8), model=model, tau0=tau0, cs=cs)


def test_basis_orthogonal_on_d3q19():
    P, N = orc.rr3_basis()
    _, w, _ = orc.lattice()
    G = (P * w) @ P.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-15
    assert np.allclose(np.diag(G), N, rtol=0, atol=1e-15)
    assert np.linalg.matrix_rank(P) == 16
    # sums and differences of mixed third-order polynomials have the discrete
    # norms 2 cs^6 and 6 cs^6 (the continuous norm would be 4 cs^6 for both)
    assert np.allclose(N[10::2], 2 * CS2 ** 3, atol=1e-15)
    assert np.allclose(N[11::2], 6 * CS2 ** 3, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium3_moments_are_the_maxwellians(seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.2 * rng.standard_normal()
    u = 0.1 * rng.standard_normal(3)
    f = orc.equilibrium3(rho, u)
    cv, _, _ = orc.lattice()
    assert abs(f.sum() - rho) < 1e-14
    assert np.abs((cv * f[:, None]).sum(0) - rho * u).max() < 1e-14
    for a in range(3):
        for b in range(3):
            m2 = float((cv[:, a] * cv[:, b] * f).sum())
            assert abs(m2 - rho * (u[a] * u[b] + CS2 * (a == b))) < 1e-14
    for p, q in COMBOS:
        for sgn in (1.0, -1.0):
            got = _q3(f, *p) + sgn * _q3(f, *q)
            want = _maxwell_q3(rho, u, *p) + sgn * _maxwell_q3(rho, u, *q)
            assert abs(got - want) < 1e-14, (p, q, sgn)


def test_equilibrium3_reduces_to_second_order_up_to_cubic_terms():
    _, w, _ = orc.lattice()
    assert np.abs(orc.equilibrium3(1.3, [0.0, 0.0, 0.0]) - 1.3 * w).max() < 1e-15
    u = np.array([0.03, -0.02, 0.01])
    d = [(orc.equilibrium3(1.0, s * u) - orc.equilibrium(1.0, s * u)) / s ** 3 for s in (1.0, 0.5, 0.25)]
    assert np.abs(d[0]).max() > 1e-7          # the third-order terms are present
    assert np.abs(d[1] - d[0]).max() < 1e-12 and np.abs(d[2] - d[0]).max() < 1e-12


def _perturbed(seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.05 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    return orc.equilibrium3(rho, u) + amp * rng.standard_normal(19)


@pytest.mark.parametrize("cs", [0.0, 0.1])
@pytest.mark.parametrize("seed", range(3))
def test_collision_relaxes_supported_moments(seed, cs):
    case = _one_cell(tau0=0.6, cs=cs)
    f = _perturbed(seed)
    fs = case.collide_cell(f)
    cv, _, _ = orc.lattice()
    rho = f.sum()
    u = (cv * f[:, None]).sum(0) / rho
    assert abs(fs.sum() - rho) < 1e-14
    assert np.abs((cv * fs[:, None]).sum(0) - rho * u).max() < 1e-14
    feq = orc.equilibrium3(rho, u)
    pi = np.array([[(cv[:, a] * cv[:, b] * (f - feq)).sum() for b in range(3)] for a in range(3)])
    tau = orc.tau_eff(0.6, cs, rho, math.sqrt((pi * pi).sum()))
    keep = 1.0 - 1.0 / tau
    for a in range(3):
        for b in range(3):
            got = (cv[:, a] * cv[:, b] * (fs - feq)).sum()
            assert abs(got - keep * pi[a, b]) < 1e-14
    for p, q in COMBOS:
        for sgn in (1.0, -1.0):
            before = _q3(f - feq, *p) + sgn * _q3(f - feq, *q)
            after = _q3(fs - feq, *p) + sgn * _q3(fs - feq, *q)
            assert abs(after - keep * before) < 1e-14


def test_collision_output_lies_in_the_basis_and_ghosts_are_removed():
    case = _one_cell(tau0=0.7)
    P, _ = orc.rr3_basis()
    cv, w, _ = orc.lattice()
    f = _perturbed(7)
    fs = case.collide_cell(f)
    rho = f.sum()
    u = (cv * f[:, None]).sum(0) / rho
    v = (fs - orc.equilibrium3(rho, u)) / w
    x, *_ = np.linalg.lstsq(P.T, v, rcond=None)
    assert np.abs(P.T @ x - v).max() < 1e-14
    # ghost directions: w h with sum_i w_i h_i P_k(c_i) = 0 for every k
    _, sv, vt = np.linalg.svd(P * w)
    ghosts = vt[16:]
    assert ghosts.shape[0] == 3 and sv[-1] > 1e-3
    base = orc.equilibrium3(1.02, [0.03, 0.01, -0.02])
    for h in ghosts:
        g = base + 1e-3 * w * h
        assert abs(g.sum() - base.sum()) < 1e-15
        assert np.abs(case.collide_cell(g) - base).max() < 1e-15


def test_taylor_green_viscosity():
    N, u0, tau, t_end = 32, 0.02, 0.6, 400
    k = 2 * math.pi / N
    x, y = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    p = -0.25 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    rho = (1.0 + 3.0 * p).ravel()
    u = np.stack([ux.ravel(), uy.ravel(), 0 * ux.ravel()])
    case = orc.Case(N, N, 1, ["periodic"] * 6, np.zeros(N * N, np.uint8), model="rr3", tau0=tau)
    f = np.stack([orc.equilibrium3(rho[c], u[:, c]) for c in range(N * N)], axis=1).copy()
    mode = (-np.cos(k * x) * np.sin(k * y)).ravel()

    def amp(f):
        _, uu = case.macros(f)
        return (uu[0] * mode).sum() / (mode * mode).sum()

    for n in range(t_end // 4):
        f = case.step(n, f)
    a0 = amp(f)
    for n in range(t_end // 4, t_end):
        f = case.step(n, f)
    rate = -math.log(amp(f) / a0) / (t_end - t_end // 4)
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (2 * nu * k * k) - 1.0) < 0.01
