"""Pins of the oracle's lattice, equilibrium and collision against closed forms.

D3Q19 (Fig. 1 of arXiv 2508.18202, c_s^2 = 1/3): weight sums and isotropy are
exact rationals; the second-order equilibrium reproduces the moments
rho, rho u and rho (c_s^2 I + u u) exactly (Sec. 2.2, truncation of the
Hermite equilibrium at order two); the Smagorinsky relaxation time satisfies
Eq. (tauEff) with Eq. (turbVisc) when |S| is taken from the non-equilibrium
stress.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc


def test_velocity_set_is_d3q19():
    c, w, opp = orc.lattice()
    shells = sorted(int((ci ** 2).sum()) for ci in c)
    assert shells == [0] + [1] * 6 + [2] * 12
    assert len({tuple(ci) for ci in c}) == 19
    assert (np.abs(c) <= 1).all()
    for i in range(19):
        assert (c[opp[i]] == -c[i]).all()


def test_weights_and_isotropy_exact():
    from fractions import Fraction as Fr
    c, w, _ = orc.lattice()
    W = [Fr(x).limit_denominator(1000) for x in w]
    assert all(abs(float(Wi) - wi) < 1e-17 for Wi, wi in zip(W, w))
    assert sum(W) == 1
    d = lambda a, b: 1 if a == b else 0
    for a in range(3):
        assert sum(Wi * int(ci[a]) for Wi, ci in zip(W, c)) == 0
        for b in range(3):
            assert sum(Wi * int(ci[a] * ci[b]) for Wi, ci in zip(W, c)) == Fr(d(a, b), 3)
            for g in range(3):
                assert sum(Wi * int(ci[a] * ci[b] * ci[g]) for Wi, ci in zip(W, c)) == 0
                for e in range(3):
                    m4 = sum(Wi * int(ci[a] * ci[b] * ci[g] * ci[e]) for Wi, ci in zip(W, c))
                    iso = Fr(d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g), 9)
                    assert m4 == iso


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.1 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    c, _, _ = orc.lattice()
    feq = orc.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.abs(c.T @ feq - rho * u).max() < 1e-15
    m2 = np.einsum("i,ia,ib->ab", feq, c, c)
    assert np.abs(m2 - rho * (np.eye(3) / 3.0 + np.outer(u, u))).max() < 1e-15


def _one_cell(model, tau0=0.6, cs=0.0):
    return orc.Case(1, 1, 1, ["periodic"] * 6, np.zeros(1, np.uint8), model=model,
                    tau0=tau0, cs=cs)


@pytest.mark.parametrize("model,cs", [("bgk", 0.0), ("smagorinsky", 0.1), ("smagorinsky", 0.25)])
def test_collision_conserves_mass_momentum(model, cs):
    rng = np.random.default_rng(7)
    c, w, _ = orc.lattice()
    case = _one_cell(model, 0.52, cs)
    for _ in range(10):
        f = orc.equilibrium(1.0, 0.05 * rng.standard_normal(3)) + 1e-3 * w * rng.standard_normal(19)
        fs = case.collide_cell(f)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert np.abs(c.T @ fs - c.T @ f).max() < 1e-15


def test_rest_state_is_fixed_point():
    _, w, _ = orc.lattice()
    for model in ("bgk", "smagorinsky"):
        fs = _one_cell(model, 0.6, 0.1).collide_cell(w)
        assert np.abs(fs - w).max() < 1e-15


def test_smagorinsky_reduces_to_bgk_at_cs0():
    rng = np.random.default_rng(3)
    _, w, _ = orc.lattice()
    f = w * (1 + 0.01 * rng.standard_normal(19))
    a = _one_cell("bgk", 0.57).collide_cell(f)
    b = _one_cell("smagorinsky", 0.57, 0.0).collide_cell(f)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("cs", [0.1, 0.25])
def test_smagorinsky_viscosity_relation(cs):
    """nu_eff = nu_0 + Cs^2 |S| (Eqs. tauEff, turbVisc) with the strain rate
    recovered from the post-collision relaxation: the collision relaxes the
    non-equilibrium stress by (1 - 1/tau), so tau = 1 / (1 - Pi*_neq / Pi_neq)
    is measured from the oracle's output and S = -Pi_neq / (2 rho cs2 tau)."""
    rng = np.random.default_rng(11)
    c, w, _ = orc.lattice()
    tau0 = 0.5015
    case = _one_cell("smagorinsky", tau0, cs)
    for _ in range(5):
        u = 0.04 * rng.standard_normal(3)
        rho = 1.0 + 0.02 * rng.standard_normal()
        feq = orc.equilibrium(rho, u)
        # a non-equilibrium part carrying only a traceless shear stress
        A = 1e-3 * rng.standard_normal((3, 3))
        A = A + A.T
        A -= np.trace(A) / 3 * np.eye(3)
        H2 = np.einsum("ia,ib->iab", c, c) - np.eye(3)[None] / 3.0
        fneq = 4.5 * w * np.einsum("iab,ab->i", H2, A)
        f = feq + fneq
        fs = case.collide_cell(f)
        pi_in = np.einsum("i,ia,ib->ab", f - feq, c, c)
        pi_out = np.einsum("i,ia,ib->ab", fs - feq, c, c)
        ratio = pi_out[0, 1] / pi_in[0, 1]
        tau = 1.0 / (1.0 - ratio)
        S = -pi_in / (2 * rho * tau / 3.0)
        Smag = np.sqrt(2.0 * (S * S).sum())
        nu_eff = (tau - 0.5) / 3.0
        nu0 = (tau0 - 0.5) / 3.0
        assert abs(nu_eff - (nu0 + cs * cs * Smag)) < 1e-12 * max(1.0, nu_eff)


def test_tau_eff_positive_root():
    for q in (0.0, 1e-6, 1e-3, 0.1):
        t = orc.tau_eff(0.51, 0.1, 1.0, q)
        assert t >= 0.51
        assert abs(t * t - 0.51 * t - 9 * 0.01 * q / np.sqrt(2.0)) < 1e-15


@pytest.mark.parametrize("model,cs", [("bgk", 0.0), ("smagorinsky", 0.2), ("rr3", 0.0), ("rr3", 0.15)])
def test_collision_jacobian_matches_finite_differences(model, cs):
    rng = np.random.default_rng(5)
    _, w, _ = orc.lattice()
    case = _one_cell(model, 0.55, cs)
    f = orc.equilibrium(1.01, [0.03, -0.02, 0.01]) + 2e-3 * w * rng.standard_normal(19)
    if model == "rr3":
        # ghost components too: the regularisation must remove their response
        f = orc.equilibrium3(1.01, [0.05, -0.03, 0.02]) + 2e-3 * w * rng.standard_normal(19)
    J = case.collision_jacobian(f)
    h = 1e-6
    for k in range(19):
        e = np.zeros(19)
        e[k] = h
        col = (case.collide_cell(f + e) - case.collide_cell(f - e)) / (2 * h)
        assert np.abs(col - J[:, k]).max() < 1e-8
