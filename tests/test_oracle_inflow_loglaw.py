"""Pins of the oracle's log-law inflow (the parametric wind profile of the
metric workloads) and of its start-up ramp.

Sec. 3 of arXiv 2508.18202 prescribes a logarithmic wind profile on the
inflow boundary; the parametric form used by the urban, adjoint and
assimilation workloads is u(z) = (u* / kappa) ln(z / z0) with kappa = 0.41,
the friction velocity u* and the roughness length z0, blowing in the
horizontal direction (cos phi, sin phi, 0).  Reading of the lattice: z is the
height of the cell centre above the half-way ground, z = k + 1/2 for layer k.
The start-up ramp multiplies u_in by r(n) = (1 - cos(pi n / T_r)) / 2 for
n < T_r.  Pins, each chosen so that a plausible slip fails it:

* layer 0 with z0 = 1/2 sits exactly at the roughness height: u = 0 exactly
  (fails for z = k instead of k + 1/2);
* with z0 = k + 1/2 the profile vanishes at layer k and only there, for
  several k (the same offset, at heights where ln is far from flat);
* lowering z0 by a factor e raises the speed at every height by exactly
  u* / kappa (pins kappa = 0.41 without evaluating a logarithm of the
  profile: ln(z / (z0/e)) = ln(z / z0) + 1);
* speeds are linear in u*, and at z0 = 1/2 layer k carries
  (u* / 0.41) ln(2k + 1);
* the velocity is horizontal with u_y / u_x = tan phi and |u| independent of
  phi (direction applied as a rotation, not a scaling);
* the ramp: r(0) = 0, r(T_r / 2) = 1/2, r(T_r / 4) = (1 - cos(pi/4)) / 2,
  r(n) = 1 from T_r on, and r increases monotonically in between.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc

KAPPA = 0.41
FACES = ("inlet", "outlet", "periodic", "periodic", "wall", "freeslip")


def _case(ustar, phi, z0, ramp=0, nz=12):
    solid = np.zeros((nz, 2, 4), np.uint8)
    return orc.Case(4, 2, nz, FACES, solid, model="bgk", tau0=0.6, inflow="loglaw",
                    theta=(ustar, phi, z0), ramp=ramp)


def _speed(u):
    return math.hypot(u[0], u[1])


def test_zero_at_the_roughness_height():
    c = _case(0.004, 0.0, 0.5)
    u = c.inflow_velocity(0, 5)
    assert u[0] == 0.0 and u[1] == 0.0 and u[2] == 0.0
    for k in (1, 3, 6):
        ck = _case(0.004, 0.0, k + 0.5)
        assert np.abs(ck.inflow_velocity(k, 5)).max() < 1e-19
        # below the roughness height the log law is negative, above positive
        assert ck.inflow_velocity(k - 1, 5)[0] < 0.0 < ck.inflow_velocity(k + 1, 5)[0]


def test_kappa_from_a_roughness_shift():
    ustar, z0 = 0.005, 0.8
    a = _case(ustar, 0.0, z0)
    b = _case(ustar, 0.0, z0 / math.e)
    for k in range(12):
        d = b.inflow_velocity(k, 3)[0] - a.inflow_velocity(k, 3)[0]
        assert abs(d - ustar / KAPPA) < 1e-15


def test_values_and_linearity_in_ustar():
    for ustar in (0.003, 0.004, 0.0046):
        c = _case(ustar, 0.0, 0.5)
        for k in range(12):
            u = c.inflow_velocity(k, 0)
            assert abs(u[0] - ustar / KAPPA * math.log(2 * k + 1)) < 1e-16
    c1, c2 = _case(0.002, 0.0, 0.5), _case(0.006, 0.0, 0.5)
    for k in range(12):
        assert abs(3.0 * c1.inflow_velocity(k, 0)[0] - c2.inflow_velocity(k, 0)[0]) < 1e-16


@pytest.mark.parametrize("phi", [0.0, 0.0872664626, -0.0872664626, 0.7, 2.5])
def test_direction_is_a_rotation(phi):
    base = _case(0.004, 0.0, 0.5)
    c = _case(0.004, phi, 0.5)
    for k in (1, 4, 9):
        u = c.inflow_velocity(k, 7)
        ref = base.inflow_velocity(k, 7)[0]
        assert u[2] == 0.0
        assert abs(_speed(u) - ref) < 1e-16
        assert abs(u[0] - ref * math.cos(phi)) < 1e-16 and abs(u[1] - ref * math.sin(phi)) < 1e-16


def test_ramp_factor():
    T = 200
    full = _case(0.004, 0.3, 0.5)
    c = _case(0.004, 0.3, 0.5, ramp=T)
    k = 5
    u_full = full.inflow_velocity(k, 0)
    assert np.abs(c.inflow_velocity(k, 0)).max() == 0.0
    assert np.allclose(c.inflow_velocity(k, T // 2), 0.5 * u_full, rtol=0, atol=1e-17)
    r4 = 0.5 * (1.0 - math.cos(math.pi / 4))
    assert np.allclose(c.inflow_velocity(k, T // 4), r4 * u_full, rtol=0, atol=1e-17)
    for n in (T, T + 1, 10 * T):
        assert np.array_equal(c.inflow_velocity(k, n), u_full)
    s = [c.inflow_velocity(k, n)[0] for n in range(T + 1)]
    assert all(b > a for a, b in zip(s, s[1:]))
