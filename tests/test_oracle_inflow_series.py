"""Pins of the oracle's time-dependent inflow (measured hourly series, Sec. 3).

The paper perturbs the recorded hourly reference speed U_H(t) and direction
Theta(t) as U_H zeta_1 and Theta + zeta_2, prescribes the normalised log
profile U ln((h + z0)/z0) / ln((H + z0)/z0) (cos, sin, 0) on the horizontal
boundaries, ramps the first value in, and blends to each new hourly value
over an interpolation interval.  Pins:

* a constant series gives the closed-form profile at every step past the
  ramp, and the speed at the reference height (cell centre h = H) is exactly
  zeta_1 U_H;
* at the end of each blending interval the hourly value is reached exactly;
  half-way through, the speed is the mean of the two hours and the direction
  the midpoint of the shorter arc (also across +-pi); the change is smooth
  (monotone, slower at both ends than mid-way);
* during the ramp the hour-0 value is scaled by the ramp factor; past the
  last hour its value is held;
* the adjoint gradient w.r.t. (zeta_1, zeta_2, z0) matches central finite
  differences.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc

FACES = ("inlet", "outlet", "periodic", "periodic", "wall", "freeslip")


def _case(series, theta, ramp=0, hour_steps=10, blend=4, H=8.0, nz=8, **kw):
    solid = np.zeros((nz, 4, 6), np.uint8)
    return orc.Case(6, 4, nz, FACES, solid, inflow="series", theta=theta, ramp=ramp, series=series,
                    hour_steps=hour_steps, blend_steps=blend, ref_height=H, **kw)


def _speed_dir(u):
    return math.hypot(u[0], u[1]), math.atan2(u[1], u[0])


def test_constant_series_is_the_normalised_log_profile():
    U, th = 0.013, math.radians(25.0)
    z1, z2, z0, H = 1.07, math.radians(-4.0), 0.1, 7.5
    case = _case([(U, th)] * 3, (z1, z2, z0), H=H, blend=3)
    for n in (0, 4, 11, 23, 57):
        for z in range(8):
            h = z + 0.5
            prof = z1 * U * math.log((h + z0) / z0) / math.log((H + z0) / z0)
            want = prof * np.array([math.cos(th + z2), math.sin(th + z2), 0.0])
            assert np.abs(case.inflow_velocity(z, n) - want).max() < 1e-17
    # cell centre at the reference height: the perturbed reference speed itself
    case = _case([(U, th)], (z1, 0.0, z0), H=6.5)
    s, _ = _speed_dir(case.inflow_velocity(6, 100))
    assert abs(s - z1 * U) < 1e-17


def _ref(case, n, z=7):
    """Reference speed and direction recovered from the profile at height z."""
    c = case.c
    h = z + 0.5
    prof = math.log((h + c.theta[2]) / c.theta[2]) / math.log((c.ref_height + c.theta[2]) / c.theta[2])
    s, d = _speed_dir(case.inflow_velocity(z, n))
    return s / (c.theta[0] * prof), d - c.theta[1]


def test_blend_reaches_each_hour_and_takes_the_shorter_arc():
    series = [(0.010, math.radians(10.0)), (0.020, math.radians(50.0)),
              (0.016, math.radians(170.0)), (0.012, math.radians(-170.0))]
    T, B, R = 12, 6, 5
    case = _case(series, (1.0, 0.0, 0.1), ramp=R, hour_steps=T, blend=B)
    for h in range(1, 4):
        start = R + h * T
        # before the blend: previous hour; at its end: this hour exactly
        u0, d0 = _ref(case, start)
        assert abs(u0 - series[h - 1][0]) < 1e-15
        u1, d1 = _ref(case, start + B)
        assert abs(u1 - series[h][0]) < 1e-15
        assert abs(math.remainder(d1 - series[h][1], 2 * math.pi)) < 1e-14
        um, dm = _ref(case, start + B // 2)
        assert abs(um - 0.5 * (series[h - 1][0] + series[h][0])) < 1e-15
        arc = math.remainder(series[h][1] - series[h - 1][1], 2 * math.pi)
        assert abs(math.remainder(dm - (series[h - 1][1] + 0.5 * arc), 2 * math.pi)) < 1e-14
    # a smooth change: monotone, slower at both ends of the blend than mid-way
    start = R + T
    us = [_ref(case, start + t)[0] for t in range(B + 1)]
    inc = np.diff(us)
    assert np.all(inc > 0)
    assert inc[0] < inc[B // 2 - 1] and inc[-1] < inc[B // 2]
    # 170 deg -> -170 deg goes through 180 deg, not through 0
    _, dm = _ref(case, R + 3 * T + B // 2)
    assert abs(abs(dm) - math.pi) < 1e-14


def test_ramp_and_hold():
    series = [(0.012, 0.3), (0.018, -0.2)]
    R, T = 20, 7
    case = _case(series, (1.0, 0.0, 0.1), ramp=R, hour_steps=T, blend=2)
    for n in (1, 7, 13):
        r = 0.5 * (1.0 - math.cos(math.pi * n / R))
        u, d = _ref(case, n)
        assert abs(u - r * series[0][0]) < 1e-15 and abs(d - series[0][1]) < 1e-14
    for n in (R + 2 * T, R + 10 * T, R + 1000):
        u, d = _ref(case, n)
        assert abs(u - series[1][0]) < 1e-15 and abs(d - series[1][1]) < 1e-14


def test_invalid_series_parameters_are_rejected():
    good = dict(series=[(0.01, 0.0)], theta=(1.0, 0.0, 0.1))
    for bad in (dict(series=[]), dict(hour_steps=0), dict(blend=11), dict(H=0.0), dict(theta=(1.0, 0.0, 0.0))):
        kw = {**good, **bad}
        with pytest.raises(ValueError):
            _case(kw.pop("series"), kw.pop("theta"), **kw)


def test_series_adjoint_matches_central_differences():
    nx, ny, nz = 20, 10, 9
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[0:4, 3:6, 8:11] = 1
    series = [(0.012, 0.05), (0.016, -0.15), (0.010, 0.2), (0.014, 0.0)]
    theta = (1.05, 0.03, 0.1)
    case = orc.Case(nx, ny, nz, FACES, solid, model="smagorinsky", tau0=0.56, cs=0.1, inflow="series",
                    theta=theta, ramp=10, series=series, hour_steps=20, blend_steps=8, ref_height=float(nz))
    steps, avg_start = 90, 60
    xp = (3 * nx) // 4
    probes = np.asarray([(z * ny + y) * nx + xp for z in range(nz // 2) for y in range(ny)
                         if not solid[z, y, xp]], dtype=np.int64)
    pw = np.full(len(probes), 1.0 / len(probes))
    grad, _ = orc.adjoint(case, steps, avg_start, probes, pw, ckpt=25)
    fd = np.zeros(3)
    for k in range(3):
        h = 1e-4 * abs(theta[k]) if k != 1 else 1e-4
        tp, tm = list(theta), list(theta)
        tp[k] += h
        tm[k] -= h
        jp = orc.probe_objective(case.with_theta(tp), steps, avg_start, probes, pw)
        jm = orc.probe_objective(case.with_theta(tm), steps, avg_start, probes, pw)
        fd[k] = (jp - jm) / (2 * h)
    assert np.abs(fd).min() > 0
    assert np.abs(grad - fd).max() < 1e-6 * np.abs(fd).max(), (grad, fd)
