"""Pins of the oracle's collocation rules and moment formula.

Sec. 2.3 of arXiv 2508.18202: statistics are quadrature sums over collocation
nodes Z^(j) with weights a_j (Eq. quad_moments).  The rules are pinned by
library routines and by exactness on polynomials against the closed-form
moments of xi ~ U(-1, 1): E[xi^k] = 1/(k+1) for even k, 0 for odd k.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as orc


def exact_moment(k):
    return 0.0 if k % 2 else 1.0 / (k + 1)


def test_gauss_legendre_matches_library():
    for n in (1, 2, 3, 5, 8, 11):
        x, a = orc.gauss_legendre(n)
        xl, wl = np.polynomial.legendre.leggauss(n)
        assert np.abs(x - xl).max() < 1e-14
        assert np.abs(a - wl / 2).max() < 1e-14


def test_gl5_closed_form():
    x, a = orc.gauss_legendre(5)
    r = math.sqrt(10.0 / 7.0)
    nodes = [-math.sqrt(5 + 2 * r) / 3, -math.sqrt(5 - 2 * r) / 3, 0.0,
             math.sqrt(5 - 2 * r) / 3, math.sqrt(5 + 2 * r) / 3]
    w70 = 13 * math.sqrt(70)
    weights = np.array([322 - w70, 322 + w70, 512, 322 + w70, 322 - w70]) / 900 / 2
    assert np.abs(x - nodes).max() < 1e-15
    assert np.abs(a - weights).max() < 1e-15


def test_gl5_exact_to_degree_9_only():
    x, a = orc.gauss_legendre(5)
    for k in range(10):
        assert abs((a * x ** k).sum() - exact_moment(k)) < 1e-15
    assert abs((a * x ** 10).sum() - exact_moment(10)) > 1e-4


def test_clenshaw_curtis_small_rules():
    x, a = orc.clenshaw_curtis(3)
    assert np.allclose(sorted(x), [-1, 0, 1]) and np.allclose(sorted(a), [1 / 6, 1 / 6, 2 / 3])
    x, a = orc.clenshaw_curtis(5)
    # CC with m nodes integrates degree m-1 (m odd: degree m) exactly
    for k in range(6):
        assert abs((a * x ** k).sum() - exact_moment(k)) < 1e-15
    assert abs((a * x ** 6).sum() - exact_moment(6)) > 1e-4


def test_smolyak_level2_structure():
    x, a = orc.smolyak_cc(2, 2)
    assert len(a) == 13
    assert abs(a.sum() - 1.0) < 1e-15
    lookup = {tuple(np.round(p, 12) + 0.0): wj for p, wj in zip(x, a)}
    s = 1 / math.sqrt(2)
    expect = {(0.0, 0.0): -4 / 45}
    for v in (1.0, -1.0):
        expect[(v, 0.0)] = expect[(0.0, v)] = -1 / 45
        for u in (1.0, -1.0):
            expect[(v, u)] = 1 / 36
    for v in (s, -s):
        expect[(round(v, 12), 0.0)] = expect[(0.0, round(v, 12))] = 4 / 15
    assert set(expect) == set(lookup)
    for k, v in expect.items():
        assert abs(lookup[k] - v) < 1e-15


def test_smolyak_exact_to_total_degree_5_only():
    x, a = orc.smolyak_cc(2, 2)
    for p, q in itertools.product(range(7), repeat=2):
        val = (a * x[:, 0] ** p * x[:, 1] ** q).sum()
        ex = exact_moment(p) * exact_moment(q)
        if p + q <= 5:
            assert abs(val - ex) < 1e-15, (p, q)
    # degree 6 is not integrated exactly
    assert abs((a * x[:, 0] ** 6).sum() - exact_moment(6)) > 1e-4


def test_moments_exact_for_polynomials():
    # E and Var of a polynomial QoI are exact when the rule integrates Q and Q^2.
    x, a = orc.gauss_legendre(5)
    q = 0.3 + 0.7 * x - 0.2 * x ** 2 + 0.1 * x ** 4        # deg 4: Q^2 has degree 8 <= 9
    e, v = orc.moments(q[:, None], a)
    from fractions import Fraction as Fr
    coef = [Fr(3, 10), Fr(7, 10), Fr(-2, 10), Fr(0), Fr(1, 10)]
    mom = lambda k: Fr(0) if k % 2 else Fr(1, k + 1)
    E = sum(c * mom(k) for k, c in enumerate(coef))
    EQ2 = sum(ci * cj * mom(i + j) for i, ci in enumerate(coef) for j, cj in enumerate(coef))
    V = EQ2 - E * E
    assert abs(e[0] - float(E)) < 1e-15 and abs(v[0] - float(V)) < 1e-15
    x2, a2 = orc.smolyak_cc(2, 2)
    q2 = 1.0 + 0.5 * x2[:, 0] - 0.25 * x2[:, 1] + 0.1 * x2[:, 0] * x2[:, 1]   # Q^2: total degree 4
    e2, v2 = orc.moments(q2[:, None], a2)
    E2 = 1.0
    V2 = 0.25 * (1 / 3) + 0.0625 * (1 / 3) + 0.01 * (1 / 9)
    assert abs(e2[0] - E2) < 1e-15 and abs(v2[0] - V2) < 1e-15


def test_small_block_inlet_speed_std():
    """Uniform inflow U = 0.05 (1 + 0.1 xi): E[U] = 0.05, Std[U] = 0.005 / sqrt(3)."""
    from paper_2508_18202_amd import inputs
    w = inputs.small_block()
    x, a = orc.collocation(w)
    U = np.array([orc.node_params(w, xi)[0] for xi in x])
    e, v = orc.moments(U[:, None], a)
    assert abs(e[0] - 0.05) < 1e-16
    assert abs(math.sqrt(v[0]) - 0.005 / math.sqrt(3)) < 1e-16


def test_negative_weight_variance_can_be_negative():
    """Smolyak weights are signed, so the quadrature variance is not a sum of
    non-negative terms; a QoI concentrated at the centre node shows it."""
    x, a = orc.smolyak_cc(2, 2)
    q = np.where(np.all(np.abs(x) < 1e-12, axis=1), 1.0, 0.0)
    _, v = orc.moments(q[:, None], a)
    assert v[0] < 0
