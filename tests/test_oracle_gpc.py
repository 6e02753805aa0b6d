"""Pins of the oracle's Gaussian collocation and gPC expansion (Sec. 2.3, Sec. 3).

The paper draws zeta_1 ~ N(1, 0.1^2) and zeta_2 ~ N(0, 6^2) (degrees), uses a
dense tensor-product Gauss-Hermite rule with 11 points per dimension (121
nodes) and expands QoIs in Hermite polynomials up to order 5 with
coefficients by projection.  Pins:

* the n-point rule integrates E[z^k] = (k-1)!! exactly up to degree 2n-1
  and not at 2n; the 3-point rule is {0, +-sqrt(3)} with weights 2/3, 1/6;
* the orthonormal chaos (He_a / sqrt(a!)) is orthonormal on the 11x11 rule,
  with C(order + d, d) = 21 terms graded by degree;
* a polynomial QoI gets its exact Hermite coefficients, worked by hand from
  z^2 = He_2 + 1, z^3 = He_3 + 3 He_1: for
  Q = 3 + 2 z1 - z2 + z1^2 + z1 z2 + z1^3, c_0 = 4, c_(1,0) = 5,
  c_(0,1) = -1, c_(2,0) = sqrt 2, c_(1,1) = 1, c_(3,0) = sqrt 6, others 0;
  mean 4, variance 35;
* the input model: over the rule, zeta_1 = 1 + 0.1 z1 has mean 1 and standard
  deviation 0.1, zeta_2 = 6 deg z2 has standard deviation 6 deg.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2508_18202_amd import inputs


def _double_factorial(k):
    return 1 if k <= 0 else k * _double_factorial(k - 2)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 11])
def test_gauss_hermite_gaussian_moments(n):
    x, w = orc.gauss_hermite(n)
    assert abs(w.sum() - 1.0) < 1e-15
    for k in range(2 * n):
        exact = 0.0 if k % 2 else float(_double_factorial(k - 1))
        scale = (w * np.abs(x) ** k).sum()          # size of the terms that cancel
        assert abs((w * x ** k).sum() - exact) <= 1e-13 * scale, (n, k)
    k = 2 * n
    assert abs((w * x ** k).sum() - _double_factorial(k - 1)) > 1e-3


def test_three_point_rule_closed_form():
    x, w = orc.gauss_hermite(3)
    assert np.allclose(x, [-math.sqrt(3), 0.0, math.sqrt(3)], atol=1e-15)
    assert np.allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)


def test_chaos_orthonormal_on_the_tensor_rule():
    nodes, w = orc.tensor_gauss_hermite(11, 2)
    assert nodes.shape == (121, 2) and abs(w.sum() - 1.0) < 1e-14
    phi, alpha = orc.gpc_basis(nodes, 5)
    assert alpha.shape == (21, 2)
    assert alpha[:6].tolist() == [[0, 0], [1, 0], [0, 1], [2, 0], [1, 1], [0, 2]]
    G = (phi * w[:, None]).T @ phi
    assert np.abs(G - np.eye(21)).max() < 1e-12


def test_polynomial_qoi_exact_coefficients():
    nodes, w = orc.tensor_gauss_hermite(11, 2)
    z1, z2 = nodes[:, 0], nodes[:, 1]
    q = (3 + 2 * z1 - z2 + z1 ** 2 + z1 * z2 + z1 ** 3)[:, None]
    r = orc.gpc(q, nodes, w, 5)
    want = {(0, 0): 4.0, (1, 0): 5.0, (0, 1): -1.0, (2, 0): math.sqrt(2), (1, 1): 1.0, (3, 0): math.sqrt(6)}
    for p, a in enumerate(r["alpha"]):
        assert abs(r["coef"][p, 0] - want.get(tuple(int(v) for v in a), 0.0)) < 1e-12, a
    assert abs(r["mean"][0] - 4.0) < 1e-12 and abs(r["var"][0] - 35.0) < 1e-10
    sd = math.sqrt(35.0)
    assert np.allclose(r["band"][:, 0], [4.0 - 1.96 * sd, 4.0 + 1.96 * sd], atol=1e-10)
    # agrees with the quadrature moments for a polynomial inside the span
    e, v = orc.moments(q, w)
    assert abs(e[0] - 4.0) < 1e-12 and abs(v[0] - 35.0) < 1e-10


def test_paper_input_model_on_the_rule():
    w = inputs.urban_gpc()
    nodes, a = orc.collocation(w)
    th = np.stack([orc.node_params(w, xi) for xi in nodes])
    m1 = (a * th[:, 0]).sum()
    s1 = math.sqrt((a * (th[:, 0] - m1) ** 2).sum())
    s2 = math.sqrt((a * th[:, 1] ** 2).sum())
    assert len(a) == 121
    assert abs(m1 - 1.0) < 1e-14 and abs(s1 - 0.1) < 1e-14
    assert abs(s2 - math.radians(6.0)) < 1e-14
