"""Pins for the oracle's quadrature rules (Section 2 collapse, Section 4.1 rule).

Every expected value here comes from exact polynomial integration with
numpy.polynomial (antiderivatives), not from the rules under test.
"""

import numpy as np
import pytest
from numpy.polynomial import Polynomial as P
from numpy.polynomial.legendre import leggauss

from oracle.rules import face_rules, gauss_jacobi, gauss_legendre, volume_rule


def _int_poly(p, lo=-1.0, hi=1.0):
    q = p.integ()
    return q(hi) - q(lo)


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_gauss_legendre_matches_numpy(n):
    x, w = gauss_legendre(n)
    x2, w2 = leggauss(n)
    assert np.allclose(x, x2, atol=1e-15, rtol=0)
    assert np.allclose(w, w2, atol=1e-15, rtol=0)
    assert np.all(np.diff(x) > 0)


@pytest.mark.parametrize("alpha", [0, 1, 2, 5])
@pytest.mark.parametrize("n", [1, 3, 6])
def test_gauss_jacobi_exact_to_degree_2n_minus_1(n, alpha):
    x, w = gauss_jacobi(n, alpha)
    weight = P([1.0, -1.0]) ** alpha
    for m in range(2 * n):
        exact = _int_poly(weight * P([0.0] * m + [1.0]))
        assert abs(np.dot(w, x ** m) - exact) <= 1e-14 * max(1.0, abs(exact)) * 10
    # weights sum to 2^(alpha+1)/(alpha+1)
    assert abs(w.sum() - 2.0 ** (alpha + 1) / (alpha + 1)) < 1e-13


def _pyramid_monomial(i, j, k):
    """Exact integral of r^i s^j t^k over r, s in [-1, -t], t in [-1, 1]."""
    t = P([0.0, 1.0])
    # int_{-1}^{-t} r^i dr = ((-t)^(i+1) - (-1)^(i+1)) / (i+1), a polynomial in t
    Ir = ((-t) ** (i + 1) - (-1.0) ** (i + 1)) / (i + 1)
    Is = ((-t) ** (j + 1) - (-1.0) ** (j + 1)) / (j + 1)
    return _int_poly(Ir * Is * t ** k)


def test_volume_rule_total_is_pyramid_volume():
    for N in range(0, 8):
        assert abs(volume_rule(N)["w"].sum() - 8.0 / 3.0) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 4])
def test_volume_rule_integrates_polynomials_exactly(N):
    vr = volume_rule(N)
    # the collapsed rule with N+1 points is exact for total degree <= 2N-1
    for i in range(0, 2 * N):
        for j in range(0, 2 * N - i):
            for k in range(0, 2 * N - i - j):
                num = np.sum(vr["w"] * vr["r"] ** i * vr["s"] ** j * vr["t"] ** k)
                assert abs(num - _pyramid_monomial(i, j, k)) < 1e-12


def test_volume_rule_points_inside_pyramid():
    vr = volume_rule(5)
    assert np.all(vr["t"] > -1) and np.all(vr["t"] < 1)
    assert np.all(vr["r"] >= -1) and np.all(vr["r"] <= -vr["t"])
    assert np.all(vr["s"] >= -1) and np.all(vr["s"] <= -vr["t"])


def test_face_rule_reference_areas():
    # reference faces: base 4, r=-1 and s=-1 area 2, slanted faces 2*sqrt(2)
    # (slanted area = parameter area 2 times |(0,1,0) x (-1,0,1)| = sqrt 2)
    for N in range(0, 6):
        fr = face_rules(N)
        assert abs(fr[0]["w"].sum() - 4.0) < 1e-13
        for f in (1, 2, 3, 4):
            assert abs(fr[f]["w"].sum() - 2.0) < 1e-13
        slant = np.linalg.norm(np.cross(fr[2]["tang"][0], fr[2]["tang"][1]))
        assert abs(slant - np.sqrt(2.0)) < 1e-15


@pytest.mark.parametrize("N", [1, 3])
def test_triangle_rule_integrates_face_polynomials(N):
    # face r = -1, parameters (s, t): s in [-1, -t], t in [-1, 1]
    fr = face_rules(N)[1]
    t = P([0.0, 1.0])
    for i in range(0, 2 * N):
        for k in range(0, 2 * N - i):
            Is = ((-t) ** (i + 1) - (-1.0) ** (i + 1)) / (i + 1)
            exact = _int_poly(Is * t ** k)
            num = np.sum(fr["w"] * fr["s"] ** i * fr["t"] ** k)
            assert abs(num - exact) < 1e-12
