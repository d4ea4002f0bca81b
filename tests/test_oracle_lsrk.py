"""Pins for the LSRK(5,4) stepper (Carpenter-Kennedy, cited in Section 4.1)."""

import math

import numpy as np

from oracle.lsrk import LSRK_A, LSRK_B, LSRK_C, lsrk_run


def _amplification(z):
    U, _ = lsrk_run(lambda U, t: z * U, np.array([1.0]), 1.0, 1)
    return U[0]


def test_stability_polynomial_matches_taylor_to_fourth_order():
    # R(z) is a degree-5 polynomial; recover it by interpolation at 6 points
    zs = np.array([-1.0, -0.5, -0.25, 0.25, 0.5, 1.0])
    R = np.array([_amplification(z) for z in zs])
    coef = np.polyfit(zs, R, 5)[::-1]
    for k in range(5):
        assert abs(coef[k] - 1.0 / math.factorial(k)) < 1e-12
    assert 0.0 < coef[5] < 1.0 / 120.0


def test_fourth_order_on_nonautonomous_ode():
    # y' = cos(t) y, y(0) = 1 -> y = exp(sin t); exercises the stage times c_s
    def run(n):
        U, _ = lsrk_run(lambda U, t: np.cos(t) * U, np.array([1.0]), 2.0 / n, n)
        return abs(U[0] - np.exp(np.sin(2.0)))

    e1, e2 = run(20), run(40)
    assert 3.8 < np.log2(e1 / e2) < 4.3


def test_stage_times_consistent():
    assert LSRK_C[0] == 0.0 and abs(LSRK_C[1] - LSRK_B[0]) < 1e-16
    assert np.all(np.diff(LSRK_C) > 0) and LSRK_C[-1] < 1.0
    assert LSRK_A[0] == 0.0
