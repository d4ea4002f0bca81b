"""Pins for the semi-nodal basis (Lemmas 2-4) in the oracle."""

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy.special import eval_jacobi

from oracle.basis import basis_ijk, eval_basis_abc, eval_basis_rst, n_basis
from oracle.rules import collapse, gauss_legendre, volume_rule


def test_np_counts():
    # Lemma 4 dimension count sum_k (k+1)^2 for N = 3..7
    assert [n_basis(N) for N in range(3, 8)] == [30, 55, 91, 140, 204]
    for N in range(0, 9):
        assert n_basis(N) == sum((k + 1) ** 2 for k in range(N + 1)) == len(basis_ijk(N))


def test_canonical_index_formula():
    for N in range(0, 7):
        for n, (i, j, k) in enumerate(basis_ijk(N)):
            assert n == k * (k + 1) * (2 * k + 1) // 6 + j * (k + 1) + i


@pytest.mark.parametrize("N", [1, 3, 5, 7])
def test_lemma2_c_orthogonality_and_constant(N):
    """int ((1-c)/2)^(2+k+k') P_{N-k}^{(2k+3,0)} P_{N-k'}^{(2k'+3,0)} dc = 2/(2k+3) delta.

    The printed constant of Lemma 2 does not match the standard Jacobi
    normalisation; 2/(2k+3) follows from the identity
    int (1-x)^(a-1) [P_n^{(a,0)}]^2 dx = 2^a / a.  Integrated here with a
    60-point Gauss-Legendre rule from numpy (exact for these degrees).
    """
    x, w = leggauss(60)
    h = (1 - x) / 2
    for k in range(N + 1):
        gk = h ** k * eval_jacobi(N - k, 2 * k + 3, 0, x)
        for k2 in range(N + 1):
            gk2 = h ** k2 * eval_jacobi(N - k2, 2 * k2 + 3, 0, x)
            val = np.sum(w * h ** 2 * gk * gk2)
            expect = 2.0 / (2 * k + 3) if k == k2 else 0.0
            assert abs(val - expect) < 1e-13


@pytest.mark.parametrize("N", [0, 1, 2, 4])
def test_reference_mass_diagonal(N):
    """Lemma 3 on the reference pyramid (J = 1): M = diag(w_i^k w_j^k 2/(2k+3))."""
    vr = volume_rule(N)
    V = eval_basis_rst(N, vr["r"], vr["s"], vr["t"])
    M = V.T @ (vr["w"][:, None] * V)
    expect = []
    for (i, j, k) in basis_ijk(N):
        _, wk = leggauss(k + 1)
        expect.append(wk[i] * wk[j] * 2.0 / (2 * k + 3))
    assert np.allclose(M, np.diag(expect), atol=1e-13, rtol=0)


def test_reference_mass_golden_N2():
    """Closed-form diagonal at N = 2 from tests/golden/reference_mass_N2.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "reference_mass_N2.txt")
    from fractions import Fraction
    vals = np.array([float(Fraction(line.split("#")[0].strip()))
                     for line in open(path) if line.split("#")[0].strip()])
    vr = volume_rule(2)
    V = eval_basis_rst(2, vr["r"], vr["s"], vr["t"])
    M = V.T @ (vr["w"][:, None] * V)
    assert vals.size == n_basis(2)
    assert np.allclose(np.diag(M), vals, atol=1e-14, rtol=0)


@pytest.mark.parametrize("N", [1, 2, 4])
def test_derivatives_match_finite_differences(N):
    rng = np.random.default_rng(5)
    a, b, c = rng.uniform(-0.9, 0.9, (3, 20))
    r, s, t = collapse(a, b, c)
    V, Vr, Vs, Vt = eval_basis_rst(N, r, s, t, deriv=True)
    eps = 1e-6
    for D, e in ((Vr, (1, 0, 0)), (Vs, (0, 1, 0)), (Vt, (0, 0, 1))):
        Vp = eval_basis_rst(N, r + eps * e[0], s + eps * e[1], t + eps * e[2])
        Vm = eval_basis_rst(N, r - eps * e[0], s - eps * e[1], t - eps * e[2])
        fd = (Vp - Vm) / (2 * eps)
        assert np.max(np.abs(fd - D)) < 1e-6 * max(1.0, np.abs(D).max())


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_lemma4_span_equals_collapsed_monomials(N):
    """span phi = span { a^m b^n ((1-c)/2)^k : max(m, n) <= k <= N } (Lemma 4)."""
    rng = np.random.default_rng(11)
    npts = 4 * n_basis(N)
    a, b, c = rng.uniform(-1, 1, (3, npts))
    V, _, _, _ = eval_basis_abc(N, a, b, c)
    cols = []
    for k in range(N + 1):
        for m in range(k + 1):
            for n in range(k + 1):
                cols.append(a ** m * b ** n * ((1 - c) / 2) ** k)
    T = np.stack(cols, axis=1)
    assert T.shape[1] == n_basis(N)
    assert np.linalg.matrix_rank(V, tol=1e-10) == n_basis(N)
    # V's columns are reproduced exactly by the monomial span, and vice versa
    coef, *_ = np.linalg.lstsq(T, V, rcond=None)
    assert np.max(np.abs(T @ coef - V)) < 1e-10
    coef2, *_ = np.linalg.lstsq(V, T, rcond=None)
    assert np.max(np.abs(V @ coef2 - T)) < 1e-10


def test_linear_functions_in_space():
    # r, s, t are (N >= 1) in the span: r = (1+a)(1-c)/2 - 1 etc.
    N = 1
    rng = np.random.default_rng(2)
    a, b, c = rng.uniform(-1, 1, (3, 40))
    r, s, t = collapse(a, b, c)
    V, _, _, _ = eval_basis_abc(N, a, b, c)
    for f in (r, s, t, np.ones_like(r)):
        coef, *_ = np.linalg.lstsq(V, f, rcond=None)
        assert np.max(np.abs(V @ coef - f)) < 1e-12


def test_lagrange_levels_use_k_plus_1_gauss_points():
    # phi_ijk restricted to c = -1 is l_i^k(a) l_j^k(b) P(-1): it vanishes at the
    # other (k+1)-point Gauss-Legendre nodes.
    N = 3
    for k in range(1, N + 1):
        xk, _ = gauss_legendre(k + 1)
        A, B = np.meshgrid(xk, xk, indexing="ij")
        V, _, _, _ = eval_basis_abc(N, A.ravel(), B.ravel(), -np.ones(A.size))
        for n, (i, j, kk) in enumerate(basis_ijk(N)):
            if kk != k:
                continue
            vals = V[:, n].reshape(k + 1, k + 1)
            mask = np.ones_like(vals, dtype=bool)
            mask[i, j] = False
            assert np.max(np.abs(vals[mask])) < 1e-12
            assert abs(vals[i, j]) > 1e-3
