"""The semi-nodal orthogonal basis of Lemma 3 (oracle).

phi_ijk(a, b, c) = l^k_i(a) l^k_j(b) ((1-c)/2)^k P^{(2k+3,0)}_{N-k}(c),
0 <= i, j <= k <= N, where l^k_i is the Lagrange polynomial on the (k+1)
Gauss-Legendre nodes and P^{(alpha,0)}_n is the Jacobi polynomial in its
standard normalisation P_n(1) = binom(n + alpha, n).

Readings of the printed text (Lemma 3 and Lemma 4): the Jacobi factor has
degree N-k (not k), and i, j range over 0..k (the Lagrange factor of level k
has k+1 nodes), giving Np = sum_k (k+1)^2 = (N+1)(N+2)(2N+3)/6.

Canonical ordering (k slowest, then j, then i):
n(i, j, k) = k(k+1)(2k+1)/6 + j(k+1) + i.
"""

from __future__ import annotations

import numpy as np
from scipy.special import eval_jacobi

from .rules import gauss_legendre


def n_basis(N: int) -> int:
    return (N + 1) * (N + 2) * (2 * N + 3) // 6


def basis_ijk(N: int):
    """List of (i, j, k) in canonical order."""
    out = []
    for k in range(N + 1):
        for j in range(k + 1):
            for i in range(k + 1):
                out.append((i, j, k))
    return out


def lagrange(nodes, x):
    """Values and derivatives of all Lagrange polynomials on ``nodes`` at x.

    Returns (L, dL), each of shape (len(nodes), len(x)).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    m = len(nodes)
    L = np.ones((m, x.size))
    dL = np.zeros((m, x.size))
    for i in range(m):
        for q in range(m):
            if q == i:
                continue
            L[i] *= (x - nodes[q]) / (nodes[i] - nodes[q])
        # derivative of a product: sum over the dropped factor
        for q in range(m):
            if q == i:
                continue
            term = np.full(x.size, 1.0 / (nodes[i] - nodes[q]))
            for l in range(m):
                if l == i or l == q:
                    continue
                term = term * (x - nodes[l]) / (nodes[i] - nodes[l])
            dL[i] += term
    return L, dL


def jacobi(n: int, alpha: float, x):
    return eval_jacobi(n, alpha, 0.0, x)


def jacobi_deriv(n: int, alpha: float, x):
    """d/dx P_n^{(alpha,0)} = (n + alpha + 1)/2 P_{n-1}^{(alpha+1,1)}."""
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return 0.5 * (n + alpha + 1.0) * eval_jacobi(n - 1, alpha + 1.0, 1.0, x)


def eval_basis_abc(N: int, a, b, c):
    """phi_ijk and its a, b, c partial derivatives at collapsed points.

    Returns V, Va, Vb, Vc of shape (npts, Np).
    """
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    c = np.asarray(c, dtype=np.float64).ravel()
    npts = a.size
    Np = n_basis(N)
    V = np.zeros((npts, Np))
    Va = np.zeros((npts, Np))
    Vb = np.zeros((npts, Np))
    Vc = np.zeros((npts, Np))
    n = 0
    h = (1.0 - c) / 2.0
    for k in range(N + 1):
        nodes, _ = gauss_legendre(k + 1)
        La, dLa = lagrange(nodes, a)
        Lb, dLb = lagrange(nodes, b)
        alpha = 2.0 * k + 3.0
        g = h ** k * jacobi(N - k, alpha, c)
        # d/dc [ ((1-c)/2)^k P(c) ] = -k/2 ((1-c)/2)^(k-1) P + ((1-c)/2)^k P'
        dg = h ** k * jacobi_deriv(N - k, alpha, c)
        if k > 0:
            dg = dg - 0.5 * k * h ** (k - 1) * jacobi(N - k, alpha, c)
        for j in range(k + 1):
            for i in range(k + 1):
                V[:, n] = La[i] * Lb[j] * g
                Va[:, n] = dLa[i] * Lb[j] * g
                Vb[:, n] = La[i] * dLb[j] * g
                Vc[:, n] = La[i] * Lb[j] * dg
                n += 1
    return V, Va, Vb, Vc


def rst_to_abc(r, s, t):
    """Inverse of the Duffy-type map (valid for t < 1)."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    a = 2.0 * (1.0 + r) / (1.0 - t) - 1.0
    b = 2.0 * (1.0 + s) / (1.0 - t) - 1.0
    return a, b, t.copy()


def eval_basis_rst(N: int, r, s, t, deriv: bool = False):
    """phi at reference points; with ``deriv`` also d/dr, d/ds, d/dt.

    Chain rule of the collapse: d/dr = 2/(1-c) d/da, d/ds = 2/(1-c) d/db,
    d/dt = d/dc + (1+a)/(1-c) d/da + (1+b)/(1-c) d/db.
    """
    a, b, c = rst_to_abc(r, s, t)
    V, Va, Vb, Vc = eval_basis_abc(N, a, b, c)
    if not deriv:
        return V
    a = a.ravel()[:, None]
    b = b.ravel()[:, None]
    c = c.ravel()[:, None]
    Vr = 2.0 / (1.0 - c) * Va
    Vs = 2.0 / (1.0 - c) * Vb
    Vt = Vc + (1.0 + a) / (1.0 - c) * Va + (1.0 + b) / (1.0 - c) * Vb
    return V, Vr, Vs, Vt
