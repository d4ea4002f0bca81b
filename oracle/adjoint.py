"""Discrete adjoint of the LSRK(5,4) DG acoustics solver (TEST INFRASTRUCTURE).

Only tests, the smoke entry point and the benchmark's CPU-baseline leg may use
this module.  Plain and slow, for small meshes:

* the semi-discrete system of Section 4.3 is dU/dt = A U + b(t), linear in U;
  ``operator_matrix`` forms A densely, one column per unit vector, from
  ``AcousticDG.rhs`` without sources, so A^T is the plain matrix transpose;
* the receiver misfit J = dt/2 sum_{n=1..nsteps} sum_r (p(x_r, t_n) - d_{r,n})^2,
  p(x_r) = sum_i phi_i(xi_r) U_{p,i} of the element containing x_r;
* ``misfit_gradient`` differentiates J with respect to the per-element bulk
  modulus kappa = rho c^2 by reverse-mode through every LSRK stage
  (Algorithm 3): for the central flux (alpha = 0) the operator depends on
  kappa_K only through the factor kappa_K of element K's pressure rows, and
  so does the point-source term (dp/dt = -kappa M^-1 (vol + surf - b)), so
  d(A U + b)/d kappa_K = (A U + b)_{p,K} / kappa_K.

Pinned by central finite differences of ``misfit`` in ``tests/test_oracle_adjoint.py``.
"""

from __future__ import annotations

import numpy as np

from .basis import eval_basis_rst
from .dg import AcousticDG, locate_point
from .lsrk import LSRK_A, LSRK_B, LSRK_C


def operator_matrix(xyz, e2v, N, rho=None, kappa=None, bc="wall", alpha=0.0):
    """Dense A with dU/dt = A U (no sources), state flattened as (K, 4, Np)."""
    dg = AcousticDG(xyz, e2v, N, rho=rho, kappa=kappa, bc=bc, alpha=alpha)
    n = dg.K * 4 * dg.Np
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = dg.rhs(e.reshape(dg.K, 4, dg.Np)).ravel()
        e[j] = 0.0
    return A


def receiver_matrix(xyz, e2v, N, points):
    """Rows r: the pressure coefficients' weights phi_i(xi_r) in the element
    (lowest index) containing receiver point r."""
    xyz = np.asarray(xyz, dtype=np.float64)
    e2v = np.asarray(e2v, dtype=np.int64)
    K = e2v.shape[0]
    Np = (N + 1) * (N + 2) * (2 * N + 3) // 6
    Rm = np.zeros((len(points), K * 4 * Np))
    for r, x in enumerate(points):
        for e in range(K):
            rst, inside = locate_point(xyz[e2v[e]], np.asarray(x, dtype=np.float64))
            if inside:
                phi = eval_basis_rst(N, rst[:1], rst[1:2], rst[2:3])[0]
                Rm[r, e * 4 * Np: e * 4 * Np + Np] = phi
                break
        else:
            raise ValueError(f"receiver {r} lies in no element")
    return Rm


def _source_fn(xyz, e2v, N, rho, kappa, bc, sources):
    if not sources:
        return lambda t: 0.0
    dg = AcousticDG(xyz, e2v, N, rho=rho, kappa=kappa, bc=bc, alpha=0.0, sources=sources)
    zero = np.zeros((dg.K, 4, dg.Np))
    return lambda t: dg.rhs(zero, t).ravel()


def misfit(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, rho=None, bc="wall", sources=None):
    """J for the central-flux solver; data: (nsteps, nrec)."""
    A = operator_matrix(xyz, e2v, N, rho=rho, kappa=kappa, bc=bc, alpha=0.0)
    b = _source_fn(xyz, e2v, N, rho, kappa, bc, sources)
    U = np.asarray(U0, dtype=np.float64).ravel().copy()
    R = np.zeros_like(U)
    J = 0.0
    for n in range(nsteps):
        t = n * dt
        for s in range(5):
            R = LSRK_A[s] * R + dt * (A @ U + b(t + LSRK_C[s] * dt))
            U = U + LSRK_B[s] * R
        res = Rm @ U - data[n]
        J += 0.5 * dt * float(res @ res)
    return J


def misfit_gradient(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, rho=None, bc="wall",
                    sources=None):
    """(J, dJ/dkappa [K], dJ/dU0) by the discrete adjoint of every stage."""
    K = np.asarray(e2v).shape[0]
    Np = (N + 1) * (N + 2) * (2 * N + 3) // 6
    kappa = np.asarray(kappa, dtype=np.float64)
    A = operator_matrix(xyz, e2v, N, rho=rho, kappa=kappa, bc=bc, alpha=0.0)
    b = _source_fn(xyz, e2v, N, rho, kappa, bc, sources)
    U = np.asarray(U0, dtype=np.float64).ravel().copy()
    R = np.zeros_like(U)
    stages = []  # stage inputs U^(s) of every step
    res = []
    J = 0.0
    for n in range(nsteps):
        t = n * dt
        Ws = []
        for s in range(5):
            Ws.append(U.copy())
            R = LSRK_A[s] * R + dt * (A @ U + b(t + LSRK_C[s] * dt))
            U = U + LSRK_B[s] * R
        stages.append(Ws)
        r = Rm @ U - data[n]
        res.append(r)
        J += 0.5 * dt * float(r @ r)
    # reverse sweep
    Ub = np.zeros_like(U)
    grad = np.zeros(K)
    prow = np.zeros((K, 4, Np), dtype=bool)
    prow[:, 0, :] = True
    prow = prow.ravel()
    for n in range(nsteps - 1, -1, -1):
        Ub = Ub + dt * (Rm.T @ res[n])
        Rb = np.zeros_like(Ub)
        for s in range(4, -1, -1):
            Rb = Rb + LSRK_B[s] * Ub
            Ub = Ub + dt * (A.T @ Rb)
            ts = n * dt + LSRK_C[s] * dt
            AW = (A @ stages[n][s] + b(ts)) * prow
            grad += dt * (Rb * AW).reshape(K, 4 * Np).sum(axis=1) / kappa
            Rb = LSRK_A[s] * Rb
    return J, grad, Ub.reshape(K, 4, Np)
