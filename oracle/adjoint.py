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
  (Algorithm 3).  The operator depends on kappa_K through the factor kappa_K
  of element K's pressure rows, which the point-source term shares
  (dp/dt = -kappa M^-1 (vol + surf - b)), giving (A U + b)_{p,K} / kappa_K,
  and, for alpha > 0, through the penalty coefficients tau_p = alpha/{rho c},
  tau_u = alpha {rho c} of every face of K, {rho c} = (z- + z+)/2 with
  z = sqrt(kappa rho): ``penalty_kappa_terms`` adds those.

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


def penalty_kappa_terms(dg, W, Rb):
    """sum over faces of <Rb, d(A W)/d kappa_K> through tau (alpha > 0), for
    every element K of ``dg`` (an AcousticDG on the whole mesh).

    With P_p = (n.[[u]] - tau_p [[p]])/2 and P_u = n ([[p]] - tau_u n.[[u]])/2
    lifted into element e's rows of A W = -Kmat M^-1 (vol + surf),
    d/d{rho c} <Rb_e, (A W)_e> = sum_q s_e(q) with
    s_e = -w sJ alpha/2 (mu_p [[p]] / {rho c}^2 - (n.mu_u) (n.[[u]])),
    mu = traces of M^-1 Kmat Rb.  d{rho c}/d kappa_x = z_x / (4 kappa_x) for
    x either side of an interior face, z_e / (2 kappa_e) on a boundary face
    (the ghost has the element's own material)."""
    K, Np = dg.K, dg.Np
    W = np.asarray(W, dtype=np.float64).reshape(K, 4, Np)
    Rb = np.asarray(Rb, dtype=np.float64).reshape(K, 4, Np)
    rho, kap, z = dg._material(np.arange(K))
    kfac = np.concatenate([kap[:, None], np.repeat((1.0 / rho)[:, None], 3, axis=1)], axis=1)
    mu = np.einsum("eij,efj->efi", dg.Minv, kfac[:, :, None] * Rb)
    TW = dg.traces(W)
    TM = dg.traces(mu)
    g = np.zeros(K)
    for f in range(5):
        Tm = TW[f]
        n = dg.fn[f]
        Tp = np.empty_like(Tm)
        zP = z.copy()
        inner = dg.nb_row[f] >= 0
        rows = np.where(inner)[0]
        for f2 in range(5):
            sel = rows[dg.nb_f[f][rows] == f2]
            if sel.size:
                src = TW[f2][dg.nb_row[f][sel]]
                Tp[sel] = np.take_along_axis(src, dg.nb_perm[f][sel][:, None, :], axis=2)
        zP[rows] = z[dg.nb_row[f][rows]]
        bnd = ~inner
        if np.any(bnd):
            pm, um, nb = Tm[bnd, 0], Tm[bnd, 1:4], n[bnd]
            un = np.einsum("mdq,mqd->mq", um, nb)
            if dg.bc == "wall":
                Tp[bnd, 0] = pm
                Tp[bnd, 1:4] = um - 2.0 * un[:, None, :] * np.transpose(nb, (0, 2, 1))
            else:
                Tp[bnd, 0] = -pm
                Tp[bnd, 1:4] = um
        zavg = 0.5 * (z + zP)
        jp = Tp[:, 0] - Tm[:, 0]
        jun = np.einsum("edq,eqd->eq", Tp[:, 1:4] - Tm[:, 1:4], n)
        mun = np.einsum("edq,eqd->eq", TM[f][:, 1:4], n)
        s_e = -dg.fw[f] * 0.5 * dg.alpha * (TM[f][:, 0] * jp / zavg[:, None] ** 2 - mun * jun)
        tot = s_e.sum(axis=1)
        # own side
        g += np.where(inner, z / (4.0 * kap), z / (2.0 * kap)) * tot
        # the neighbour's {rho c} on this face
        nbr = dg.nb_row[f][rows]
        np.add.at(g, nbr, z[nbr] / (4.0 * kap[nbr]) * tot[rows])
    return g


def misfit(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, rho=None, bc="wall", sources=None,
           alpha=0.0):
    """J; data: (nsteps, nrec)."""
    A = operator_matrix(xyz, e2v, N, rho=rho, kappa=kappa, bc=bc, alpha=alpha)
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
                    sources=None, alpha=0.0):
    """(J, dJ/dkappa [K], dJ/dU0) by the discrete adjoint of every stage."""
    K = np.asarray(e2v).shape[0]
    Np = (N + 1) * (N + 2) * (2 * N + 3) // 6
    kappa = np.asarray(kappa, dtype=np.float64)
    A = operator_matrix(xyz, e2v, N, rho=rho, kappa=kappa, bc=bc, alpha=alpha)
    dgp = AcousticDG(xyz, e2v, N, rho=rho, kappa=kappa, bc=bc, alpha=alpha) if alpha else None
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
            if dgp is not None:
                grad += dt * penalty_kappa_terms(dgp, stages[n][s], Rb)
            Rb = LSRK_A[s] * Rb
    return J, grad, Ub.reshape(K, 4, Np)
