"""Pins of the oracle's discrete adjoint: its gradient of the receiver misfit
with respect to per-element kappa (and to the initial state) against central
finite differences of the misfit itself, and the transpose of the assembled
operator against the energy identity."""

import numpy as np

from oracle import AcousticDG
from oracle.adjoint import misfit, misfit_gradient, operator_matrix, receiver_matrix
from oracle.dg import wall_mode
from synth import hex_pyramid_mesh, random_state


def _setup(N=2, k1d=1, nsteps=6, seed=0):
    xyz, e2v = hex_pyramid_mesh(k1d, seed=seed)
    K = e2v.shape[0]
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(0.5, 2.0, K)
    U0 = AcousticDG(xyz, e2v, N).project(wall_mode(1), xyz, e2v)
    pts = rng.uniform(0.15, 0.85, (3, 3))
    Rm = receiver_matrix(xyz, e2v, N, pts)
    data = rng.normal(0.0, 0.1, (nsteps, 3))
    dt = 0.02
    src = [dict(x=[0.4, 0.55, 0.45], f0=10.0)]
    return xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, src


def test_kappa_gradient_matches_central_differences():
    xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, src = _setup()
    J, g, _ = misfit_gradient(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, sources=src)
    assert abs(J - misfit(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, sources=src)) < 1e-14 * J
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.normal(size=kappa.size)
        h = 1e-5
        Jp = misfit(xyz, e2v, N, kappa + h * d, U0, dt, nsteps, Rm, data, sources=src)
        Jm = misfit(xyz, e2v, N, kappa - h * d, U0, dt, nsteps, Rm, data, sources=src)
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-7 * max(abs(fd), 1e-12), (fd, g @ d)


def test_initial_state_gradient_matches_central_differences():
    xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, src = _setup(N=1)
    J, _, gU = misfit_gradient(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, sources=src)
    rng = np.random.default_rng(6)
    d = rng.normal(size=U0.shape)
    h = 1e-4
    Jp = misfit(xyz, e2v, N, kappa, U0 + h * d, dt, nsteps, Rm, data, sources=src)
    Jm = misfit(xyz, e2v, N, kappa, U0 - h * d, dt, nsteps, Rm, data, sources=src)
    fd = (Jp - Jm) / (2 * h)
    assert abs(fd - float((gU * d).sum())) <= 1e-8 * abs(fd)


def test_operator_is_skew_in_energy_product_for_central_flux():
    """W A + A^T W = 0 for alpha = 0 (W = blkdiag(M/kappa, rho M, ...)): the
    transpose the adjoint uses is the one the energy identity fixes."""
    xyz, e2v = hex_pyramid_mesh(1, seed=2)
    K = e2v.shape[0]
    N = 2
    rng = np.random.default_rng(1)
    kappa = rng.uniform(0.5, 2.0, K)
    A = operator_matrix(xyz, e2v, N, kappa=kappa, alpha=0.0)
    dg = AcousticDG(xyz, e2v, N, kappa=kappa)
    U = random_state(K, N, seed=3).ravel()
    V = random_state(K, N, seed=4).ravel()
    # energy product <U, V>_W through the oracle's own energy (polarisation)
    def E(x):
        return dg.energy(x.reshape(K, 4, -1))
    def inner(x, y):
        return 0.5 * (E(x + y) - E(x) - E(y))
    lhs = inner(A @ U, V) + inner(U, A @ V)
    assert abs(lhs) <= 1e-11 * (abs(inner(A @ U, V)) + 1e-30)


def test_kappa_gradient_with_penalty_flux_matches_central_differences():
    """alpha = 1: kappa also enters through tau_p = alpha/{rho c} and
    tau_u = alpha {rho c} on every face (walls and free surface)."""
    for bc in ("wall", "free"):
        xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, src = _setup(seed=3)
        rho = np.random.default_rng(11).uniform(0.7, 1.4, kappa.size)
        J, g, _ = misfit_gradient(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, rho=rho, bc=bc,
                                  sources=src, alpha=1.0)
        g0 = misfit_gradient(xyz, e2v, N, kappa, U0, dt, nsteps, Rm, data, rho=rho, bc=bc,
                             sources=src, alpha=0.0)[1]
        rng = np.random.default_rng(7)
        for _ in range(3):
            d = rng.normal(size=kappa.size)
            h = 1e-5
            Jp = misfit(xyz, e2v, N, kappa + h * d, U0, dt, nsteps, Rm, data, rho=rho, bc=bc,
                        sources=src, alpha=1.0)
            Jm = misfit(xyz, e2v, N, kappa - h * d, U0, dt, nsteps, Rm, data, rho=rho, bc=bc,
                        sources=src, alpha=1.0)
            fd = (Jp - Jm) / (2 * h)
            assert abs(fd - g @ d) <= 1e-7 * max(abs(fd), 1e-12), (bc, fd, g @ d)
        # the penalty terms are not negligible here
        assert np.abs(g - g0).max() > 1e-3 * np.abs(g).max()
