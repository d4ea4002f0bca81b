"""The transposed operator (dgpyr_adjoint_rhs) against the oracle's assembled
A^T on small meshes, and the adjoint identity <lam, A u> = <A^T lam, u> with
the device's own forward operator at every order and at the benchmark size."""

import numpy as np
import pytest

from gpu_helpers import log, rel_err_per_field
from oracle.adjoint import operator_matrix
from synth import hex_pyramid_mesh, random_materials, random_state

pytestmark = pytest.mark.gpu


def _solver(xyz, e2v, N, **kw):
    import paper_1502_07703_amd as dg
    return dg.Solver(xyz, e2v, N, **kw)


@pytest.mark.parametrize("N", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("alpha,bc", [(0.0, "wall"), (1.0, "wall"), (0.37, "free")])
def test_adjoint_rhs_matches_oracle_transpose(N, alpha, bc):
    import torch
    xyz, e2v = hex_pyramid_mesh(1, seed=N + 3)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=N)
    A = operator_matrix(xyz, e2v, N, rho=rho, kappa=kap, bc=bc, alpha=alpha)
    lam = random_state(K, N, seed=40 + N)
    ref = (A.T @ lam.ravel()).reshape(lam.shape)
    with _solver(xyz, e2v, N, rho=rho, kappa=kap, bc=bc, alpha=alpha) as s:
        L = s.pack(torch.from_numpy(lam).cuda())
        got = s.unpack(s.adjoint_rhs(L)).cpu().numpy()
    err = rel_err_per_field(got, ref)
    log(f"[adjoint] N={N} alpha={alpha} bc={bc} rel err {err}")
    assert np.all(err < 1e-12), err


def _identity_gap(s, K, N, seed):
    import torch
    u = torch.from_numpy(random_state(K, N, seed=seed)).cuda()
    lam = torch.from_numpy(random_state(K, N, seed=seed + 1)).cuda()
    U = s.pack(u)
    L = s.pack(lam)
    Au = s.rhs(U)
    ATl = s.adjoint_rhs(L)
    a = float((L * Au).sum().item())
    b = float((ATl * U).sum().item())
    scale = float(L.norm().item() * Au.norm().item())
    return abs(a - b) / scale, a, b


@pytest.mark.parametrize("N", list(range(0, 9)))
def test_adjoint_identity_all_orders(N):
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=N)
    with _solver(xyz, e2v, N, rho=rho, kappa=kap, alpha=1.0) as s:
        gap, a, b = _identity_gap(s, K, N, 50 + N)
    log(f"[adjoint] identity N={N}: {a:.15e} vs {b:.15e} (gap {gap:.2e})")
    assert gap < 1e-13


def test_adjoint_identity_full_size():
    """40^3 x 6 = 384000 pyramids, N = 4: a property that holds at any size."""
    xyz, e2v = hex_pyramid_mesh(40, seed=2)
    K = e2v.shape[0]
    with _solver(xyz, e2v, 4, alpha=1.0) as s:
        gap, a, b = _identity_gap(s, K, 4, 7)
    log(f"[adjoint] identity full size: {a:.15e} vs {b:.15e} (gap {gap:.2e})")
    assert gap < 1e-13


def _misfit_case(N, k1d, nsteps, nrec, seed):
    from oracle import AcousticDG
    from oracle.dg import wall_mode
    xyz, e2v = hex_pyramid_mesh(k1d, seed=seed)
    K = e2v.shape[0]
    rng = np.random.default_rng(seed)
    kap = rng.uniform(0.5, 2.0, K)
    U0 = AcousticDG(xyz, e2v, N).project(wall_mode(1), xyz, e2v)
    pts = rng.uniform(0.15, 0.85, (nrec, 3))
    data = rng.normal(0.0, 0.1, (nsteps, nrec))
    src = [dict(x=[0.4, 0.55, 0.45], f0=10.0)]
    return xyz, e2v, kap, U0, pts, data, src


def _gpu_misfit(xyz, e2v, N, kap, U0, pts, data, src, dt, nsteps, every, grad=True, alpha=0.0,
                bc="wall", rho=None, reserve=False):
    import torch

    import paper_1502_07703_amd as dg
    from paper_1502_07703_amd.adjoint import receiver_misfit
    s = dg.Solver(xyz, e2v, N, alpha=alpha, bc=bc, rho=rho, sources=src, adjoint=reserve)
    s.set_receivers(pts)
    U = s.pack(torch.from_numpy(U0).cuda())
    k = torch.tensor(kap, dtype=torch.float64, requires_grad=grad)
    J = receiver_misfit(k, s, U, torch.from_numpy(data).cuda(), dt, nsteps, every)
    g = None
    if grad:
        J.backward()
        g = k.grad.numpy().copy()
    out = float(J.item())
    s.close()
    return out, g


@pytest.mark.parametrize("reserve", [False, True])
def test_misfit_gradient_matches_oracle_discrete_adjoint(reserve):
    """reserve: every adjoint buffer reserved at setup (DGPYR_FLAG_ADJOINT), so
    receivers and adjoint steps allocate nothing afterwards."""
    from oracle.adjoint import misfit_gradient, receiver_matrix
    N, nsteps, dt = 2, 6, 0.02
    xyz, e2v, kap, U0, pts, data, src = _misfit_case(N, 1, nsteps, 4, 3)
    Rm = receiver_matrix(xyz, e2v, N, pts)
    J_ref, g_ref, _ = misfit_gradient(xyz, e2v, N, kap, U0, dt, nsteps, Rm, data, sources=src)
    J, g = _gpu_misfit(xyz, e2v, N, kap, U0, pts, data, src, dt, nsteps, every=4,
                       reserve=reserve)
    log(f"[adjoint] J {J:.15e} oracle {J_ref:.15e}")
    assert abs(J - J_ref) <= 1e-12 * J_ref
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    log(f"[adjoint] kappa gradient rel err {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_misfit_gradient_central_differences(alpha):
    """Gradient through the device adjoint against central differences of the
    device misfit on 10 seeded directions (162 pyramids, N = 3, 30 steps,
    checkpoints every 10), central and penalty flux."""
    N, nsteps, dt = 3, 30, 0.01
    xyz, e2v, kap, U0, pts, data, src = _misfit_case(N, 3, nsteps, 8, 5)
    J, g = _gpu_misfit(xyz, e2v, N, kap, U0, pts, data, src, dt, nsteps, every=10, alpha=alpha)
    rng = np.random.default_rng(9)
    for i in range(10):
        d = rng.normal(size=kap.size)
        h = 1e-4
        Jp, _ = _gpu_misfit(xyz, e2v, N, kap + h * d, U0, pts, data, src, dt, nsteps, 10, False,
                            alpha=alpha)
        Jm, _ = _gpu_misfit(xyz, e2v, N, kap - h * d, U0, pts, data, src, dt, nsteps, 10, False,
                            alpha=alpha)
        fd = (Jp - Jm) / (2 * h)
        log(f"[adjoint] direction {i}: fd {fd:.12e} adjoint {g @ d:.12e}")
        assert abs(fd - g @ d) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("k1d,N,bc", [(1, 2, "wall"), (1, 2, "free"), (2, 1, "wall")])
def test_misfit_gradient_penalty_flux_matches_oracle(k1d, N, bc):
    """alpha = 1: kappa also enters the penalty coefficients of every face;
    heterogeneous rho, walls or free surface, interior quad faces (k1d = 2)."""
    from oracle.adjoint import misfit_gradient, receiver_matrix
    nsteps, dt = 6, 0.02
    xyz, e2v, kap, U0, pts, data, src = _misfit_case(N, k1d, nsteps, 4, 3)
    rho = np.random.default_rng(11).uniform(0.7, 1.4, kap.size)
    Rm = receiver_matrix(xyz, e2v, N, pts)
    J_ref, g_ref, _ = misfit_gradient(xyz, e2v, N, kap, U0, dt, nsteps, Rm, data, rho=rho, bc=bc,
                                      sources=src, alpha=1.0)
    log(f"[adjoint] penalty flux k1d={k1d} N={N} {bc}")
    J, g = _gpu_misfit(xyz, e2v, N, kap, U0, pts, data, src, dt, nsteps, every=4, alpha=1.0,
                       bc=bc, rho=rho)
    assert abs(J - J_ref) <= 1e-12 * J_ref
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    log(f"[adjoint] penalty flux kappa gradient rel err {err:.2e}")
    assert err < 1e-10


def test_set_kappa_updates_cfl_step_and_reserved_receivers():
    """New material: the CFL step of Section 4.3 follows the new sound speeds
    (c = 2 everywhere halves it); the receiver tables reserved at setup take
    up to DGPYR_MAX_RESERVED_RECEIVERS points and reject more."""
    from oracle import AcousticDG
    import paper_1502_07703_amd as dg
    from paper_1502_07703_amd import _binding as B
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    N = 3
    with _solver(xyz, e2v, N, adjoint=True) as s:
        dt1 = s.stable_dt(0.5)
        o = AcousticDG(xyz, e2v, N)
        ref = 0.5 / (2.0 * (N + 1) * (N + 3) / 3.0 * o.inverse_length().max())
        assert abs(dt1 - ref) <= 1e-12 * ref, (dt1, ref)
        s.set_kappa(np.full(K, 4.0))
        assert abs(s.stable_dt(0.5) - 0.5 * dt1) <= 1e-14 * dt1
        assert abs(s.info["inv_length_max"] - 2.0 * o.inverse_length().max()) <= \
            1e-12 * s.info["inv_length_max"]
        rng = np.random.default_rng(2)
        s.set_receivers(rng.uniform(0.1, 0.9, (B.MAX_RESERVED_RECEIVERS, 3)))
        with pytest.raises(dg.DgpyrError) as ex:
            s.set_receivers(rng.uniform(0.1, 0.9, (B.MAX_RESERVED_RECEIVERS + 1, 3)))
        assert ex.value.status == B.E_ARG
