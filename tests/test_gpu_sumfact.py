"""Sum-factorised kernels on the device beyond the shared parity cases of
test_gpu_parity.py: both boundary conditions and flux parameters, the 64^3 x 6
precision-study mesh sampled, bitwise agreement of repeated launches, the
discrete adjoint (A^T and the reverse LSRK step) on a sum-factorised context,
and agreement with the dense matrix-core path over a trajectory."""

import numpy as np
import pytest

from gpu_helpers import gpu_rhs, log, rel_err_per_field
from oracle import AcousticDG
from synth import hex_pyramid_mesh, random_materials, random_state

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _solver(xyz, e2v, N, **kw):
    import paper_1502_07703_amd as dg
    return dg.Solver(xyz, e2v, N, sum_factorized=True, **kw)


@pytest.mark.parametrize("bc", ["wall", "free"])
@pytest.mark.parametrize("alpha", [0.0, 1.0, 0.37])
@pytest.mark.parametrize("N", [2, 5])
def test_sumfact_flux_and_bc(bc, alpha, N):
    xyz, e2v = hex_pyramid_mesh(2, seed=2)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=5)
    U = random_state(K, N, seed=7)
    log(f"[sumfact] bc={bc} alpha={alpha} N={N}")
    ref = AcousticDG(xyz, e2v, N, rho=rho, kappa=kap, bc=bc, alpha=alpha).rhs(U)
    with _solver(xyz, e2v, N, rho=rho, kappa=kap, bc=bc, alpha=alpha) as s:
        got = gpu_rhs(s, U)
    err = rel_err_per_field(got, ref)
    log(f"[sumfact] rel err {err}")
    assert np.all(err < TOL), err


@pytest.mark.parametrize("N", [5, 7])
def test_sumfact_cfg3_sampled(N):
    """64^3 x 6 = 1572864 pyramids (seed 3): the device computes every
    element (whole hexahedra at N = 5, all-face traces at N = 7), the oracle a
    seeded sample of 1500 elements."""
    import torch

    import paper_1502_07703_amd as dg  # noqa: F401
    xyz, e2v = hex_pyramid_mesh(64, seed=3)
    K = e2v.shape[0]
    rng = np.random.default_rng(41 + N)
    sample = np.unique(np.concatenate([rng.choice(K, 1500, replace=False), [0, K - 1]]))
    o = AcousticDG(xyz, e2v, N, elems=sample)
    log(f"[sumfact] 64^3 x 6 K={K} N={N}")
    with _solver(xyz, e2v, N) as s:
        g = torch.Generator(device="cuda").manual_seed(50 + N)
        Uc = torch.randn((K, 4, s.Np), dtype=torch.float64, device="cuda", generator=g)
        out = s.unpack(s.rhs(s.pack(Uc)))
        got = out[torch.from_numpy(o.elems).cuda()].cpu().numpy()
        Uh = np.zeros((K, 4, s.Np))
        Uh[o.active] = Uc[torch.from_numpy(o.active).cuda()].cpu().numpy()
        del Uc, out
    err = rel_err_per_field(got, o.rhs(Uh))
    log(f"[sumfact] 64^3 x 6 N={N} rel err {err}")
    assert np.all(err < TOL), err


def test_sumfact_bitwise_deterministic():
    import torch
    N = 4
    xyz, e2v = hex_pyramid_mesh(3, seed=6)
    U = random_state(e2v.shape[0], N, seed=2)
    with _solver(xyz, e2v, N) as s:
        Ud = s.pack(torch.from_numpy(U).cuda())
        a = s.rhs(Ud).clone()
        b = s.rhs(Ud).clone()
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("N", [2, 4])
def test_sumfact_adjoint_identity_and_step(N):
    """A^T on a sum-factorised context (its trace buffer holds (p, u.n) pairs,
    the adjoint kernels use their own layout) and a reverse LSRK step with the
    penalty-coefficient gradient, against the dense path's."""
    import torch

    import paper_1502_07703_amd as dg
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=N)
    u = torch.from_numpy(random_state(K, N, seed=60 + N)).cuda()
    lam = torch.from_numpy(random_state(K, N, seed=61 + N)).cuda()
    res = {}
    for sf in (False, True):
        with dg.Solver(xyz, e2v, N, rho=rho, kappa=kap, alpha=1.0, sum_factorized=sf) as s:
            U, L = s.pack(u), s.pack(lam)
            a = float((L * s.rhs(U)).sum().item())
            ATl = s.adjoint_rhs(L)
            b = float((ATl * U).sum().item())
            Ub = L.clone()
            grad = torch.zeros(K, dtype=torch.float64, device="cuda")
            s.adjoint_step(U, Ub, grad, 0.0, 1e-3)
            res[sf] = (a, b, ATl.cpu().numpy(), Ub.cpu().numpy(), grad.cpu().numpy())
    a, b = res[True][0], res[True][1]
    log(f"[sumfact] adjoint identity N={N}: {a:.15e} vs {b:.15e}")
    assert abs(a - b) <= 1e-12 * abs(a)
    for i in (2, 3, 4):
        d, r = res[True][i], res[False][i]
        assert np.abs(d - r).max() <= 1e-11 * np.abs(r).max(), i


def test_sumfact_trajectory_matches_dense_path():
    """200 LSRK steps of the projected wall mode on 4^3 x 6 pyramids, N = 4:
    sum-factorised and dense matrix-core paths within 1e-10."""
    import torch

    import paper_1502_07703_amd as dg
    from oracle.dg import wall_mode
    N = 4
    xyz, e2v = hex_pyramid_mesh(4, seed=9)
    U0 = AcousticDG(xyz, e2v, N).project(wall_mode(1), xyz, e2v)
    out = []
    for sf in (False, True):
        with dg.Solver(xyz, e2v, N, sum_factorized=sf) as s:
            U = s.pack(torch.from_numpy(U0).cuda())
            R = s.empty_state()
            s.step(U, R, s.stable_dt(0.5), 200)
            out.append(s.unpack(U).cpu().numpy())
    err = rel_err_per_field(out[1], out[0])
    log(f"[sumfact] 200 steps vs dense path rel err {err}")
    assert np.all(err < 1e-10), err
