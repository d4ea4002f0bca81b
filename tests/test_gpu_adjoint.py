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
