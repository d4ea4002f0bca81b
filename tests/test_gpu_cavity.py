"""The paper's own experiment setting (Section 4.3): the bi-unit cavity
[-1, 1]^3 with a free surface (p = 0) on every boundary face, whose first
mode is p = cos(k x) cos(k y) cos(k z) cos(w t), k = pi/2, w = sqrt(3) k,
u = sin(w t)/sqrt(3) (sin(k x) cos(k y) cos(k z), ...)."""

import numpy as np
import pytest

from gpu_helpers import log, rel_err_per_field
from oracle import AcousticDG, lsrk_run
from synth import hex_pyramid_mesh

pytestmark = pytest.mark.gpu

K_WAVE = np.pi / 2
OMEGA = np.sqrt(3.0) * K_WAVE


def cavity_mode(X, t):
    """numpy (npts, 3) -> (npts, 4)."""
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    cx, cy, cz = np.cos(K_WAVE * x), np.cos(K_WAVE * y), np.cos(K_WAVE * z)
    sx, sy, sz = np.sin(K_WAVE * x), np.sin(K_WAVE * y), np.sin(K_WAVE * z)
    a = np.sin(OMEGA * t) / np.sqrt(3.0)
    return np.stack([cx * cy * cz * np.cos(OMEGA * t), a * sx * cy * cz, a * cx * sy * cz,
                     a * cx * cy * sz], axis=-1)


def _cavity_torch(P, t):
    import torch
    x, y, z = P[..., 0], P[..., 1], P[..., 2]
    cx, cy, cz = torch.cos(K_WAVE * x), torch.cos(K_WAVE * y), torch.cos(K_WAVE * z)
    sx, sy, sz = torch.sin(K_WAVE * x), torch.sin(K_WAVE * y), torch.sin(K_WAVE * z)
    a = np.sin(OMEGA * t) / np.sqrt(3.0)
    return torch.stack([cx * cy * cz * np.cos(OMEGA * t), a * sx * cy * cz, a * cx * sy * cz,
                        a * cx * cy * sz], dim=1).contiguous()


def test_cavity_trajectory_matches_oracle():
    import torch

    import paper_1502_07703_amd as dg
    N, k1d, nsteps = 3, 2, 10
    xyz, e2v = hex_pyramid_mesh(k1d, seed=4, lo=-1.0, hi=1.0)
    o = AcousticDG(xyz, e2v, N, bc="free")
    U0 = o.project(cavity_mode, xyz, e2v)
    dt = 0.5 / (2.0 * (N + 1) * (N + 3) / 3.0 * o.inverse_length().max())
    ref, _ = lsrk_run(o.rhs, U0, dt, nsteps)
    with dg.Solver(xyz, e2v, N, bc="free") as s:
        U = s.pack(torch.from_numpy(U0).cuda())
        R = s.empty_state().zero_()
        s.step(U, R, dt, nsteps)
        got = s.unpack(U).cpu().numpy()
    err = rel_err_per_field(got, ref)
    log(f"[cavity] trajectory rel err {err}")
    assert np.all(err < 1e-11), err


def test_cavity_mode_converges():
    """L2 error at T = 0.5 after the projected initial data, on meshes with
    2^3 and 4^3 hexahedra (x 6 pyramids): the evolved error falls at least
    like h^(N + 1/2)."""
    import torch

    import paper_1502_07703_amd as dg
    N, T = 2, 0.5
    errs = []
    for k1d in (2, 4):
        xyz, e2v = hex_pyramid_mesh(k1d, seed=6, lo=-1.0, hi=1.0)
        with dg.Solver(xyz, e2v, N, bc="free") as s:
            P, wJ = s.volume_points()
            U = s.project(_cavity_torch(P, 0.0))
            R = s.empty_state().zero_()
            n = int(np.ceil(T / s.stable_dt(0.5)))
            s.step(U, R, T / n, n)
            d = s.evaluate(U) - _cavity_torch(P, T)
            errs.append(float(torch.sqrt((wJ[:, None, :] * d * d).sum()).item()))
    rate = np.log2(errs[0] / errs[1])
    log(f"[cavity] L2 errors {errs}, rate {rate:.2f}")
    assert rate > N + 0.5
