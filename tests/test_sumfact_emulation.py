"""The sum-factorised kernels (kernels_sumfact.hip) compiled for the CPU with
AddressSanitizer (tests/cpu_emu) against the oracle: every access stays in
its buffer and the right-hand side and LSRK steps meet the FP64 bar, for
every order, in the whole-hexahedron variant (triangle traces exchanged in
LDS) and the general one (ragged and shuffled meshes, N >= 6)."""

import numpy as np
import pytest

from cpu_emu import run as emu
from gpu_helpers import rel_err_per_field
from oracle import AcousticDG, lsrk_run
from synth import hex_pyramid_mesh, random_materials, random_state, single_pyramid

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _build():
    emu.build()


@pytest.mark.parametrize("N", list(range(9)))
def test_emulated_rhs_all_orders(N):
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    rho, kap = random_materials(K, seed=N)
    U = random_state(K, N, seed=100 + N)
    ref = AcousticDG(xyz, e2v, N, rho=rho, kappa=kap).rhs(U)
    got, local = emu.run(xyz, e2v, N, U, rho=rho, kappa=kap)
    assert local == (N <= 5)
    err = rel_err_per_field(got, ref)
    assert np.all(err < TOL), err


@pytest.mark.parametrize("case", ["ragged", "shuffled", "free", "single", "hex3"])
def test_emulated_rhs_general_meshes(case):
    N, bc, alpha = 3, "wall", 1.0
    if case == "hex3":  # 162 pyramids: whole hexahedra (12 per workgroup at N = 3), the last
        xyz, e2v = hex_pyramid_mesh(3, seed=5)  # workgroup half filled
        N = 3
    elif case == "ragged":
        xyz, e2v = hex_pyramid_mesh(2, seed=4)
        e2v = e2v[:13]
    elif case == "shuffled":
        xyz, e2v = hex_pyramid_mesh(3, seed=3, shuffle=True)
        N = 4
    elif case == "free":
        xyz, e2v = hex_pyramid_mesh(2, seed=2)
        bc, alpha = "free", 0.37
    else:
        xyz, e2v = single_pyramid()
    K = e2v.shape[0]
    U = random_state(K, N, seed=9)
    ref = AcousticDG(xyz, e2v, N, bc=bc, alpha=alpha).rhs(U)
    got, local = emu.run(xyz, e2v, N, U, bc=bc, alpha=alpha)
    assert local == (case in ("free", "hex3"))
    err = rel_err_per_field(got, ref)
    assert np.all(err < TOL), err


@pytest.mark.parametrize("N", [2, 5, 7])
def test_emulated_lsrk_steps(N):
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    K = e2v.shape[0]
    U0 = random_state(K, N, seed=7)
    o = AcousticDG(xyz, e2v, N)
    dt, n = 2e-3, 3
    ref, _ = lsrk_run(o.rhs, U0, dt, n)
    got, _ = emu.run(xyz, e2v, N, U0, nsteps=n, dt=dt)
    err = rel_err_per_field(got, ref)
    assert np.all(err < 1e-11), err
