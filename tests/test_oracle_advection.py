"""Pins for the oracle's advection right-hand side (Section 4.1).

* energy identity: u^T M du/dt equals minus alpha/2 times the face integral
  of |beta_n| [[u]]^2 (zero for the central flux), for random u on periodic
  and non-periodic meshes -- a dropped factor, a wrong sign of the volume or
  face term, or a transposed operator breaks it;
* constants are steady on a periodic mesh;
* a linear u = c . x has du/dt = -beta . c exactly on elements whose faces
  all see the same linear function;
* LSRK transport of a smooth periodic wave matches u0(x - beta t) with the
  error falling as N grows (direction and speed of transport).
"""

import numpy as np
import pytest

from oracle.advection import AdvectionDG
from oracle.lsrk import lsrk_run
from synth import hex_pyramid_mesh, periodic_pair_ids

BETA = np.array([1.0, 0.3, -0.5])


@pytest.fixture(scope="module")
def periodic_mesh():
    return hex_pyramid_mesh(2, seed=1, lo=-1.0, hi=1.0)


@pytest.mark.parametrize("N", [1, 2, 3])
@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_energy_identity_periodic(periodic_mesh, N, alpha):
    xyz, e2v = periodic_mesh
    dg = AdvectionDG(xyz, e2v, N, BETA, alpha=alpha, period=(-1.0, 1.0))
    assert (dg.nb_elem >= 0).all()
    u = np.random.default_rng(10 + N).standard_normal((dg.K, dg.Np))
    rate = np.einsum("ei,eij,ej->", u, dg.M, dg.rhs(u))
    ref = dg.energy_rate(u)
    scale = np.einsum("ei,eij,ej->", u, dg.M, u)
    if alpha == 0.0:
        assert ref == 0.0
        assert abs(rate) <= 1e-13 * scale
    else:
        assert ref < 0.0
        assert abs(rate - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("alpha", [0.0, 1.0])
def test_energy_identity_open_boundary(alpha):
    xyz, e2v = hex_pyramid_mesh(2, seed=2)
    dg = AdvectionDG(xyz, e2v, 2, BETA, alpha=alpha)
    assert (dg.nb_elem < 0).sum() == 6 * 2 * 2
    u = np.random.default_rng(3).standard_normal((dg.K, dg.Np))
    rate = np.einsum("ei,eij,ej->", u, dg.M, dg.rhs(u))
    ref = dg.energy_rate(u)
    scale = np.einsum("ei,eij,ej->", u, dg.M, u)
    # central flux with a zero ghost: the boundary adds nothing either
    assert (ref == 0.0) == (alpha == 0.0)
    assert abs(rate - ref) <= 1e-13 * max(abs(ref), scale)


@pytest.mark.parametrize("N", [0, 2, 4])
def test_constant_is_steady(periodic_mesh, N):
    xyz, e2v = periodic_mesh
    dg = AdvectionDG(xyz, e2v, N, BETA, alpha=1.0, period=(-1.0, 1.0))
    u = dg.project(lambda x: np.full(x.shape[:2], 2.5))
    assert np.allclose(u @ dg.V.T, 2.5, atol=1e-13)
    assert np.abs(dg.rhs(u)).max() <= 1e-12


@pytest.mark.parametrize("N", [1, 3])
def test_linear_field_interior(N):
    xyz, e2v = hex_pyramid_mesh(3, seed=5)
    dg = AdvectionDG(xyz, e2v, N, BETA, alpha=1.0)
    c = np.array([0.7, -1.1, 0.4])
    u = dg.project(lambda x: x @ c)
    r = dg.rhs(u)
    # the 6 pyramids of the centre hexahedron (1, 1, 1) only see the linear field
    centre = 6 * (1 + 3 * (1 + 3 * 1)) + np.arange(6)
    vals = r[centre] @ dg.V.T
    assert np.allclose(vals, -BETA @ c, atol=1e-12)
    # everywhere else the field differs (boundary ghosts are zero)
    assert not np.allclose(r @ dg.V.T, -BETA @ c, atol=1e-6)


def test_transport_of_periodic_wave(periodic_mesh):
    xyz, e2v = periodic_mesh
    k = np.pi * np.array([1.0, 1.0, 0.0])

    def wave(t):
        return lambda x: np.sin((x - BETA * t) @ k)

    T, nsteps = 0.25, 50
    errs = []
    for N in (3, 4, 5):
        dg = AdvectionDG(xyz, e2v, N, BETA, alpha=1.0, period=(-1.0, 1.0))
        u = dg.project(wave(0.0))
        u = lsrk_run(lambda U, t: dg.rhs(U), u, T / nsteps, nsteps)[0]
        errs.append(dg.l2_error(u, wave(T)))
    assert errs[0] < 0.1
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1]
    # transporting the other way is far off
    dg = AdvectionDG(xyz, e2v, 4, BETA, alpha=1.0, period=(-1.0, 1.0))
    u = lsrk_run(lambda U, t: dg.rhs(U), dg.project(wave(0.0)), T / nsteps, nsteps)[0]
    assert dg.l2_error(u, wave(-T)) > 10 * errs[2]


def test_periodic_pair_ids_match_geometric_pairs(periodic_mesh):
    xyz, e2v = periodic_mesh
    ids = periodic_pair_ids(xyz)
    dg = AdvectionDG(xyz, e2v, 1, BETA, period=(-1.0, 1.0))
    fv = ((0, 1, 2, 3), (0, 3, 4), (1, 2, 4), (0, 1, 4), (3, 2, 4))
    for e in range(dg.K):
        for f in range(5):
            nb, g = dg.nb_elem[e, f], dg.nb_face[e, f]
            a = sorted(ids[e2v[e, list(fv[f])]])
            b = sorted(ids[e2v[nb, list(fv[g])]])
            assert a == b
