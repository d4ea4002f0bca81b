"""Pins for the vertex map of Section 2 and Lemma 1 in the oracle."""

import numpy as np
import pytest

from oracle.dg import _face_geometry
from oracle.geometry import jacobian_matrix, map_points, vertex_functions
from oracle.rules import collapse, volume_rule
from synth import hex_pyramid_mesh, single_pyramid, warped_pyramid

REF = single_pyramid()[0]


def test_vertex_functions_partition_of_unity_and_nodality():
    rng = np.random.default_rng(0)
    a, b, c = rng.uniform(-1, 0.99, (3, 50))
    r, s, t = collapse(a, b, c)
    val, grd = vertex_functions(r, s, t)
    assert np.allclose(val.sum(axis=0), 1.0, atol=1e-14)
    assert np.allclose(grd.sum(axis=0), 0.0, atol=1e-12)
    # nodal at the four base corners (t = -1)
    corners = REF[:4]
    val, _ = vertex_functions(corners[:, 0], corners[:, 1], corners[:, 2])
    assert np.allclose(val[:4], np.eye(4), atol=1e-15)
    assert np.allclose(val[4], 0.0)
    # the apex function is 1 at t = 1 and the base functions tend to 0 there
    val, _ = vertex_functions(np.array([-1.0 + 1e-9]), np.array([-1.0 + 1e-9]), np.array([1.0 - 1e-9]))
    assert abs(val[4, 0] - 1.0) < 1e-8 and np.all(np.abs(val[:4, 0]) < 1e-8)


def test_identity_map_has_unit_jacobian():
    vr = volume_rule(4)
    G = jacobian_matrix(REF[None], vr["r"], vr["s"], vr["t"])
    assert np.allclose(G, np.eye(3), atol=1e-13)
    X = map_points(REF[None], vr["r"], vr["s"], vr["t"])[0]
    assert np.allclose(X, np.stack([vr["r"], vr["s"], vr["t"]], axis=1), atol=1e-14)


def test_affine_map_has_constant_jacobian():
    rng = np.random.default_rng(3)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    verts = REF @ A.T + b
    vr = volume_rule(3)
    G = jacobian_matrix(verts[None], vr["r"], vr["s"], vr["t"])
    assert np.allclose(G, A[None, None], atol=1e-12)


@pytest.mark.parametrize("gamma", [0.2, 0.5, 1.0])
def test_lemma1_jacobian_bilinear_in_ab_constant_in_c(gamma):
    """Lemma 1: J in Q_{1,1,0}; the whole Jacobian matrix depends on (a, b) only."""
    verts = warped_pyramid(gamma)[0]
    rng = np.random.default_rng(4)
    a, b = rng.uniform(-1, 1, (2, 30))
    Gs = []
    for c in (-0.9, -0.2, 0.4, 0.95):
        r, s, t = collapse(a, b, np.full_like(a, c))
        Gs.append(jacobian_matrix(verts[None], r, s, t)[0])
    for G in Gs[1:]:
        assert np.allclose(G, Gs[0], atol=1e-12)
    J = np.linalg.det(Gs[0])
    basis = np.stack([np.ones_like(a), a, b, a * b], axis=1)
    coef, *_ = np.linalg.lstsq(basis, J, rcond=None)
    assert np.max(np.abs(basis @ coef - J)) < 1e-12
    assert abs(coef[3]) > 1e-6 or gamma == 0  # genuinely non-constant


def test_reference_face_normals_and_areas():
    xs, ns, ws, _ = _face_geometry(REF[None], 3)
    expect_n = [(0, 0, -1), (-1, 0, 0), (1 / np.sqrt(2), 0, 1 / np.sqrt(2)),
                (0, -1, 0), (0, 1 / np.sqrt(2), 1 / np.sqrt(2))]
    expect_a = [4.0, 2.0, 2.0 * np.sqrt(2.0), 2.0, 2.0 * np.sqrt(2.0)]
    for f in range(5):
        assert np.allclose(ns[f][0], np.array(expect_n[f])[None], atol=1e-14)
        assert abs(ws[f][0].sum() - expect_a[f]) < 1e-13


def test_closed_surface_normals_sum_to_zero():
    xyz, e2v = hex_pyramid_mesh(3, seed=9)
    verts = xyz[e2v]
    xs, ns, ws, _ = _face_geometry(verts, 2)
    tot = sum(np.einsum("kq,kqd->kd", ws[f], ns[f]) for f in range(5))
    assert np.max(np.abs(tot)) < 1e-14


def test_mesh_volumes_sum_to_cube():
    xyz, e2v = hex_pyramid_mesh(4, seed=2)
    vr = volume_rule(1)
    J = np.linalg.det(jacobian_matrix(xyz[e2v], vr["r"], vr["s"], vr["t"]))
    assert np.all(J > 0)
    assert abs((J * vr["w"]).sum() - 1.0) < 1e-13


def test_mesh_orientation_convention():
    xyz, e2v = hex_pyramid_mesh(3, seed=5, shuffle=True)
    x = xyz[e2v]
    tri = np.einsum("kd,kd->k", np.cross(x[:, 1] - x[:, 0], x[:, 3] - x[:, 0]), x[:, 4] - x[:, 0])
    assert np.all(tri > 0)
