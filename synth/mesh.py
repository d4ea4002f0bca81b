"""Seeded pyramid meshes.

The meshes follow the construction used for every experiment on meshes in the
paper (Sections 3.2 and 4.3): a cube is cut into K1D x K1D x K1D hexahedra,
each hexahedron is split into 6 pyramids through its centroid, and vertex
positions are perturbed randomly so that the Jacobian of each pyramid's map is
non-constant.

Element-to-vertex convention (shared by every consumer): row e of ``e2v`` is
(v0, v1, v2, v3, v4); v0..v3 are the base corners, counter-clockwise when seen
from the apex v4, i.e. ((x1 - x0) x (x3 - x0)) . (x4 - x0) > 0; in collapsed
coordinates v0 sits at (a, b) = (-1, -1), v1 at (+1, -1), v2 at (+1, +1),
v3 at (-1, +1).

Perturbation (a reading of "perturbed randomly"; the paper gives no recipe):
only vertices of the hexahedral grid that lie strictly inside the cube move,
by delta = amp * h * xi / max(1, |xi|) with xi ~ U[-1, 1]^3 drawn from
``numpy.random.default_rng(seed)`` in grid order; each apex is the mean of the
8 perturbed corners of its hexahedron.  Boundary vertices stay on the cube
faces, so the domain is exactly the cube.
"""

from __future__ import annotations

import numpy as np

# Corners of a unit hexahedron, indexed by (i, j, k) bits.
_HEX_FACES = (
    # face on x = lo, x = hi, y = lo, y = hi, z = lo, z = hi; corners listed
    # as a closed loop around the face.
    ((0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1)),
    ((1, 0, 0), (1, 0, 1), (1, 1, 1), (1, 1, 0)),
    ((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 0, 0)),
    ((0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1)),
    ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)),
    ((0, 0, 1), (0, 1, 1), (1, 1, 1), (1, 0, 1)),
)


def _orient_loop(loop, centre):
    """Return the 4-corner loop ordered counter-clockwise seen from ``centre``."""
    p = [np.asarray(c, dtype=np.float64) for c in loop]
    tri = np.dot(np.cross(p[1] - p[0], p[3] - p[0]), centre - p[0])
    if tri > 0:
        return tuple(loop)
    return (loop[0], loop[3], loop[2], loop[1])


_HEX_FACES_ORIENTED = tuple(_orient_loop(f, np.array([0.5, 0.5, 0.5])) for f in _HEX_FACES)


def hex_pyramid_mesh(k1d: int, seed: int = 0, amp: float = 0.15, lo: float = 0.0,
                     hi: float = 1.0, shuffle: bool = False):
    """Cube [lo, hi]^3 as k1d^3 hexahedra, each split into 6 pyramids.

    Returns ``(xyz, e2v)``: float64 array (nverts, 3) and int64 array
    (6 * k1d**3, 5).  Without ``shuffle`` the 6 pyramids of hexahedron
    (I, J, K) are elements 6 * (I + k1d * (J + k1d * K)) + f, f = 0..5 in the
    face order x-, x+, y-, y+, z-, z+.  With ``shuffle`` the element order is
    permuted and each base loop is rotated by a random number of positions
    (keeping its orientation), from a second seeded stream.
    """
    if k1d < 1:
        raise ValueError("k1d must be >= 1")
    n1 = k1d + 1
    h = (hi - lo) / k1d
    g = np.linspace(lo, hi, n1)
    # grid vertex (i, j, k) -> i + n1 * (j + n1 * k)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    grid = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=grid.shape)
    nrm = np.maximum(1.0, np.linalg.norm(xi, axis=1))[:, None]
    delta = amp * h * xi / nrm
    kk, jj, ii = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    interior = ((ii > 0) & (ii < k1d) & (jj > 0) & (jj < k1d) & (kk > 0) & (kk < k1d)).ravel()
    grid = grid + delta * interior[:, None]

    nhex = k1d ** 3
    KH, JH, IH = np.meshgrid(np.arange(k1d), np.arange(k1d), np.arange(k1d), indexing="ij")
    IH, JH, KH = IH.ravel(), JH.ravel(), KH.ravel()

    def vid(di, dj, dk):
        return (IH + di) + n1 * ((JH + dj) + n1 * (KH + dk))

    corners = np.stack([vid(i, j, k) for k in (0, 1) for j in (0, 1) for i in (0, 1)], axis=1)
    apex_xyz = grid[corners].mean(axis=1)
    apex_id = grid.shape[0] + np.arange(nhex)
    xyz = np.concatenate([grid, apex_xyz], axis=0)

    e2v = np.empty((nhex, 6, 5), dtype=np.int64)
    for f, loop in enumerate(_HEX_FACES_ORIENTED):
        for v, (i, j, k) in enumerate(loop):
            e2v[:, f, v] = vid(i, j, k)
        e2v[:, f, 4] = apex_id
    e2v = e2v.reshape(nhex * 6, 5)

    if shuffle:
        rng2 = np.random.default_rng(seed + 7919)
        perm = rng2.permutation(e2v.shape[0])
        e2v = e2v[perm]
        rot = rng2.integers(0, 4, size=e2v.shape[0])
        base = e2v[:, :4].copy()
        for r in range(4):
            sel = rot == r
            e2v[sel, :4] = np.roll(base[sel], -r, axis=1)
    return xyz, e2v


def octahedron_mesh(height: float = 1.0, half: float = 1.0):
    """Two pyramids sharing the square base [-half, half]^2 x {0}.

    Element 0 has its apex at (0, 0, +height), element 1 at (0, 0, -height).
    """
    base = np.array([[-half, -half, 0.0], [half, -half, 0.0], [half, half, 0.0], [-half, half, 0.0]])
    xyz = np.concatenate([base, [[0.0, 0.0, height], [0.0, 0.0, -height]]], axis=0)
    e2v = np.array([[0, 1, 2, 3, 4], [0, 3, 2, 1, 5]], dtype=np.int64)
    return xyz, e2v


def single_pyramid():
    """The bi-unit right pyramid itself: r, s in [-1, -t], t in [-1, 1]."""
    xyz = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [1.0, 1.0, -1.0],
                    [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
    return xyz, np.arange(5, dtype=np.int64)[None, :]


def warped_pyramid(gamma: float):
    """Reference pyramid whose base corners are displaced out of plane by gamma.

    The base becomes a twisted (non-planar) quadrilateral and the apex is
    shifted sideways, so the map is non-affine with a non-constant Jacobian.
    """
    xyz, e2v = single_pyramid()
    xyz = xyz.copy()
    xyz[:4, 2] += 0.25 * gamma * np.array([1.0, -1.0, 1.0, -1.0])
    xyz[:4, 0] += 0.1 * gamma * np.array([0.0, 1.0, 0.5, -0.5])
    xyz[4, :2] += 0.3 * gamma
    return xyz, e2v


def periodic_pair_ids(xyz, lo: float = -1.0, hi: float = 1.0, tol: float = 1e-9):
    """Vertex identities of the periodic cube [lo, hi]^3: vertices whose
    coordinates agree modulo hi - lo share one id (the lowest vertex index
    among them); every other vertex keeps its own index.  Meshes from
    ``hex_pyramid_mesh`` keep their boundary vertices on the regular grid, so
    opposite boundary faces then have equal vertex-id sets."""
    xyz = np.asarray(xyz, dtype=np.float64)
    L = hi - lo
    w = np.mod(xyz - lo, L)
    w[w >= L - tol] = 0.0
    key = np.round(w / (tol * 10.0)).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    return first[inv.ravel()].astype(np.int64)
