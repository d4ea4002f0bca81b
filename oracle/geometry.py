"""Bedrosian vertex functions and the vertex map of Section 2 (oracle).

On the bi-unit pyramid (apex at (r, s, t) = (-1, -1, 1)), with D = 2(1 - t):
  v_(-1,-1) = (r+t)(s+t)/D        v_(-1,+1) = -(r+t)(s+1)/D
  v_(+1,-1) = -(r+1)(s+t)/D       v_(+1,+1) = (r+1)(s+1)/D
  v_apex    = (1+t)/2
The paper prints the third function as -(r+t)(s+t)/D, which is minus the
first; the function that vanishes at every other vertex and equals 1 at
(r, s) = (1, -1) on the base is -(r+1)(s+t)/D, used here.

The returned arrays follow the element convention of the mesh tables:
index 0 <-> base corner (-1, -1), 1 <-> (+1, -1), 2 <-> (+1, +1),
3 <-> (-1, +1), 4 <-> apex.
"""

from __future__ import annotations

import numpy as np


def vertex_functions(r, s, t):
    """Values (5, npts) and gradients (5, 3, npts) of the vertex functions."""
    r = np.asarray(r, dtype=np.float64).ravel()
    s = np.asarray(s, dtype=np.float64).ravel()
    t = np.asarray(t, dtype=np.float64).ravel()
    D = 2.0 * (1.0 - t)
    D2 = D * D
    val = np.empty((5, r.size))
    grd = np.empty((5, 3, r.size))
    # (-1,-1): (r+t)(s+t)/D
    val[0] = (r + t) * (s + t) / D
    grd[0, 0] = (s + t) / D
    grd[0, 1] = (r + t) / D
    grd[0, 2] = (r + s + 2.0 * t) / D + 2.0 * (r + t) * (s + t) / D2
    # (+1,-1): -(r+1)(s+t)/D
    val[1] = -(r + 1.0) * (s + t) / D
    grd[1, 0] = -(s + t) / D
    grd[1, 1] = -(r + 1.0) / D
    grd[1, 2] = -(r + 1.0) / D - 2.0 * (r + 1.0) * (s + t) / D2
    # (+1,+1): (r+1)(s+1)/D
    val[2] = (r + 1.0) * (s + 1.0) / D
    grd[2, 0] = (s + 1.0) / D
    grd[2, 1] = (r + 1.0) / D
    grd[2, 2] = 2.0 * (r + 1.0) * (s + 1.0) / D2
    # (-1,+1): -(r+t)(s+1)/D
    val[3] = -(r + t) * (s + 1.0) / D
    grd[3, 0] = -(s + 1.0) / D
    grd[3, 1] = -(r + t) / D
    grd[3, 2] = -(s + 1.0) / D - 2.0 * (r + t) * (s + 1.0) / D2
    # apex: (1+t)/2
    val[4] = (1.0 + t) / 2.0
    grd[4, 0] = 0.0
    grd[4, 1] = 0.0
    grd[4, 2] = 0.5
    return val, grd


def map_points(verts, r, s, t):
    """Physical points F(r,s,t) = sum_i V_i v_i for each element.

    verts: (K, 5, 3).  Returns (K, npts, 3).
    """
    val, _ = vertex_functions(r, s, t)
    return np.einsum("ip,kid->kpd", val, verts)


def jacobian_matrix(verts, r, s, t):
    """G[k, p, d, m] = d x_d / d rho_m at each point (rho = r, s, t)."""
    _, grd = vertex_functions(r, s, t)
    return np.einsum("imp,kid->kpdm", grd, verts)
