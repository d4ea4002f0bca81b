"""Quadrature rules on the collapsed cube and the pyramid (oracle).

Section 2: the Duffy-type map r = (1+a)(1-c)/2 - 1, s = (1+b)(1-c)/2 - 1,
t = c takes [-1,1]^3 onto the bi-unit pyramid with change-of-variables factor
((1-c)/2)^2.

Section 4.1: the volume rule is the tensor product of (N+1)-point
Gauss-Legendre in a and b with an (N+1)-point Gauss-Jacobi (2,0) rule in c,
mapped to the pyramid.  The paper leaves the surface rule unspecified beyond
"minimal points that integrate the mass matrix exactly"; the reading used here
is an (N+1)^2 Gauss-Legendre grid on the base and, on each triangle, (N+1)
Gauss-Legendre points along the edge times (N+1) Gauss-Jacobi (1,0) points
collapsed towards the apex.
"""

from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi, roots_legendre


def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    x, w = roots_legendre(n)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gauss_jacobi(n: int, alpha: float):
    """n-point Gauss-Jacobi rule for the weight (1 - x)^alpha on [-1, 1]."""
    x, w = roots_jacobi(n, alpha, 0.0)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def collapse(a, b, c):
    """Duffy-type map (a, b, c) -> (r, s, t) of Section 2."""
    r = (1.0 + a) * (1.0 - c) / 2.0 - 1.0
    s = (1.0 + b) * (1.0 - c) / 2.0 - 1.0
    return r, s, np.array(c, dtype=np.float64, copy=True)


def volume_rule(N: int, npts: int | None = None):
    """Collapsed tensor-product rule on the reference pyramid.

    With ``npts = N + 1`` (default) this is the minimal rule of Section 4.1.
    Returns a dict with the collapsed coordinates a, b, c, the reference
    coordinates r, s, t and reference weights w (the pyramid's volume element
    dr ds dt = ((1-c)/2)^2 da db dc is folded into w).
    """
    n = N + 1 if npts is None else npts
    xa, wa = gauss_legendre(n)
    xc, wc = gauss_jacobi(n, 2.0)
    A, B, C = np.meshgrid(xa, xa, xc, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wa, wc, indexing="ij")
    a, b, c = A.ravel(), B.ravel(), C.ravel()
    # Gauss-Jacobi(2,0) integrates against (1-c)^2 = 4 ((1-c)/2)^2.
    w = (WA * WB * WC).ravel() / 4.0
    r, s, t = collapse(a, b, c)
    return dict(a=a, b=b, c=c, r=r, s=s, t=t, w=w)


# Faces of the reference pyramid, in the order used throughout:
#   0: base t = -1       1: r = -1       2: r = -t       3: s = -1       4: s = -t
FACE_NAMES = ("t=-1", "r=-1", "r=-t", "s=-1", "s=-t")


def face_rules(N: int, npts: int | None = None):
    """Per-face reference points and weights.

    Each entry is a dict with reference coordinates r, s, t of the points,
    the reference weight w of the face parametrisation, and ``tang`` -- a pair
    of reference-space vectors (d(r,s,t)/dp1, d(r,s,t)/dp2) for the face's
    parameters (p1, p2), so that the physical area element is
    |(G tang[0]) x (G tang[1])| dp1 dp2 with G the map's Jacobian matrix.
    """
    n = N + 1 if npts is None else npts
    xg, wg = gauss_legendre(n)
    xj, wj = gauss_jacobi(n, 1.0)
    faces = []
    # base: parameters (r, s) on [-1,1]^2
    R, S = np.meshgrid(xg, xg, indexing="ij")
    WR, WS = np.meshgrid(wg, wg, indexing="ij")
    faces.append(dict(r=R.ravel(), s=S.ravel(), t=-np.ones(n * n), w=(WR * WS).ravel(),
                      tang=(np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))))
    # triangles: edge parameter sigma (GL) and c (GJ(1,0)); the in-face
    # coordinate q = (1+sigma)(1-c)/2 - 1 runs over [-1, -c]; dq dc =
    # ((1-c)/2) dsigma dc and GJ(1,0) integrates against (1-c) = 2 (1-c)/2.
    SG, CC = np.meshgrid(xg, xj, indexing="ij")
    WSG, WCC = np.meshgrid(wg, wj, indexing="ij")
    sg, cc = SG.ravel(), CC.ravel()
    wt = (WSG * WCC).ravel() / 2.0
    q = (1.0 + sg) * (1.0 - cc) / 2.0 - 1.0
    one = np.ones_like(cc)
    # r = -1: parameters (s, t)
    faces.append(dict(r=-one, s=q, t=cc, w=wt,
                      tang=(np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0]))))
    # r = -t: parameters (s, t), r follows -t
    faces.append(dict(r=-cc, s=q, t=cc, w=wt,
                      tang=(np.array([0.0, 1.0, 0.0]), np.array([-1.0, 0.0, 1.0]))))
    # s = -1: parameters (r, t)
    faces.append(dict(r=q, s=-one, t=cc, w=wt,
                      tang=(np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0]))))
    # s = -t: parameters (r, t), s follows -t
    faces.append(dict(r=q, s=-cc, t=cc, w=wt,
                      tang=(np.array([1.0, 0.0, 0.0]), np.array([0.0, -1.0, 1.0]))))
    return faces
