"""Semi-discrete DG for linear advection on vertex-mapped pyramids (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.1: u_t + div(beta u) = 0 with a constant vector beta, here on a
cube with periodic boundary conditions.  On each element K with outward
normal n, beta_n = beta . n and the jump [[u]] = u+ - u-,
    int_K v (u_t + beta . grad u) + int_dK (beta_n - alpha |beta_n|)/2 [[u]] v = 0,
so that, in the semi-nodal basis,
    du/dt = -M^-1 (S u + L^f F),   S_ij = int_K phi_i beta . grad phi_j,
    F = (beta_n - alpha |beta_n|)/2 [[u]]  at the face points, times w sJ.
alpha = 1 gives the upwind flux, alpha = 0 the central flux.

Two readings (the printed text is inconsistent):
* the jump is printed as u- - u+; with that sign the upwind face term would
  feed energy in, contradicting the energy stability stated for alpha in
  [0, 1].  The jump here is u+ - u-, the convention of the acoustic flux of
  Section 4.3, for which (pinned in tests) u^T M du/dt = -alpha/2 sum over
  faces of int |beta_n| [[u]]^2 <= 0;
* the surface-kernel description drops the factor 1/2 of the variational
  form; the variational form decides (alpha = 0 must be the central flux).

Faces without a partner (only on non-periodic meshes) see the ghost value
u+ = 0 (homogeneous inflow data).

The cubatures are the acoustic ones (the minimal rule of Section 4.1), every
element mass matrix is assembled by quadrature and inverted through an LU
factorisation, and neighbours are found geometrically: face centroids and
face points are matched modulo the period when the mesh is periodic.
"""

from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .basis import eval_basis_rst, n_basis
from .dg import FACE_VERTS, _face_geometry
from .geometry import jacobian_matrix, map_points
from .rules import volume_rule


def _wrap_diff(d, L):
    """Differences reduced to the nearest periodic image (L: (3,) or None)."""
    if L is None:
        return d
    return d - L * np.round(d / L)


class AdvectionDG:
    """Advection DG right-hand side on a pyramid mesh.

    period: None (faces without a partner see u+ = 0) or (lo, hi): the mesh
    fills [lo, hi]^3 and opposite boundary faces are neighbours.  ``elems``
    restricts the evaluation to a subset of elements (their neighbours' traces
    are still used); ``rhs`` then returns rows for ``self.elems`` in order.
    """

    def __init__(self, xyz, e2v, N, beta, alpha=1.0, period=None, match_tol=1e-9, elems=None):
        xyz = np.asarray(xyz, dtype=np.float64)
        e2v = np.asarray(e2v, dtype=np.int64)
        K = e2v.shape[0]
        self.N, self.Np, self.K = N, n_basis(N), K
        self.beta = np.asarray(beta, dtype=np.float64).reshape(3)
        self.alpha = float(alpha)
        L = None
        if period is not None:
            lo, hi = float(period[0]), float(period[1])
            L = np.full(3, hi - lo)
        self.L = L
        S = np.arange(K) if elems is None else np.unique(np.asarray(elems, dtype=np.int64))
        self.elems = S

        # ---- neighbours by face-centroid search (geometric, periodic) -------
        fcent = np.stack([xyz[e2v[:, list(fv)]].mean(axis=1) for fv in FACE_VERTS], axis=1)
        hscale = np.linalg.norm(xyz[e2v[:, 1]] - xyz[e2v[:, 0]], axis=1).mean()
        tol = match_tol * max(hscale, 1e-300) * 10.0
        pts = fcent.reshape(-1, 3)
        if L is None:
            tree = cKDTree(pts)
        else:
            pts = np.mod(pts - lo, L)
            pts[pts >= L - tol] = 0.0
            tree = cKDTree(pts, boxsize=L)
        nb_elem = -np.ones((S.size, 5), dtype=np.int64)
        nb_face = -np.ones((S.size, 5), dtype=np.int64)
        for f in range(5):
            hits = tree.query_ball_point(pts.reshape(K, 5, 3)[S, f], r=tol)
            for row, h in enumerate(hits):
                others = [x for x in h if x != S[row] * 5 + f]
                if len(others) > 1:
                    raise ValueError("face matched more than one neighbour")
                if others:
                    nb_elem[row, f], nb_face[row, f] = divmod(others[0], 5)
        self.nb_elem, self.nb_face = nb_elem, nb_face
        active = np.unique(np.concatenate([S, nb_elem[nb_elem >= 0]]))
        pos = -np.ones(K, dtype=np.int64)
        pos[active] = np.arange(active.size)
        self.active, self._pos = active, pos

        # ---- volume: reference operators and geometry on S ------------------
        vr = volume_rule(N)
        verts = xyz[e2v[S]]
        self.vr, self.verts = vr, verts
        self.V, self.Dr, self.Ds, self.Dt = eval_basis_rst(N, vr["r"], vr["s"], vr["t"], deriv=True)
        G = jacobian_matrix(verts, vr["r"], vr["s"], vr["t"])
        J = np.linalg.det(G)
        if np.any(J <= 0.0):
            raise ValueError("non-positive Jacobian at a volume cubature point")
        self.Ginv = np.linalg.inv(G)  # Ginv[..., m, d] = d rho_m / d x_d
        self.wJ = vr["w"][None, :] * J
        self.M = np.einsum("qi,eq,qj->eij", self.V, self.wJ, self.V, optimize=True)
        self.Minv = np.linalg.inv(self.M)

        # ---- faces: normals and weights on S, points matched on the active set
        xs, ns, ws, frules = _face_geometry(verts, N)
        self.fn, self.fw = ns, ws
        self.Vf = [eval_basis_rst(N, fr["r"], fr["s"], fr["t"]) for fr in frules]
        verts_A = xyz[e2v[active]]
        xs_A = [map_points(verts_A, fr["r"], fr["s"], fr["t"]) for fr in frules]
        self.perm = []
        for f in range(5):
            nq = self.Vf[f].shape[0]
            perm = np.zeros((S.size, nq), dtype=np.int64)
            for f2 in range(5):
                sel = np.where((nb_elem[:, f] >= 0) & (nb_face[:, f] == f2))[0]
                if sel.size == 0:
                    continue
                if self.Vf[f2].shape[0] != nq:
                    raise ValueError("face type mismatch between neighbours")
                X = xs[f][sel]
                Y = xs_A[f2][pos[nb_elem[sel, f]]]
                d = np.linalg.norm(_wrap_diff(X[:, :, None, :] - Y[:, None, :, :], L), axis=3)
                am = d.argmin(axis=2)
                dmin = np.take_along_axis(d, am[:, :, None], axis=2)[..., 0]
                if np.any(dmin > tol):
                    raise ValueError("non-conforming face: face points do not coincide")
                if np.any(np.sort(am, axis=1) != np.arange(nq)[None, :]):
                    raise ValueError("face point matching is not a bijection")
                perm[sel] = am
            self.perm.append(perm)

    def jumps(self, u):
        """Per face, for the rows of S: (u- (nS, nq), u+ (nS, nq), beta_n (nS, nq)).
        u is the full (K, Np) array."""
        u = np.asarray(u, dtype=np.float64)
        uA = u[self.active]
        T = [uA @ Vf.T for Vf in self.Vf]
        rowS = self._pos[self.elems]
        out = []
        for f in range(5):
            um = T[f][rowS]
            up = np.zeros_like(um)
            for f2 in range(5):
                sel = np.where((self.nb_elem[:, f] >= 0) & (self.nb_face[:, f] == f2))[0]
                if sel.size:
                    src = T[f2][self._pos[self.nb_elem[sel, f]]]
                    up[sel] = np.take_along_axis(src, self.perm[f][sel], axis=1)
            bn = self.fn[f] @ self.beta
            out.append((um, up, bn))
        return out

    def rhs(self, u):
        """du/dt on the rows of S for the full coefficient array u (K, Np)."""
        u = np.asarray(u, dtype=np.float64)
        uS = u[self.elems]
        # volume (Algorithm 1): beta . grad u at the cubature points
        dU = np.stack([uS @ D.T for D in (self.Dr, self.Ds, self.Dt)])  # (3, nS, Nc)
        grad = np.einsum("eqmd,meq->eqd", self.Ginv, dU)
        bgrad = grad @ self.beta
        tot = (self.wJ * bgrad) @ self.V
        # surface (Algorithm 2)
        for f, (um, up, bn) in enumerate(self.jumps(u)):
            F = 0.5 * (bn - self.alpha * np.abs(bn)) * (up - um)
            tot += (self.fw[f] * F) @ self.Vf[f]
        # inverse mass (Algorithm 3)
        return -np.einsum("eij,ej->ei", self.Minv, tot)

    def energy_rate(self, u):
        """What u^T M du/dt must equal when S and the face integrals are exact:
        -alpha/2 int |beta_n| [[u]]^2 over every interior face (each face is
        visited from both sides, hence -alpha/4 per side), plus, on faces
        without a partner (ghost u+ = 0), -int (beta_n u-^2 / 2 + u- F)."""
        rate = 0.0
        for f, (um, up, bn) in enumerate(self.jumps(u)):
            w = self.fw[f]
            inner = self.nb_elem[:, f] >= 0
            j2 = (up - um) ** 2
            rate += -0.25 * self.alpha * np.sum((w * np.abs(bn) * j2)[inner])
            if np.any(~inner):
                F = 0.5 * (bn - self.alpha * np.abs(bn)) * (up - um)
                b = ~inner
                rate += np.sum((w * (-0.5 * bn * um * um - um * F))[b])
        return rate

    def points(self):
        """Physical volume cubature points of the elements of S (nS, Nc, 3)."""
        return map_points(self.verts, self.vr["r"], self.vr["s"], self.vr["t"])

    def project(self, fun):
        """L2 projection of fun(x (nS, Nc, 3)) -> (nS, Nc) onto the basis of each element of S."""
        f = fun(self.points())
        return np.einsum("eij,ej->ei", self.Minv, (self.wJ * f) @ self.V)

    def l2_error(self, u, fun):
        """sqrt(sum_K int_K (u_h - fun)^2) on the volume rule."""
        d = u @ self.V.T - fun(self.points())
        return float(np.sqrt(np.sum(self.wJ * d * d)))
