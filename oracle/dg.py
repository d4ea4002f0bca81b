"""Semi-discrete DG for first-order acoustics on vertex-mapped pyramids (oracle).

Section 4.3: with piecewise-constant density rho and bulk modulus kappa,
    (1/kappa) p_t + div u = f,      rho u_t + grad p = 0,
and, on each element K with outward normal n, jumps [[q]] = q+ - q-,
tau_p = 1/{rho c}, tau_u = {rho c}, c^2 = kappa/rho,
    int_K (p_t/kappa + div u) v + int_dK 1/2 (n.[[u]] - tau_p [[p]]) v = int_K f v
    int_K (rho u_t + grad p) v + int_dK n 1/2 ([[p]] - tau_u n.[[u]]) v = 0.
Discretised in the semi-nodal basis this is
    dp/dt   = -kappa M^-1 (sum_k S^k u_k + L^f P_p)
    du_k/dt = -(1/rho) M^-1 (S^k p + L^{f,k} P_u),
where S^k_ij = int_K phi_i d phi_j / dx_k (strong form, Algorithm 1),
L^f lifts the scalar penalty P_p and L^{f,k} lifts n_k P_u (Algorithm 2).
The printed system has rho where 1/rho belongs, S^k u_k where S^k p belongs,
and no n_k inside L^{f,k}; the variational form above decides.  The {.}
average is the arithmetic mean, as printed.  A scalar alpha multiplies both
penalties (alpha = 0: central flux, alpha = 1: the flux of Section 4.3).

Boundary conditions by mirror states: wall (n.u = 0) p+ = p-,
u+ = u- - 2 (n.u-) n; free surface (p = 0) p+ = -p-, u+ = u-; the ghost has
the element's own material.

Everything here is plain FP64 NumPy: every element mass matrix M_K is
assembled by quadrature and inverted through an LU factorisation
(numpy.linalg.inv, LAPACK getrf/getri); neighbours are found geometrically
by matching face-point coordinates.
"""

from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .basis import eval_basis_rst, n_basis
from .geometry import jacobian_matrix, map_points
from .rules import face_rules, volume_rule

# Vertices on each reference face, faces ordered t=-1, r=-1, r=-t, s=-1, s=-t.
FACE_VERTS = ((0, 1, 2, 3), (0, 3, 4), (1, 2, 4), (0, 1, 4), (3, 2, 4))


def _face_geometry(verts, N, npts=None):
    """Physical points, unit outward normals and weight*|n dS| on every face.

    Returns lists (one entry per face) of arrays x (K, nq, 3), n (K, nq, 3),
    wsJ (K, nq), and the face rules.
    """
    rules = face_rules(N, npts)
    centre = verts.mean(axis=1)  # (K, 3)
    xs, ns, ws = [], [], []
    for fr in rules:
        x = map_points(verts, fr["r"], fr["s"], fr["t"])
        G = jacobian_matrix(verts, fr["r"], fr["s"], fr["t"])
        t1 = np.einsum("kpdm,m->kpd", G, fr["tang"][0])
        t2 = np.einsum("kpdm,m->kpd", G, fr["tang"][1])
        nv = np.cross(t1, t2)
        # orient outward: away from the element's vertex mean
        side = np.einsum("kpd,kpd->k", nv, x - centre[:, None, :])
        nv = nv * np.where(side >= 0.0, 1.0, -1.0)[:, None, None]
        sj = np.linalg.norm(nv, axis=2)
        xs.append(x)
        ns.append(nv / sj[..., None])
        ws.append(fr["w"][None, :] * sj)
    return xs, ns, ws, rules


def ricker(t, f0, t0=None):
    """Ricker wavelet (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = t - t0,
    t0 = 1/f0 by default."""
    t0 = 1.0 / f0 if t0 is None else t0
    a = (np.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def locate_point(verts, x, tol=1e-12, maxit=50):
    """Reference coordinates (r, s, t) of physical point x in a pyramid with
    vertices verts (5, 3), by Newton iteration on Bedrosian's vertex map from
    the reference centroid.  Returns (rst, inside) with inside judged on the
    reference pyramid r, s in [-1, -t], t in [-1, 1] (slack 1e-10)."""
    lo, hi = verts.min(axis=0), verts.max(axis=0)
    pad = 1e-9 * max(1.0, float(np.abs(hi - lo).max()))
    if np.any(x < lo - pad) or np.any(x > hi + pad):
        return None, False
    rst = np.array([-0.5, -0.5, -0.5])
    for _ in range(maxit):
        r, s, t = rst
        t = min(t, 1.0 - 1e-12)
        X = map_points(verts[None], np.array([r]), np.array([s]), np.array([t]))[0, 0]
        G = jacobian_matrix(verts[None], np.array([r]), np.array([s]), np.array([t]))[0, 0]
        try:
            d = np.linalg.solve(G, x - X)
        except np.linalg.LinAlgError:
            return None, False
        rst = np.array([r, s, t]) + d
        if np.linalg.norm(d) < tol:
            break
    r, s, t = rst
    sl = 1e-10
    inside = (-1 - sl <= t <= 1 + sl) and (-1 - sl <= r <= -t + sl) and (-1 - sl <= s <= -t + sl)
    return rst, inside


class AcousticDG:
    """Acoustic DG right-hand side on a pyramid mesh.

    ``elems`` restricts the evaluation to a subset of elements (their
    neighbours' traces are still used); ``rhs`` then returns values for those
    elements only, in the order of ``self.elems``.
    """

    def __init__(self, xyz, e2v, N, rho=None, kappa=None, bc="wall", alpha=1.0,
                 elems=None, match_tol=1e-9, vol_npts=None, face_npts=None, sources=None):
        xyz = np.asarray(xyz, dtype=np.float64)
        e2v = np.asarray(e2v, dtype=np.int64)
        K = e2v.shape[0]
        if bc not in ("wall", "free"):
            raise ValueError("bc must be 'wall' or 'free'")
        self.N, self.Np, self.K = N, n_basis(N), K
        self.bc, self.alpha = bc, float(alpha)
        self.rho = np.ones(K) if rho is None else np.asarray(rho, dtype=np.float64)
        self.kappa = np.ones(K) if kappa is None else np.asarray(kappa, dtype=np.float64)
        self.elems = np.arange(K) if elems is None else np.unique(np.asarray(elems, dtype=np.int64))
        S = self.elems

        # ---- neighbours by face-centroid search (geometric) ---------------
        fcent = np.stack([xyz[e2v[:, list(fv)]].mean(axis=1) for fv in FACE_VERTS], axis=1)
        hscale = np.linalg.norm(xyz[e2v[:, 1]] - xyz[e2v[:, 0]], axis=1).mean()
        tol = match_tol * max(hscale, 1e-300) * 10.0
        tree = cKDTree(fcent.reshape(-1, 3))
        nb_elem = -np.ones((S.size, 5), dtype=np.int64)
        nb_face = -np.ones((S.size, 5), dtype=np.int64)
        for f in range(5):
            hits = tree.query_ball_point(fcent[S, f], r=tol)
            for row, h in enumerate(hits):
                others = [x for x in h if x != S[row] * 5 + f]
                if len(others) > 1:
                    raise ValueError("face matched more than one neighbour")
                if others:
                    nb_elem[row, f], nb_face[row, f] = divmod(others[0], 5)
        active = np.unique(np.concatenate([S, nb_elem[nb_elem >= 0]]))
        pos = -np.ones(K, dtype=np.int64)
        pos[active] = np.arange(active.size)
        self.active = active
        self._sidx = pos[S]

        # ---- reference operators -------------------------------------------
        vr = volume_rule(N, vol_npts)
        self.vrule = vr
        self.V, self.Dr, self.Ds, self.Dt = eval_basis_rst(N, vr["r"], vr["s"], vr["t"], deriv=True)
        self.W = vr["w"]

        # ---- volume geometry on S --------------------------------------------
        verts_S = xyz[e2v[S]]
        G = jacobian_matrix(verts_S, vr["r"], vr["s"], vr["t"])  # (nS, Nc, 3, 3)
        self.J = np.linalg.det(G)
        if np.any(self.J <= 0.0):
            raise ValueError("non-positive Jacobian at a volume cubature point")
        self.Ginv = np.linalg.inv(G)  # Ginv[..., m, d] = d rho_m / d x_d
        wJ = self.W[None, :] * self.J
        self.M = np.einsum("qi,eq,qj->eij", self.V, wJ, self.V, optimize=True)
        self.Minv = np.linalg.inv(self.M)  # LU factorisation + inverse (LAPACK)
        self._wJ = wJ

        # ---- faces: own geometry on S, points on the active set -----------------
        xs_S, ns_S, ws_S, frules = _face_geometry(verts_S, N, face_npts)
        self.frules = frules
        self.Vf = [eval_basis_rst(N, fr["r"], fr["s"], fr["t"]) for fr in frules]
        self.nq = [fr["w"].size for fr in frules]
        self.fn, self.fw = ns_S, ws_S
        verts_A = xyz[e2v[active]]
        xs_A = [map_points(verts_A, fr["r"], fr["s"], fr["t"]) for fr in frules]

        # ---- point matching across each interior face ------------------------
        self.nb_row = []   # (nS,) row in the active set, -1 on the boundary
        self.nb_f = []     # neighbour's face id
        self.nb_perm = []  # (nS, nq) point index in the neighbour's face
        for f in range(5):
            nq = self.nq[f]
            rows = np.where(nb_elem[:, f] >= 0)[0]
            perm = np.zeros((S.size, nq), dtype=np.int64)
            for f2 in range(5):
                sel = rows[nb_face[rows, f] == f2]
                if sel.size == 0:
                    continue
                if self.nq[f2] != nq:
                    raise ValueError("face type mismatch between neighbours")
                X = xs_S[f][sel]                      # (m, nq, 3)
                Y = xs_A[f2][pos[nb_elem[sel, f]]]   # (m, nq, 3)
                d = np.linalg.norm(X[:, :, None, :] - Y[:, None, :, :], axis=3)
                am = d.argmin(axis=2)
                dmin = np.take_along_axis(d, am[:, :, None], axis=2)[..., 0]
                if np.any(dmin > tol):
                    raise ValueError("non-conforming face: face points do not coincide")
                srt = np.sort(am, axis=1)
                if np.any(srt != np.arange(nq)[None, :]):
                    raise ValueError("face point matching is not a bijection")
                perm[sel] = am
            self.nb_row.append(np.where(nb_elem[:, f] >= 0, pos[np.maximum(nb_elem[:, f], 0)], -1))
            self.nb_f.append(nb_face[:, f].copy())
            self.nb_perm.append(perm)
        self.nb_elem = nb_elem

        # ---- point sources: f = amp R(t) delta(x - x_s) in the pressure equation
        # (Section 4.3 right-hand side b); b_i = amp R(t) phi_i(xi_s) in the
        # element containing x_s (lowest element index among those containing it)
        self.sources = []
        for src in (sources or []):
            xs = np.asarray(src["x"], dtype=np.float64)
            found = None
            for row, e in enumerate(S):
                rst, inside = locate_point(xyz[e2v[e]], xs)
                if inside:
                    found = (row, rst)
                    break
            if found is None:
                continue  # not inside the evaluated subset
            row, rst = found
            phi = eval_basis_rst(N, rst[:1], rst[1:2], rst[2:3])[0]
            self.sources.append(dict(row=row, phi=phi, f0=float(src["f0"]),
                                     t0=src.get("t0"), amp=float(src.get("amp", 1.0)), rst=rst))

    # ------------------------------------------------------------------------
    def _material(self, idx):
        rho, kap = self.rho[idx], self.kappa[idx]
        return rho, kap, np.sqrt(kap / rho) * rho  # rho * c

    def traces(self, U_active):
        """Traces (nA, 4, nq) on every face of every active element."""
        return [np.einsum("qn,efn->efq", Vf, U_active) for Vf in self.Vf]

    def rhs(self, U, t=0.0, return_parts=False):
        """dU/dt for the elements in ``self.elems``.

        U: (K, 4, Np) full coefficient array (canonical layout: p, u, v, w).
        """
        U = np.asarray(U, dtype=np.float64)
        UA = U[self.active]
        US = UA[self._sidx]
        S = self.elems
        rhoS, kapS, zS = self._material(S)

        # volume term (Algorithm 1, strong form)
        dU = [np.einsum("qn,efn->efq", D, US) for D in (self.Dr, self.Ds, self.Dt)]
        # grad of each field: d/dx_d = sum_m (d rho_m / d x_d) d/d rho_m
        grad = np.einsum("eqmd,mefq->efqd", self.Ginv, np.stack(dU))
        divu = grad[:, 1, :, 0] + grad[:, 2, :, 1] + grad[:, 3, :, 2]
        gradp = grad[:, 0, :, :]  # (nS, Nc, 3)
        vol = np.empty_like(US)
        vol[:, 0] = np.einsum("qi,eq->ei", self.V, self._wJ * divu)
        for d in range(3):
            vol[:, 1 + d] = np.einsum("qi,eq->ei", self.V, self._wJ * gradp[:, :, d])

        # surface term (Algorithm 2)
        TA = self.traces(UA)
        surf = np.zeros_like(US)
        for f in range(5):
            Tm = TA[f][self._sidx]                    # (nS, 4, nq)
            n = self.fn[f]                            # (nS, nq, 3)
            Tp = np.empty_like(Tm)
            zP = zS.copy()
            inner = self.nb_row[f] >= 0
            if np.any(inner):
                rows = np.where(inner)[0]
                nbr = self.nb_row[f][rows]
                for f2 in range(5):
                    sel = self.nb_f[f][rows] == f2
                    if not np.any(sel):
                        continue
                    r2 = rows[sel]
                    src = TA[f2][nbr[sel]]           # (m, 4, nq)
                    perm = self.nb_perm[f][r2]        # (m, nq)
                    Tp[r2] = np.take_along_axis(src, perm[:, None, :], axis=2)
                zP[rows] = self._material(self.active[nbr])[2]
            bnd = ~inner
            if np.any(bnd):
                pm = Tm[bnd, 0]
                um = Tm[bnd, 1:4]                          # (m, 3, nq)
                nb = n[bnd]                                # (m, nq, 3)
                un = np.einsum("mdq,mqd->mq", um, nb)
                if self.bc == "wall":
                    Tp[bnd, 0] = pm
                    Tp[bnd, 1:4] = um - 2.0 * un[:, None, :] * np.transpose(nb, (0, 2, 1))
                else:
                    Tp[bnd, 0] = -pm
                    Tp[bnd, 1:4] = um
            zavg = 0.5 * (zS + zP)
            tau_p = self.alpha / zavg
            tau_u = self.alpha * zavg
            jp = Tp[:, 0] - Tm[:, 0]                                  # (nS, nq)
            jun = np.einsum("edq,eqd->eq", Tp[:, 1:4] - Tm[:, 1:4], n)  # n.[[u]]
            Pp = 0.5 * (jun - tau_p[:, None] * jp)
            Pu = 0.5 * (jp - tau_u[:, None] * jun)
            wf = self.fw[f]
            surf[:, 0] += np.einsum("qi,eq->ei", self.Vf[f], wf * Pp)
            for d in range(3):
                surf[:, 1 + d] += np.einsum("qi,eq->ei", self.Vf[f], wf * n[:, :, d] * Pu)

        tot = vol + surf
        for src in self.sources:
            # dp/dt = -kappa M^-1 (vol + surf - b)
            tot[src["row"], 0] -= src["amp"] * ricker(t, src["f0"], src["t0"]) * src["phi"]
        out = np.einsum("eij,efj->efi", self.Minv, tot)
        out[:, 0] *= -kapS[:, None]
        out[:, 1:] *= -(1.0 / rhoS)[:, None, None]
        if return_parts:
            return out, vol, surf
        return out

    # ------------------------------------------------------------------------
    def element_operators(self):
        """Per-element M, strong stiffness S^k and face matrices E^k (Section 4.1).

        S^k_ij = int_K phi_i d phi_j / dx_k, E^k_ij = int_dK phi_i phi_j n_k,
        both by the rules this object was built with.  Shapes (nS, Np, Np) and
        (3, nS, Np, Np).
        """
        Dx = np.einsum("eqmd,mqj->deqj", self.Ginv, np.stack([self.Dr, self.Ds, self.Dt]))
        S = np.einsum("qi,eq,deqj->deij", self.V, self._wJ, Dx, optimize=True)
        E = np.zeros_like(S)
        for f in range(5):
            Vf = self.Vf[f]
            E += np.einsum("qi,eq,eqd,qj->deij", Vf, self.fw[f], self.fn[f], Vf, optimize=True)
        return self.M, S, E

    def energy(self, U):
        """E = 1/2 sum_K [ p.M p / kappa + rho sum_k u_k.M u_k ] over self.elems."""
        US = np.asarray(U, dtype=np.float64)[self.elems]
        Mu = np.einsum("eij,efj->efi", self.M, US)
        quad = np.einsum("efi,efi->ef", US, Mu)
        return 0.5 * np.sum(quad[:, 0] / self.kappa[self.elems]
                            + self.rho[self.elems] * quad[:, 1:].sum(axis=1))

    def energy_rate(self, U, dU):
        """dE/dt along dU (same inner product as ``energy``)."""
        U = np.asarray(U, dtype=np.float64)[self.elems]
        Mu = np.einsum("eij,efj->efi", self.M, dU)
        quad = np.einsum("efi,efi->ef", U, Mu)
        return np.sum(quad[:, 0] / self.kappa[self.elems]
                      + self.rho[self.elems] * quad[:, 1:].sum(axis=1))

    def penalty_dissipation(self, U):
        """-1/4 sum over element faces of w sJ (tau_p [[p]]^2 + tau_u (n.[[u]])^2).

        Each interior face is visited once from each side.  With the
        arithmetic in ``rhs`` this equals ``energy_rate(U, rhs(U))`` when the
        discrete operators satisfy summation by parts.
        """
        U = np.asarray(U, dtype=np.float64)
        UA = U[self.active]
        TA = self.traces(UA)
        S = self.elems
        _, _, zS = self._material(S)
        total = 0.0
        for f in range(5):
            Tm = TA[f][self._sidx]
            n = self.fn[f]
            Tp = np.empty_like(Tm)
            zP = zS.copy()
            inner = self.nb_row[f] >= 0
            rows = np.where(inner)[0]
            for f2 in range(5):
                sel = self.nb_f[f][rows] == f2
                if not np.any(sel):
                    continue
                r2 = rows[sel]
                src = TA[f2][self.nb_row[f][r2]]
                Tp[r2] = np.take_along_axis(src, self.nb_perm[f][r2][:, None, :], axis=2)
            if rows.size:
                zP[rows] = self._material(self.active[self.nb_row[f][rows]])[2]
            bnd = ~inner
            if np.any(bnd):
                um = Tm[bnd, 1:4]
                nb = n[bnd]
                un = np.einsum("mdq,mqd->mq", um, nb)
                if self.bc == "wall":
                    Tp[bnd, 0] = Tm[bnd, 0]
                    Tp[bnd, 1:4] = um - 2.0 * un[:, None, :] * np.transpose(nb, (0, 2, 1))
                else:
                    Tp[bnd, 0] = -Tm[bnd, 0]
                    Tp[bnd, 1:4] = um
            zavg = 0.5 * (zS + zP)
            jp = Tp[:, 0] - Tm[:, 0]
            jun = np.einsum("edq,eqd->eq", Tp[:, 1:4] - Tm[:, 1:4], n)
            total += np.sum(self.fw[f] * ((self.alpha / zavg)[:, None] * jp ** 2
                                          + (self.alpha * zavg)[:, None] * jun ** 2))
        return -0.25 * total

    # ------------------------------------------------------------------------
    def project(self, func, xyz, e2v, t=0.0, extra=3):
        """L2 projection of func(x, t) -> (npts, 4) onto the space, per element.

        Uses a collapsed rule with N + extra points per direction.  Returns
        (len(elems), 4, Np).
        """
        S = self.elems
        vr = volume_rule(self.N, self.N + extra)
        verts = np.asarray(xyz, dtype=np.float64)[np.asarray(e2v)[S]]
        X = map_points(verts, vr["r"], vr["s"], vr["t"])
        J = np.linalg.det(jacobian_matrix(verts, vr["r"], vr["s"], vr["t"]))
        V = eval_basis_rst(self.N, vr["r"], vr["s"], vr["t"])
        F = func(X.reshape(-1, 3), t).reshape(S.size, -1, 4)
        b = np.einsum("qi,eq,eqf->efi", V, vr["w"][None, :] * J, F)
        return np.einsum("eij,efj->efi", self.Minv, b)

    def l2_error(self, U, func, xyz, e2v, t=0.0, extra=4):
        """sqrt( sum_K int_K |U_h - func|^2 ) over all four fields."""
        S = self.elems
        vr = volume_rule(self.N, self.N + extra)
        verts = np.asarray(xyz, dtype=np.float64)[np.asarray(e2v)[S]]
        X = map_points(verts, vr["r"], vr["s"], vr["t"])
        J = np.linalg.det(jacobian_matrix(verts, vr["r"], vr["s"], vr["t"]))
        V = eval_basis_rst(self.N, vr["r"], vr["s"], vr["t"])
        F = func(X.reshape(-1, 3), t).reshape(S.size, -1, 4)
        Uh = np.einsum("qi,efi->eqf", V, np.asarray(U, dtype=np.float64)[S])
        return float(np.sqrt(np.sum(vr["w"][None, :, None] * J[..., None] * (Uh - F) ** 2)))

    def inverse_length(self):
        """|dK| / |K| per element of self.elems (surface area over volume)."""
        vol = self._wJ.sum(axis=1)
        area = sum(w.sum(axis=1) for w in self.fw)
        return area / vol


def wall_mode(m: int = 1):
    """Standing wave in the unit cube with rigid walls (rho = kappa = 1).

    p = cos(m pi x) cos(m pi y) cos(m pi z) cos(sqrt(3) m pi t),
    u = sin(sqrt(3) m pi t)/sqrt(3) * (sin cos cos, cos sin cos, cos cos sin)
    (arguments m pi x, m pi y, m pi z).  It solves p_t + div u = 0,
    u_t + grad p = 0 with n.u = 0 on the faces of [0, 1]^3.
    """
    k = m * np.pi
    om = np.sqrt(3.0) * k

    def f(X, t):
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        cx, cy, cz = np.cos(k * x), np.cos(k * y), np.cos(k * z)
        sx, sy, sz = np.sin(k * x), np.sin(k * y), np.sin(k * z)
        out = np.empty((X.shape[0], 4))
        out[:, 0] = cx * cy * cz * np.cos(om * t)
        amp = np.sin(om * t) / np.sqrt(3.0)
        out[:, 1] = amp * sx * cy * cz
        out[:, 2] = amp * cx * sy * cz
        out[:, 3] = amp * cx * cy * sz
        return out

    return f
