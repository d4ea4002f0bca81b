"""dgpyr: DG acoustics on vertex-mapped pyramids for MI355X (gfx950).

Python face of libdgpyr.so.  ``Solver`` marshals a pyramid mesh into
``dgpyr_setup`` and calls ``dgpyr_rhs`` / ``dgpyr_step`` on torch device
tensors and the current torch stream; all arithmetic runs in the library's
HIP kernels.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _binding as B
from ._binding import DgpyrError

__all__ = ["Solver", "Advection", "Batch", "DgpyrError", "n_basis", "LSRK_CFL_CONSTANT"]


def n_basis(N: int) -> int:
    return (N + 1) * (N + 2) * (2 * N + 3) // 6


def LSRK_CFL_CONSTANT(N: int) -> float:
    """2(N+1)(N+3)/3, the constant the spectral radius tracks (Section 4.3)."""
    return 2.0 * (N + 1) * (N + 3) / 3.0


def _to_numpy(x):
    if hasattr(x, "detach"):
        return x.detach().cpu().numpy()
    return np.asarray(x)


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t, length=None, name="array"):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if length is not None and t.numel() != length:
        raise ValueError(f"{name} has {t.numel()} elements, expected {length}")
    return ctypes.c_void_p(t.data_ptr())


def _sources_array(sources):
    """Point sources as an (n, 6) float64 array: x, y, z, amplitude, f0, delay.
    Accepts such an array or a list of dicts with keys x (3), f0, and optional
    amp (1) and t0 (delay; <= 0 or missing means 1/f0)."""
    if sources is None or len(sources) == 0:
        return None
    if isinstance(sources, np.ndarray):
        a = np.ascontiguousarray(sources, dtype=np.float64)
    else:
        a = np.array([[*s["x"], s.get("amp", 1.0), s["f0"], s.get("t0") or 0.0] for s in sources],
                     dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 6:
        raise ValueError("sources must have shape (n, 6)")
    return a


class _HostMesh:
    """Host arrays of one mesh kept alive while the library reads them."""

    def __init__(self, xyz, e2v, rho=None, kappa=None, bc="wall", sources=None):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.e2v = np.ascontiguousarray(e2v, dtype=np.int64)
        if self.xyz.ndim != 2 or self.xyz.shape[1] != 3:
            raise ValueError("xyz must have shape (nverts, 3)")
        if self.e2v.ndim != 2 or self.e2v.shape[1] != 5:
            raise ValueError("e2v must have shape (nelems, 5)")
        K = self.e2v.shape[0]
        self.rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        self.kappa = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
        for a, nm in ((self.rho, "rho"), (self.kappa, "kappa")):
            if a is not None and a.shape != (K,):
                raise ValueError(f"{nm} must have shape ({K},)")
        self.src = _sources_array(sources)
        dptr = ctypes.POINTER(ctypes.c_double)
        self.struct = B.Mesh(
            nverts=self.xyz.shape[0], xyz=self.xyz.ctypes.data_as(dptr),
            nelems=K, e2v=self.e2v.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            rho=None if self.rho is None else self.rho.ctypes.data_as(dptr),
            kappa=None if self.kappa is None else self.kappa.ctypes.data_as(dptr),
            bc=B.BC[bc], nsources=0 if self.src is None else self.src.shape[0],
            sources=None if self.src is None else self.src.ctypes.data_as(dptr))


def _opts(precision, alpha, reference_kernels=False, unfused=False, sum_factorized=False,
          adjoint=False, watchdog=False):
    flags = (B.FLAG_REFERENCE_KERNELS if reference_kernels else 0) | \
        (B.FLAG_UNFUSED if unfused else 0) | \
        (B.FLAG_SUM_FACTORIZED if sum_factorized else 0) | \
        (B.FLAG_ADJOINT if adjoint else 0) | \
        (B.FLAG_WATCHDOG if watchdog else 0)
    return B.Opts(precision=B.PRECISION[precision], alpha=float(alpha), flags=flags)


class Solver:
    """A mesh and a discretisation set up on the current HIP device."""

    def __init__(self, xyz, e2v, N, rho=None, kappa=None, bc="wall", alpha=1.0,
                 precision="fp64", reference_kernels=False, unfused=False,
                 sum_factorized=False, groups_per_wave=0, sources=None, lds_operators=None,
                 trace_groups=0, adjoint=False, watchdog=False, stream=None):
        L = B.lib()
        self._host = _HostMesh(xyz, e2v, rho, kappa, bc, sources)
        mesh = self._host.struct
        opts = _opts(precision, alpha, reference_kernels, unfused, sum_factorized, adjoint,
                     watchdog)
        handle = ctypes.c_void_p()
        st = L.dgpyr_setup(ctypes.byref(mesh), int(N), ctypes.byref(opts),
                           _stream_handle(stream) if stream is not None else None,
                           ctypes.byref(handle))
        B.check(st, "dgpyr_setup")
        self._h = handle
        info = B.Info()
        B.check(L.dgpyr_get_info(self._h, ctypes.byref(info)), "dgpyr_get_info")
        self._set_info(info)
        if groups_per_wave:
            self.set_groups(groups_per_wave)
        if lds_operators is not None:
            self.set_operator_staging(lds_operators)
        if trace_groups:
            self.set_trace_groups(trace_groups)

    def _set_info(self, info):
        self.info = {k: getattr(info, k) for k, _ in B.Info._fields_}
        self.N, self.Np, self.K = info.N, info.Np, info.nelems
        self.nfields = info.nfields
        self.state_len, self.canon_len = info.state_len, info.canon_len

    def set_trace_groups(self, groups: int):
        """Element groups per wave of the trace kernel (0 = default)."""
        B.check(B.lib().dgpyr_set_trace_groups(self._h, int(groups)), "dgpyr_set_trace_groups")

    def set_operator_staging(self, enable: bool):
        """Stage operator tiles in LDS per workgroup in the fused stage kernel."""
        B.check(B.lib().dgpyr_set_operator_staging(self._h, 1 if enable else 0),
                "dgpyr_set_operator_staging")

    # -- state helpers -----------------------------------------------------------
    def empty_state(self):
        import torch
        return torch.empty(self.state_len, dtype=torch.float64, device="cuda")

    def pack(self, canon, out=None, stream=None):
        """Canonical (K, nfields, Np) device tensor -> state array."""
        out = self.empty_state() if out is None else out
        B.check(B.lib().dgpyr_pack(self._h, _dptr(canon, self.canon_len, "canon"),
                                   _dptr(out, self.state_len, "U"), _stream_handle(stream)),
                "dgpyr_pack")
        return out

    def unpack(self, U, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.K, self.nfields, self.Np), dtype=torch.float64, device="cuda")
        B.check(B.lib().dgpyr_unpack(self._h, _dptr(U, self.state_len, "U"),
                                     _dptr(out, self.canon_len, "canon"), _stream_handle(stream)),
                "dgpyr_unpack")
        return out

    # -- the hot path ---------------------------------------------------------------
    def rhs(self, U, out=None, t=0.0, stream=None):
        out = self.empty_state() if out is None else out
        B.check(B.lib().dgpyr_rhs(self._h, _dptr(U, self.state_len, "U"),
                                  _dptr(out, self.state_len, "dUdt"), float(t),
                                  _stream_handle(stream)), "dgpyr_rhs")
        return out

    def adjoint_rhs(self, lam, out=None, stream=None):
        """A^T lam: the transpose of the operator rhs() applies (no sources)."""
        out = self.empty_state() if out is None else out
        B.check(B.lib().dgpyr_adjoint_rhs(self._h, _dptr(lam, self.state_len, "lam"),
                                          _dptr(out, self.state_len, "out"),
                                          _stream_handle(stream)), "dgpyr_adjoint_rhs")
        return out

    # -- discrete adjoint ---------------------------------------------------------
    def set_kappa(self, kappa):
        """New per-element bulk modulus (host or device array of nelems values)."""
        k = np.ascontiguousarray(_to_numpy(kappa), dtype=np.float64)
        if k.shape != (self.K,):
            raise ValueError(f"kappa must have shape ({self.K},)")
        B.check(B.lib().dgpyr_set_kappa(self._h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                "dgpyr_set_kappa")
        info = B.Info()
        B.check(B.lib().dgpyr_get_info(self._h, ctypes.byref(info)), "dgpyr_get_info")
        self._set_info(info)

    def set_receivers(self, points):
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        B.check(B.lib().dgpyr_set_receivers(self._h, pts.shape[0],
                                            pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                "dgpyr_set_receivers")
        self.nrec = pts.shape[0]

    def sample_receivers(self, U, out, stream=None):
        B.check(B.lib().dgpyr_receivers_sample(self._h, _dptr(U, self.state_len, "U"),
                                               _dptr(out, self.nrec, "out"),
                                               _stream_handle(stream)), "dgpyr_receivers_sample")
        return out

    def inject_receivers(self, Ubar, coef, stream=None):
        B.check(B.lib().dgpyr_receivers_inject(self._h, _dptr(Ubar, self.state_len, "Ubar"),
                                               _dptr(coef, self.nrec, "coef"),
                                               _stream_handle(stream)), "dgpyr_receivers_inject")
        return Ubar

    def adjoint_step(self, U0, Ubar, grad, t0, dt, stream=None):
        B.check(B.lib().dgpyr_adjoint_step(self._h, _dptr(U0, self.state_len, "U0"),
                                           _dptr(Ubar, self.state_len, "Ubar"),
                                           _dptr(grad, self.K, "grad"), float(t0), float(dt),
                                           _stream_handle(stream)), "dgpyr_adjoint_step")
        return Ubar, grad

    def step(self, U, R, dt, nsteps=1, t0=0.0, stream=None):
        B.check(B.lib().dgpyr_step(self._h, _dptr(U, self.state_len, "U"),
                                   _dptr(R, self.state_len, "R"), float(t0), float(dt),
                                   int(nsteps), _stream_handle(stream)), "dgpyr_step")
        return U, R

    def watchdog(self, stream=None):
        """NaN/Inf watchdog (Solver(..., watchdog=True)): -1 if every state
        checked since the previous call was finite, else the 0-based index of
        the first step, counted over the step calls since then, after which the
        state held a non-finite entry.  Synchronises the stream."""
        v = ctypes.c_int64()
        B.check(B.lib().dgpyr_watchdog(self._h, ctypes.byref(v), _stream_handle(stream)),
                "dgpyr_watchdog")
        return v.value

    # -- initial data and errors ------------------------------------------------------
    def volume_points(self, stream=None):
        """Physical cubature points (K, Nc, 3) and weights w J (K, Nc)."""
        import torch
        Nc = self.info["Nc"]
        xyz = torch.empty((self.K, Nc, 3), dtype=torch.float64, device="cuda")
        wJ = torch.empty((self.K, Nc), dtype=torch.float64, device="cuda")
        B.check(B.lib().dgpyr_volume_points(self._h, _dptr(xyz), _dptr(wJ), _stream_handle(stream)),
                "dgpyr_volume_points")
        return xyz, wJ

    def project(self, f, out=None, stream=None):
        """L2 projection of values f (K, nfields, Nc) at the cubature points -> state."""
        out = self.empty_state() if out is None else out
        B.check(B.lib().dgpyr_project(self._h, _dptr(f, self.K * self.nfields * self.info["Nc"], "f"),
                                      _dptr(out, self.state_len, "U"), _stream_handle(stream)),
                "dgpyr_project")
        return out

    def evaluate(self, U, out=None, stream=None):
        """Values (K, nfields, Nc) of state U at the cubature points."""
        import torch
        if out is None:
            out = torch.empty((self.K, self.nfields, self.info["Nc"]), dtype=torch.float64,
                              device="cuda")
        B.check(B.lib().dgpyr_eval(self._h, _dptr(U, self.state_len, "U"),
                                   _dptr(out, self.K * self.nfields * self.info["Nc"], "f"),
                                   _stream_handle(stream)), "dgpyr_eval")
        return out

    def set_groups(self, groups_per_wave: int):
        """Element groups per wave of the fused matrix-core kernels (0 = default)."""
        B.check(B.lib().dgpyr_set_groups(self._h, int(groups_per_wave)), "dgpyr_set_groups")

    def info_groups(self) -> int:
        """Element groups per wave currently in effect."""
        info = B.Info()
        B.check(B.lib().dgpyr_get_info(self._h, ctypes.byref(info)), "dgpyr_get_info")
        return int(info.groups_per_wave)

    def stable_dt(self, cfl=0.5):
        """CFL / (2(N+1)(N+3)/3 * max_K c_K |dK|/|K|) (Section 4.3 scaling), for
        the current material, as computed by ``dgpyr_stable_dt``."""
        dt = ctypes.c_double()
        B.check(B.lib().dgpyr_stable_dt(self._h, float(cfl), ctypes.byref(dt)), "dgpyr_stable_dt")
        return dt.value

    def close(self):
        if getattr(self, "_h", None):
            B.lib().dgpyr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class _GroupView(Solver):
    """Solver methods on one group context of a batch (not owned)."""

    def __init__(self, handle):  # noqa: D107  (no mesh: the batch built it)
        L = B.lib()
        self._h = handle
        info = B.Info()
        B.check(L.dgpyr_get_info(self._h, ctypes.byref(info)), "dgpyr_get_info")
        self._set_info(info)

    def close(self):
        self._h = None


class Advection(Solver):
    """Linear advection u_t + div(beta u) = 0 (Section 4.1) on a pyramid mesh:
    one field per element, state (K, 1, Np).  ``pair_ids`` ([nverts], optional)
    pair faces through vertex identities (periodic meshes); alpha = 1 upwind,
    0 central.  Serves rhs, step, project, evaluate, volume_points, stable_dt
    (CFL against |beta| max |dK| / |K|)."""

    def __init__(self, xyz, e2v, N, beta, alpha=1.0, pair_ids=None, precision="fp64",
                 stream=None):  # noqa: D107
        L = B.lib()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self._e2v = np.ascontiguousarray(e2v, dtype=np.int64)
        if self._xyz.ndim != 2 or self._xyz.shape[1] != 3:
            raise ValueError("xyz must have shape (nverts, 3)")
        if self._e2v.ndim != 2 or self._e2v.shape[1] != 5:
            raise ValueError("e2v must have shape (nelems, 5)")
        self._pid = None
        if pair_ids is not None:
            self._pid = np.ascontiguousarray(pair_ids, dtype=np.int64)
            if self._pid.shape != (self._xyz.shape[0],):
                raise ValueError("pair_ids must have shape (nverts,)")
        i64 = ctypes.POINTER(ctypes.c_int64)
        mesh = B.AdvectionMesh(
            nverts=self._xyz.shape[0],
            xyz=self._xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            nelems=self._e2v.shape[0], e2v=self._e2v.ctypes.data_as(i64),
            pair_ids=None if self._pid is None else self._pid.ctypes.data_as(i64))
        b = [float(x) for x in beta]
        if len(b) != 3:
            raise ValueError("beta must have 3 components")
        opts = B.AdvectionOpts(beta=(ctypes.c_double * 3)(*b), alpha=float(alpha),
                               precision=B.PRECISION[precision], flags=0)
        handle = ctypes.c_void_p()
        st = L.dgpyr_advection_setup(ctypes.byref(mesh), int(N), ctypes.byref(opts),
                                     _stream_handle(stream) if stream is not None else None,
                                     ctypes.byref(handle))
        B.check(st, "dgpyr_advection_setup")
        self._h = handle
        info = B.Info()
        B.check(L.dgpyr_get_info(self._h, ctypes.byref(info)), "dgpyr_get_info")
        self._set_info(info)
        self.beta = np.array(b)


class Batch:
    """Independent problems of uneven sizes and orders advanced together.

    ``problems``: list of dicts with keys ``xyz``, ``e2v``, ``N`` and optional
    ``rho``, ``kappa``, ``bc``, ``sources``.  Each problem has its own time
    step (``dts`` or the CFL rule).  The batch state is one device array;
    ``view(U, i)`` is problem i's (nelems, 4, Np) part.
    """

    def __init__(self, problems, precision="fp64", alpha=1.0, dts=None, cfl=0.5):
        L = B.lib()
        self._hosts = [_HostMesh(p["xyz"], p["e2v"], p.get("rho"), p.get("kappa"),
                                 p.get("bc", "wall"), p.get("sources")) for p in problems]
        n = len(problems)
        meshes = (B.Mesh * n)(*[h.struct for h in self._hosts])
        orders = (ctypes.c_int32 * n)(*[int(p["N"]) for p in problems])
        dts_arr = None if dts is None else (ctypes.c_double * n)(*[float(x) for x in dts])
        opts = _opts(precision, alpha)
        h = ctypes.c_void_p()
        B.check(L.dgpyr_batch_setup(meshes, orders, dts_arr, float(cfl), n, ctypes.byref(opts),
                                    ctypes.byref(h)), "dgpyr_batch_setup")
        self._h = h
        sl, ng = ctypes.c_int64(), ctypes.c_int32()
        B.check(L.dgpyr_batch_info(h, ctypes.byref(sl), ctypes.byref(ng)), "dgpyr_batch_info")
        self.state_len, self.ngroups = sl.value, ng.value
        self.slots = []
        for i in range(n):
            s = B.BatchSlot()
            B.check(L.dgpyr_batch_problem(h, i, ctypes.byref(s)), "dgpyr_batch_problem")
            self.slots.append({k: getattr(s, k) for k, _ in B.BatchSlot._fields_ if k != "reserved"})
        self.groups = []
        for g in range(self.ngroups):
            c, off = ctypes.c_void_p(), ctypes.c_int64()
            B.check(L.dgpyr_batch_group(h, g, ctypes.byref(c), ctypes.byref(off)),
                    "dgpyr_batch_group")
            self.groups.append((_GroupView(c), off.value))

    def empty_state(self):
        import torch
        return torch.empty(self.state_len, dtype=torch.float64, device="cuda")

    def view(self, U, i):
        """Problem i's part of a batch state array, shape (nelems, 4, Np)."""
        s = self.slots[i]
        return U[s["offset"]:s["offset"] + s["len"]].view(s["nelems"], 4, s["Np"])

    def group_state(self, U, g):
        """Group g's part of a batch state array (flat)."""
        view, off = self.groups[g]
        return U[off:off + view.state_len]

    def step(self, U, R, nsteps=1, step0=0, stream=None):
        B.check(B.lib().dgpyr_batch_step(self._h, _dptr(U, self.state_len, "U"),
                                         _dptr(R, self.state_len, "R"), int(step0), int(nsteps),
                                         _stream_handle(stream)), "dgpyr_batch_step")
        return U, R

    def tune(self, nsteps=2, stream=None):
        """Autotune the work shape of every group; returns the choice per group.
        Two batch-sized scratch arrays are allocated here (torch) and handed to
        the library, which allocates nothing itself."""
        import torch
        U = torch.empty(self.state_len, dtype=torch.float64, device="cuda")
        R = torch.empty_like(U)
        out = (ctypes.c_int32 * self.ngroups)()
        B.check(B.lib().dgpyr_batch_tune(self._h, _dptr(U), _dptr(R), int(nsteps),
                                         _stream_handle(stream), out), "dgpyr_batch_tune")
        del U, R
        return list(out)

    def close(self):
        if getattr(self, "_h", None):
            for view, _ in getattr(self, "groups", []):
                view.close()
            B.lib().dgpyr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
