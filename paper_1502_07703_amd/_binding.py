"""ctypes binding of libdgpyr.so (argument marshalling only).

Every computation runs in the library's HIP kernels; PyTorch provides device
memory and the current stream.  There is no CPU fallback: if the library is
missing the import of ``lib()`` raises.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint32, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdgpyr.so")

OK, E_ARG, E_ORDER, E_MESH, E_NONCONFORMING, E_HIP, E_OOM, E_STATE, E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
BC = {"wall": 0, "free": 1}
PRECISION = {"fp64": 0, "fp32_mfma": 1, "split_bf16": 2}
FLAG_REFERENCE_KERNELS = 1
FLAG_UNFUSED = 2
FLAG_SUM_FACTORIZED = 4
FLAG_ADJOINT = 8
FLAG_WATCHDOG = 16
MAX_RESERVED_RECEIVERS = 4096
NOALLOC_SCRATCH_BYTES = 64 << 20

# Symbols the header declares; tests check that the library exports them all.
EXPORTS = (
    "dgpyr_setup", "dgpyr_get_info", "dgpyr_stable_dt", "dgpyr_pack", "dgpyr_unpack", "dgpyr_rhs",
    "dgpyr_step", "dgpyr_step_timed", "dgpyr_watchdog", "dgpyr_adjoint_rhs", "dgpyr_adjoint_rhs_noalloc",
    "dgpyr_set_kappa",
    "dgpyr_set_receivers", "dgpyr_receivers_sample", "dgpyr_receivers_inject",
    "dgpyr_adjoint_step", "dgpyr_set_operator_staging", "dgpyr_set_trace_groups", "dgpyr_set_groups", "dgpyr_kernel_names", "dgpyr_host_reference",
    "dgpyr_host_mesh", "dgpyr_host_sources", "dgpyr_volume_points", "dgpyr_project", "dgpyr_eval",
    "dgpyr_destroy", "dgpyr_status_string", "dgpyr_last_error",
    "dgpyr_batch_setup", "dgpyr_batch_info", "dgpyr_batch_problem", "dgpyr_batch_group",
    "dgpyr_batch_step", "dgpyr_batch_tune", "dgpyr_batch_destroy",
    "dgpyr_advection_setup", "dgpyr_host_advection_mesh",
)


class Mesh(ctypes.Structure):
    _fields_ = [
        ("nverts", c_int64),
        ("xyz", POINTER(c_double)),
        ("nelems", c_int64),
        ("e2v", POINTER(c_int64)),
        ("rho", POINTER(c_double)),
        ("kappa", POINTER(c_double)),
        ("bc", c_int32),
        ("nsources", c_int32),
        ("sources", POINTER(c_double)),
    ]


class BatchSlot(ctypes.Structure):
    _fields_ = [
        ("group", c_int32), ("N", c_int32), ("Np", c_int32), ("reserved", c_int32),
        ("nelems", c_int64), ("elem_offset", c_int64), ("offset", c_int64), ("len", c_int64),
        ("dt", c_double), ("inv_length_max", c_double),
    ]


class Opts(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("alpha", c_double), ("flags", c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [
        ("N", c_int32), ("Np", c_int32), ("Nc", c_int32), ("Nfc", c_int32),
        ("nelems", c_int64), ("state_len", c_int64), ("canon_len", c_int64),
        ("inv_length_max", c_double), ("hex_groups", c_int32), ("precision", c_int32),
        ("device_bytes", c_int64), ("groups_per_wave", c_int32), ("nfields", c_int32),
    ]


class AdvectionMesh(ctypes.Structure):
    _fields_ = [
        ("nverts", c_int64),
        ("xyz", POINTER(c_double)),
        ("nelems", c_int64),
        ("e2v", POINTER(c_int64)),
        ("pair_ids", POINTER(c_int64)),
    ]


class AdvectionOpts(ctypes.Structure):
    _fields_ = [("beta", c_double * 3), ("alpha", c_double), ("precision", c_int32),
                ("flags", c_uint32)]


class DgpyrError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    """Load libdgpyr.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} not found: build it with `python -m paper_1502_07703_amd.build` "
            "(the HIP library is required; there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    L.dgpyr_setup.argtypes = [POINTER(Mesh), c_int32, POINTER(Opts), c_void_p, POINTER(c_void_p)]
    L.dgpyr_setup.restype = c_int32
    L.dgpyr_advection_setup.argtypes = [POINTER(AdvectionMesh), c_int32, POINTER(AdvectionOpts),
                                        c_void_p, POINTER(c_void_p)]
    L.dgpyr_advection_setup.restype = c_int32
    L.dgpyr_host_advection_mesh.argtypes = [POINTER(AdvectionMesh), c_int32, POINTER(c_int32),
                                            POINTER(c_int32)]
    L.dgpyr_host_advection_mesh.restype = c_int32
    L.dgpyr_get_info.argtypes = [c_void_p, POINTER(Info)]
    L.dgpyr_get_info.restype = c_int32
    L.dgpyr_stable_dt.argtypes = [c_void_p, c_double, POINTER(c_double)]
    L.dgpyr_stable_dt.restype = c_int32
    for name in ("dgpyr_pack", "dgpyr_unpack"):
        getattr(L, name).argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        getattr(L, name).restype = c_int32
    L.dgpyr_rhs.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_void_p]
    L.dgpyr_rhs.restype = c_int32
    L.dgpyr_step.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_double, c_int32, c_void_p]
    L.dgpyr_step.restype = c_int32
    L.dgpyr_step_timed.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_double, c_int32,
                                   c_void_p, c_int32, POINTER(c_double), POINTER(c_int64)]
    L.dgpyr_step_timed.restype = c_int32
    L.dgpyr_adjoint_rhs.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    L.dgpyr_adjoint_rhs.restype = c_int32
    L.dgpyr_adjoint_rhs_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    L.dgpyr_adjoint_rhs_noalloc.restype = c_int32
    L.dgpyr_set_kappa.argtypes = [c_void_p, POINTER(c_double)]
    L.dgpyr_set_kappa.restype = c_int32
    L.dgpyr_set_receivers.argtypes = [c_void_p, c_int32, POINTER(c_double)]
    L.dgpyr_set_receivers.restype = c_int32
    for name in ("dgpyr_receivers_sample", "dgpyr_receivers_inject"):
        getattr(L, name).argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        getattr(L, name).restype = c_int32
    L.dgpyr_adjoint_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double,
                                     c_void_p]
    L.dgpyr_adjoint_step.restype = c_int32
    L.dgpyr_set_trace_groups.argtypes = [c_void_p, c_int32]
    L.dgpyr_set_trace_groups.restype = c_int32
    L.dgpyr_set_operator_staging.argtypes = [c_void_p, c_int32]
    L.dgpyr_set_operator_staging.restype = c_int32
    L.dgpyr_set_groups.argtypes = [c_void_p, c_int32]
    L.dgpyr_set_groups.restype = c_int32
    L.dgpyr_watchdog.argtypes = [c_void_p, POINTER(c_int64), c_void_p]
    L.dgpyr_watchdog.restype = c_int32
    L.dgpyr_kernel_names.argtypes = [c_void_p]
    L.dgpyr_kernel_names.restype = c_char_p
    L.dgpyr_host_reference.argtypes = [c_int32, c_int32, POINTER(c_double), c_int64, POINTER(c_int64)]
    L.dgpyr_host_reference.restype = c_int32
    L.dgpyr_host_mesh.argtypes = [POINTER(Mesh), c_int32, POINTER(c_int32), POINTER(c_double),
                                  POINTER(c_int32)]
    L.dgpyr_host_mesh.restype = c_int32
    L.dgpyr_host_sources.argtypes = [POINTER(Mesh), c_int32, POINTER(c_int64), POINTER(c_double)]
    L.dgpyr_host_sources.restype = c_int32
    for name in ("dgpyr_volume_points", "dgpyr_project", "dgpyr_eval"):
        getattr(L, name).argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        getattr(L, name).restype = c_int32
    L.dgpyr_destroy.argtypes = [c_void_p]
    L.dgpyr_destroy.restype = None
    L.dgpyr_batch_setup.argtypes = [POINTER(Mesh), POINTER(c_int32), POINTER(c_double), c_double,
                                    c_int32, POINTER(Opts), POINTER(c_void_p)]
    L.dgpyr_batch_setup.restype = c_int32
    L.dgpyr_batch_info.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int32)]
    L.dgpyr_batch_info.restype = c_int32
    L.dgpyr_batch_problem.argtypes = [c_void_p, c_int32, POINTER(BatchSlot)]
    L.dgpyr_batch_problem.restype = c_int32
    L.dgpyr_batch_group.argtypes = [c_void_p, c_int32, POINTER(c_void_p), POINTER(c_int64)]
    L.dgpyr_batch_group.restype = c_int32
    L.dgpyr_batch_step.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_void_p]
    L.dgpyr_batch_step.restype = c_int32
    L.dgpyr_batch_tune.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                   POINTER(c_int32)]
    L.dgpyr_batch_tune.restype = c_int32
    L.dgpyr_batch_destroy.argtypes = [c_void_p]
    L.dgpyr_batch_destroy.restype = None
    L.dgpyr_status_string.argtypes = [c_int32]
    L.dgpyr_status_string.restype = c_char_p
    L.dgpyr_last_error.argtypes = []
    L.dgpyr_last_error.restype = c_char_p
    _lib = L
    return L


def check(status: int, where: str):
    if status != OK:
        L = lib()
        detail = (L.dgpyr_last_error() or b"").decode(errors="replace")
        kind = (L.dgpyr_status_string(status) or b"").decode(errors="replace")
        raise DgpyrError(status, where, f"{kind}: {detail}")
