"""Helpers shared by the GPU tests: run the library and compare with the oracle."""

from __future__ import annotations

import sys

import numpy as np
import pytest


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_rhs(solver, canon: np.ndarray) -> np.ndarray:
    import torch
    c = torch.from_numpy(np.ascontiguousarray(canon, dtype=np.float64)).cuda()
    U = solver.pack(c)
    out = solver.rhs(U)
    res = solver.unpack(out)
    torch.cuda.synchronize()
    return res.cpu().numpy()


def rel_err_per_field(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """max |got - ref| / max |ref| for each of the four fields.

    A field that vanishes in exact arithmetic (e.g. dp/dt of a single pyramid
    at N = 0 with walls, where the closed-surface normal sum cancels) carries
    only the oracle's roundoff; its denominator is floored at 1e-3 of the
    largest field, so such a field is held to about 1e-15 of the result's
    scale, i.e. a few ulps.
    """
    num = np.abs(got - ref).max(axis=(0, 2))
    fmax = np.abs(ref).max(axis=(0, 2))
    den = np.maximum(fmax, max(1e-3 * fmax.max(), 1e-300))
    return num / den
