"""Parity on the named workload shapes, end to end.

* 48 pyramids (2^3 perturbed hexes x 6), N = 3, projected wall eigenmode,
  penalty flux: the whole LSRK(5,4) trajectory to T = 0.5 at CFL 0.5
  (Section 4.3 time-step rule) against the oracle's trajectory;
* 64^3 x 6 = 1572864 pyramids at N = 7 (the largest order of the precision
  study): the device computes every element, the oracle a seeded sample;
* the two precision forms on the 40^3 x 6 = 384000-pyramid mesh, sampled.
"""

import numpy as np
import pytest

from gpu_helpers import log, rel_err_per_field
from oracle import AcousticDG, lsrk_run
from oracle.dg import wall_mode
from synth import hex_pyramid_mesh

pytestmark = pytest.mark.gpu


def test_cfg1_trajectory_to_half():
    """Trajectory to T = 0.5: dt from the library's CFL rule (checked against
    the oracle's |dK|/|K|), n = ceil(T / dt0) steps of T / n; per field within
    1e-10 of the oracle (about 2400 stages of rounding on either side)."""
    import torch

    import paper_1502_07703_amd as dg
    N, T = 3, 0.5
    xyz, e2v = hex_pyramid_mesh(2, seed=1)
    o = AcousticDG(xyz, e2v, N)
    U0 = o.project(wall_mode(1), xyz, e2v)
    dt0_ref = 0.5 / (2.0 * (N + 1) * (N + 3) / 3.0 * o.inverse_length().max())
    with dg.Solver(xyz, e2v, N) as s:
        dt0 = s.stable_dt(0.5)
        assert abs(dt0 - dt0_ref) <= 1e-12 * dt0_ref, (dt0, dt0_ref)
        n = int(np.ceil(T / dt0))
        dt = T / n
        log(f"[configs] 48 pyramids N=3 to T=0.5: {n} steps of {dt:.6e}")
        U = s.pack(torch.from_numpy(U0).cuda())
        R = s.empty_state()
        s.step(U, R, dt, n)
        got = s.unpack(U).cpu().numpy()
    ref, _ = lsrk_run(o.rhs, U0, dt, n)
    err = rel_err_per_field(got, ref)
    e_gpu = o.l2_error(got, wall_mode(1), xyz, e2v, t=T)
    e_ref = o.l2_error(ref, wall_mode(1), xyz, e2v, t=T)
    log(f"[configs] trajectory rel err per field {err}; L2 error vs mode {e_gpu:.6e} "
        f"(oracle {e_ref:.6e})")
    assert np.all(err < 1e-10), err
    assert abs(e_gpu - e_ref) <= 1e-8 * e_ref


def _sampled_rhs(s, o, K, Np, seed):
    """Random device state, the device right-hand side on every element, and
    the oracle's on its sampled elements (only their rows and their face
    neighbours' rows are copied to the host)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    Uc = torch.randn((K, 4, Np), dtype=torch.float64, device="cuda", generator=g)
    U = s.pack(Uc)
    out = s.unpack(s.rhs(U))
    got = out[torch.from_numpy(o.elems).cuda()].cpu().numpy()
    Uh = np.zeros((K, 4, Np))
    Uh[o.active] = Uc[torch.from_numpy(o.active).cuda()].cpu().numpy()
    del Uc, U, out
    torch.cuda.synchronize()
    return got, o.rhs(Uh)


def test_cfg3_sampled_fp64_N7():
    """64^3 x 6 = 1572864 pyramids (seed 3), N = 7 (Np = 204): 2000 sampled
    elements plus the first and last, FP64 within 1e-12 per field."""
    import paper_1502_07703_amd as dg
    N, k1d = 7, 64
    xyz, e2v = hex_pyramid_mesh(k1d, seed=3)
    K = e2v.shape[0]
    rng = np.random.default_rng(31)
    sample = np.unique(np.concatenate([rng.choice(K, 2000, replace=False), [0, K - 1]]))
    o = AcousticDG(xyz, e2v, N, elems=sample)
    log(f"[configs] 64^3 x 6 K={K} N={N} sample={sample.size}")
    with dg.Solver(xyz, e2v, N) as s:
        got, ref = _sampled_rhs(s, o, K, s.Np, 32)
    err = rel_err_per_field(got, ref)
    log(f"[configs] 64^3 x 6 N=7 rel err per field {err}")
    assert np.all(err < 1e-12), err


# Right-hand-side bars of the precision forms (relative per field against the
# FP64 oracle, random data), as in test_gpu_parity.py: measured 4.5e-7 (FP32)
# and 1.04e-5 (split-BF16) at this size.
PRECISION_BARS = {"fp32_mfma": 3e-6, "split_bf16": 5e-5}


@pytest.mark.parametrize("prec", ["fp32_mfma", "split_bf16"])
def test_precision_forms_full_size_sampled(prec):
    """40^3 x 6 = 384000 pyramids (seed 2), N = 4, both precision forms: 3000
    sampled elements against the FP64 oracle at each form's bar."""
    import paper_1502_07703_amd as dg
    N, k1d = 4, 40
    xyz, e2v = hex_pyramid_mesh(k1d, seed=2)
    K = e2v.shape[0]
    rng = np.random.default_rng(12)
    sample = np.unique(np.concatenate([rng.choice(K, 3000, replace=False), [0, K - 1]]))
    o = AcousticDG(xyz, e2v, N, elems=sample)
    log(f"[configs] 40^3 x 6 {prec} K={K} N={N}")
    with dg.Solver(xyz, e2v, N, precision=prec) as s:
        got, ref = _sampled_rhs(s, o, K, s.Np, 33)
    err = rel_err_per_field(got, ref)
    log(f"[configs] 40^3 x 6 {prec} rel err per field {err}")
    assert np.all(err < PRECISION_BARS[prec]), err
    assert np.any(err > 1e-10), "reduced-precision form gave FP64-accurate results"
