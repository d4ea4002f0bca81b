"""Advection path (Section 4.1) on the device against the oracle.

* right-hand side, element by element, on a periodic 3^3 x 6 mesh (162
  pyramids: three workgroups, the last one ragged) for N = 0..8, upwind and
  central flux, and on a ragged non-periodic mesh (13 shuffled pyramids);
* LSRK steps against the oracle's LSRK;
* 40^3 x 6 periodic pyramids (the bench's launch shape): sampled elements
  against the oracle evaluated on those elements only, constants steady;
* transport of a smooth wave converging to u0(x - beta t).
"""

import numpy as np
import pytest

from gpu_helpers import log
from oracle.advection import AdvectionDG
from oracle.lsrk import lsrk_run
from synth import hex_pyramid_mesh, periodic_pair_ids

pytestmark = pytest.mark.gpu

BETA = np.array([1.0, 0.3, -0.5])
TOL = 1e-12


@pytest.fixture(scope="module")
def periodic3():
    xyz, e2v = hex_pyramid_mesh(3, seed=1, lo=-1.0, hi=1.0)
    return xyz, e2v, periodic_pair_ids(xyz)


def _dot3(P, k):
    """P (..., 3) . k (3 numbers), elementwise (no BLAS call on huge shapes)."""
    return float(k[0]) * P[..., 0] + float(k[1]) * P[..., 1] + float(k[2]) * P[..., 2]


def _gpu_rhs(s, u):
    import torch
    U = torch.from_numpy(np.ascontiguousarray(u)).cuda().reshape(-1)
    out = s.rhs(U)
    torch.cuda.synchronize()
    return out.reshape(u.shape).cpu().numpy()


def _rel(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("N", list(range(9)))
@pytest.mark.parametrize("alpha", [1.0, 0.0])
def test_adv_rhs_parity_periodic(periodic3, N, alpha):
    import paper_1502_07703_amd as dg
    xyz, e2v, pid = periodic3
    o = AdvectionDG(xyz, e2v, N, BETA, alpha=alpha, period=(-1.0, 1.0))
    u = np.random.default_rng(30 + N).standard_normal((o.K, o.Np))
    ref = o.rhs(u)
    log(f"[adv] rhs periodic N={N} alpha={alpha}")
    with dg.Advection(xyz, e2v, N, BETA, alpha=alpha, pair_ids=pid) as s:
        assert s.nfields == 1 and s.state_len == o.K * o.Np
        got = _gpu_rhs(s, u)
    err = _rel(got, ref)
    log(f"[adv] rhs periodic N={N} alpha={alpha} rel err {err:.2e}")
    assert err < TOL


@pytest.mark.parametrize("N", [0, 3, 6])
def test_adv_rhs_parity_open_ragged(N):
    import paper_1502_07703_amd as dg
    xyz, e2v = hex_pyramid_mesh(2, seed=4, shuffle=True)
    e2v = e2v[:13]
    o = AdvectionDG(xyz, e2v, N, BETA, alpha=1.0)
    u = np.random.default_rng(50 + N).standard_normal((o.K, o.Np))
    log(f"[adv] rhs open ragged N={N}")
    with dg.Advection(xyz, e2v, N, BETA, alpha=1.0) as s:
        got = _gpu_rhs(s, u)
    err = _rel(got, o.rhs(u))
    log(f"[adv] rhs open ragged N={N} rel err {err:.2e}")
    assert err < TOL


@pytest.mark.parametrize("N", [2, 4, 7, 8])
def test_adv_steps_match_oracle(periodic3, N):
    import torch

    import paper_1502_07703_amd as dg
    xyz, e2v, pid = periodic3
    o = AdvectionDG(xyz, e2v, N, BETA, alpha=1.0, period=(-1.0, 1.0))
    u0 = np.random.default_rng(70 + N).standard_normal((o.K, o.Np))
    dt, n = 0.005, 6
    ref = lsrk_run(lambda u, t: o.rhs(u), u0, dt, n)[0]
    log(f"[adv] steps N={N}")
    with dg.Advection(xyz, e2v, N, BETA, alpha=1.0, pair_ids=pid) as s:
        U = torch.from_numpy(u0.copy()).cuda().reshape(-1)
        R = s.empty_state().zero_()
        s.step(U, R, dt, n)
        got = U.reshape(u0.shape).cpu().numpy()
    err = _rel(got, ref)
    log(f"[adv] steps N={N} rel err {err:.2e}")
    assert err < 1e-11


@pytest.mark.parametrize("N", [4, 6])
def test_adv_full_size_sampled(N):
    """40^3 x 6 periodic pyramids, the bench's mesh shape."""
    import torch

    import paper_1502_07703_amd as dg
    k1d = 40
    xyz, e2v = hex_pyramid_mesh(k1d, seed=2, lo=-1.0, hi=1.0)
    pid = periodic_pair_ids(xyz)
    K = e2v.shape[0]
    sample = np.unique(np.concatenate([np.random.default_rng(9).choice(K, 200, replace=False),
                                       [0, 1, K - 1], 6 * (k1d - 1) + np.arange(6)]))
    log(f"[adv] full size N={N} K={K}")
    with dg.Advection(xyz, e2v, N, BETA, alpha=1.0, pair_ids=pid) as s:
        Np = s.Np
        g = torch.Generator(device="cuda").manual_seed(5)
        U = torch.randn(K * Np, dtype=torch.float64, device="cuda", generator=g)
        out = s.rhs(U)
        one = s.project(torch.ones((K, 1, s.info["Nc"]), dtype=torch.float64, device="cuda"))
        steady = s.rhs(one)
        torch.cuda.synchronize()
        u = U.reshape(K, Np).cpu().numpy()
        got = out.reshape(K, Np).cpu().numpy()[sample]
        st = float(steady.abs().max())
    o = AdvectionDG(xyz, e2v, N, BETA, alpha=1.0, period=(-1.0, 1.0), elems=sample)
    err = _rel(got, o.rhs(u))
    log(f"[adv] full size N={N} sampled rel err {err:.2e}, constant rhs {st:.1e}")
    assert err < TOL
    assert st < 1e-10


def test_adv_transport_converges():
    import torch

    import paper_1502_07703_amd as dg
    xyz, e2v = hex_pyramid_mesh(6, seed=3, lo=-1.0, hi=1.0)
    pid = periodic_pair_ids(xyz)
    kv = np.pi * np.array([1.0, 1.0, 0.0])
    T = 0.5
    errs = []
    for N in (2, 3, 4, 5):
        with dg.Advection(xyz, e2v, N, BETA, alpha=1.0, pair_ids=pid) as s:
            P, wJ = s.volume_points()
            U = s.project(torch.sin(_dot3(P, kv)).unsqueeze(1).contiguous())
            R = s.empty_state().zero_()
            dt0 = s.stable_dt(0.5)
            n = int(np.ceil(T / dt0))
            s.step(U, R, T / n, n)
            f = s.evaluate(U)[:, 0]
            bt = torch.from_numpy(BETA * T).cuda()
            exact = torch.sin(_dot3(P - bt, kv))
            e = float(torch.sqrt((wJ * (f - exact) ** 2).sum()))
            errs.append(e)
        log(f"[adv] transport N={N} steps={n} L2 error {e:.3e}")
    assert errs[0] < 0.05
    for a, b in zip(errs, errs[1:]):
        assert b < 0.5 * a
