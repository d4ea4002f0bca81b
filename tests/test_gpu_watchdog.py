"""NaN/Inf watchdog of the step calls (DGPYR_FLAG_WATCHDOG): silent on a
stable run and without effect on its results, names the first step after which
the state held a non-finite entry (planted, or reached by steps far beyond the
CFL rule of Section 4.3), and starts a new count after each query."""

import numpy as np
import pytest

from gpu_helpers import log
from synth import hex_pyramid_mesh, random_state

pytestmark = pytest.mark.gpu

N = 3


def _setup(sum_factorized):
    import torch

    import paper_1502_07703_amd as dg
    xyz, e2v = hex_pyramid_mesh(3, seed=1)
    U0 = torch.from_numpy(random_state(e2v.shape[0], N, seed=5)).cuda()
    return dg, xyz, e2v, U0


@pytest.mark.parametrize("sum_factorized", [False, True])
def test_watchdog_silent_and_transparent(sum_factorized):
    import torch
    dg, xyz, e2v, U0 = _setup(sum_factorized)
    log(f"[watchdog] stable run sum_factorized={sum_factorized}")
    with dg.Solver(xyz, e2v, N, sum_factorized=sum_factorized, watchdog=True) as s, \
            dg.Solver(xyz, e2v, N, sum_factorized=sum_factorized) as r:
        dt = s.stable_dt(0.5)
        U, U2 = s.pack(U0), r.pack(U0)
        R, R2 = torch.zeros_like(U), torch.zeros_like(U2)
        s.step(U, R, dt, nsteps=6)
        r.step(U2, R2, dt, nsteps=6)
        assert s.watchdog() == -1
        assert torch.equal(U, U2) and torch.equal(R, R2)
        s.step(U, R, dt, nsteps=2)
        assert s.watchdog() == -1


@pytest.mark.parametrize("where,value", [(0, float("nan")), (-1, float("inf")),
                                         ("mid", float("-inf"))])
def test_watchdog_planted(where, value):
    import torch
    dg, xyz, e2v, U0 = _setup(False)
    with dg.Solver(xyz, e2v, N, watchdog=True) as s:
        dt = s.stable_dt(0.5)
        flat_len = s.state_len
        pos = flat_len // 2 + 7 if where == "mid" else where
        log(f"[watchdog] planted {value} at {pos} of {flat_len}")
        U = s.pack(U0)
        R = torch.zeros_like(U)
        U.view(-1)[pos] = value
        s.step(U, R, dt, nsteps=3)
        assert s.watchdog() == 0
        # a new count: two clean steps, then a planted value before the third
        U = s.pack(U0)
        R.zero_()
        s.step(U, R, dt, nsteps=2)
        U.view(-1)[pos] = value
        s.step(U, R, dt, nsteps=2)
        assert s.watchdog() == 2
        assert s.watchdog() == -1  # nothing stepped since the last query


@pytest.mark.parametrize("sum_factorized", [False, True])
def test_watchdog_finds_the_first_overflowing_step(sum_factorized):
    """Steps 100x the CFL step grow the state until it overflows; the step
    found by checking the state on the host after every step must be the one
    the watchdog reports for the same steps taken in one call."""
    import torch
    dg, xyz, e2v, U0 = _setup(sum_factorized)
    with dg.Solver(xyz, e2v, N, sum_factorized=sum_factorized, watchdog=True) as s, \
            dg.Solver(xyz, e2v, N, sum_factorized=sum_factorized) as r:
        dt = 100.0 * s.stable_dt(0.5)
        U, R = r.pack(U0), torch.zeros_like(r.pack(U0))
        first = None
        for n in range(400):
            r.step(U, R, dt, nsteps=1)
            if not bool(torch.isfinite(U).all()):
                first = n
                break
        log(f"[watchdog] sum_factorized={sum_factorized}: first non-finite state after step {first}")
        assert first is not None, "the state stayed finite for 400 steps"
        U, R = s.pack(U0), torch.zeros_like(s.pack(U0))
        s.step(U, R, dt, nsteps=first + 3)
        assert s.watchdog() == first
        assert not np.isfinite(U.cpu().numpy()).all()
