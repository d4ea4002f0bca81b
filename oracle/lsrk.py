"""Low-storage RK(5,4) of Carpenter and Kennedy (Section 4.1, Algorithm 3).

Each of the five stages does
    R <- A_s R + dt * rhs(U, t + c_s dt),      U <- U + B_s R.
A and B are the 2N-storage coefficients of the cited method.  The stage times
c_s are derived from A and B as the value of U at the start of stage s when
integrating U' = 1 from U = 0 with dt = 1 (so they are consistent with A, B to
the last bit instead of being a separately rounded table).
"""

from __future__ import annotations

import numpy as np

LSRK_A = np.array([
    0.0,
    -567301805773.0 / 1357537059087.0,
    -2404267990393.0 / 2016746695238.0,
    -3550918686646.0 / 2091501179385.0,
    -1275806237668.0 / 842570457699.0,
])
LSRK_B = np.array([
    1432997174477.0 / 9575080441755.0,
    5161836677717.0 / 13612068292357.0,
    1720146321549.0 / 2090206949498.0,
    3134564353537.0 / 4481467310338.0,
    2277821191437.0 / 14882151754819.0,
])


def _stage_times():
    u, r = 0.0, 0.0
    c = np.zeros(5)
    for s in range(5):
        c[s] = u
        r = LSRK_A[s] * r + 1.0
        u = u + LSRK_B[s] * r
    return c


LSRK_C = _stage_times()


def lsrk_run(rhs, U, dt, nsteps, t0=0.0, R=None):
    """Advance U by nsteps LSRK(5,4) steps of size dt; returns (U, R)."""
    U = np.array(U, dtype=np.float64, copy=True)
    R = np.zeros_like(U) if R is None else np.array(R, dtype=np.float64, copy=True)
    t = t0
    for _ in range(nsteps):
        for s in range(5):
            R = LSRK_A[s] * R + dt * rhs(U, t + LSRK_C[s] * dt)
            U = U + LSRK_B[s] * R
        t += dt
    return U, R
