"""Receiver misfit and its gradient with respect to per-element bulk modulus
kappa, as a ``torch.autograd.Function``.  With c^2 = kappa / rho the gradient
with respect to c^2 is rho times this one (equal to it for rho = 1, the
workload of the adjoint benchmark).

Forward: set kappa, run nsteps LSRK(5,4) steps from U0, sample the pressure
at the receivers after every step, and return
    J = dt/2 sum_{n=1..nsteps} sum_r (p(x_r, t_n) - d_{r,n})^2,
keeping the state every ``checkpoint_every`` steps.  Backward: segment by
segment from the end, recompute the segment's states from its checkpoint,
then reverse every step with ``dgpyr_adjoint_step`` (the discrete adjoint of
all five stages), injecting the receiver residuals before each step.  All
device work runs in the library's kernels; torch holds the arrays and forms
the scalar misfit.
"""

from __future__ import annotations

import torch

__all__ = ["ReceiverMisfit", "receiver_misfit"]


class ReceiverMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, solver, U0, data, dt, nsteps, checkpoint_every):
        solver.set_kappa(kappa)
        nrec = solver.nrec
        U = U0.clone()
        R = solver.empty_state().zero_()
        ckpts = {0: U.clone()}
        traces = torch.empty((nsteps, nrec), dtype=torch.float64, device=U.device)
        for n in range(nsteps):
            solver.step(U, R, dt, 1, t0=n * dt)
            solver.sample_receivers(U, traces[n])
            if (n + 1) % checkpoint_every == 0 and n + 1 < nsteps:
                ckpts[n + 1] = U.clone()
        res = traces - data
        J = 0.5 * dt * (res * res).sum()
        ctx.solver, ctx.dt, ctx.nsteps, ctx.every = solver, dt, nsteps, checkpoint_every
        ctx.ckpts, ctx.res = ckpts, res
        ctx.kappa_device, ctx.kappa_dtype = kappa.device, kappa.dtype
        return J

    @staticmethod
    def backward(ctx, gJ):
        s, dt, nsteps, every = ctx.solver, ctx.dt, ctx.nsteps, ctx.every
        Ub = s.empty_state().zero_()
        grad = torch.zeros(s.K, dtype=torch.float64, device=Ub.device)
        starts = sorted(ctx.ckpts)
        R = s.empty_state()
        for k in range(len(starts) - 1, -1, -1):
            n0 = starts[k]
            n1 = starts[k + 1] if k + 1 < len(starts) else nsteps
            # states U_{n0} .. U_{n1 - 1} of the segment
            states = [ctx.ckpts[n0].clone()]
            U = states[0].clone()
            R.zero_()
            for n in range(n0, n1 - 1):
                s.step(U, R, dt, 1, t0=n * dt)
                states.append(U.clone())
            for n in range(n1 - 1, n0 - 1, -1):
                coef = (dt * gJ) * ctx.res[n]
                s.inject_receivers(Ub, coef.contiguous())
                s.adjoint_step(states[n - n0], Ub, grad, n * dt, dt)
            del states
        g = grad.to(device=ctx.kappa_device, dtype=ctx.kappa_dtype)
        return g, None, None, None, None, None, None


def receiver_misfit(kappa, solver, U0, data, dt, nsteps, checkpoint_every=20):
    """J(kappa) with a gradient through the discrete adjoint (see module docstring)."""
    return ReceiverMisfit.apply(kappa, solver, U0, data, float(dt), int(nsteps),
                                int(checkpoint_every))
