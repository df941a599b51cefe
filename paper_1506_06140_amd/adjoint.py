"""Gradients of final-time functionals through the DG + SSP-RK3 trajectory.

``trajectory(solver, w0, nsteps, dt, checkpoint)`` runs ``nsteps`` unlimited
SSP-RK3 steps at a fixed time step (a device scalar) and is differentiable
with respect to the initial modal weights ``w0``.  The backward pass is the
hand-written discrete adjoint of the library (``dg_adjoint_rk_stage``): the
trajectory is stored every ``checkpoint`` steps in the forward pass; each
segment is recomputed (keeping the three stage inputs of every step) and
swept in reverse, stage 3 to stage 1.  The time step is held fixed so that
the map w0 -> w_T is differentiable; limiters are not part of it (smooth,
unlimited flow).
"""
from __future__ import annotations

import torch


def _forward_run(solver, w0, nsteps, dt, checkpoint):
    u1, u2 = solver.empty(), solver.empty()
    a = w0.detach().clone()
    b = solver.empty()
    saved = []
    for n in range(nsteps):
        if n % checkpoint == 0:
            saved.append(a.clone())
        out = solver.step(a, [u1, u2, b], dt=dt)
        a, b = out, a
    return a, saved


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w0, solver, nsteps, dt, checkpoint):
        if solver.limited:
            raise ValueError("the adjoint covers unlimited runs only")
        wT, saved = _forward_run(solver, w0, nsteps, dt, checkpoint)
        ctx.solver = solver
        ctx.nsteps = nsteps
        ctx.dt = dt
        ctx.checkpoint = checkpoint
        ctx.saved = saved
        return wT

    @staticmethod
    def backward(ctx, grad_out):
        s = ctx.solver
        dt = ctx.dt
        lam = grad_out.detach().contiguous().clone()
        lam_a, lam_b, acc = s.empty(), s.empty(), s.empty()
        nseg = len(ctx.saved)
        for seg in reversed(range(nseg)):
            n0 = seg * ctx.checkpoint
            n1 = min(n0 + ctx.checkpoint, ctx.nsteps)
            stages = []
            u = ctx.saved[seg]
            for _ in range(n0, n1):
                u1 = s.rk_stage(1, dt, None, u)
                u2 = s.rk_stage(2, dt, u, u1)
                u3 = s.rk_stage(3, dt, u, u2)
                stages.append((u, u1, u2))
                u = u3
            for u0, u1, u2 in reversed(stages):
                s.adjoint_rk_stage(3, dt, u2, lam, None, lam_a, acc)
                s.adjoint_rk_stage(2, dt, u1, lam_a, acc, lam_b, acc)
                s.adjoint_rk_stage(1, dt, u0, lam_b, acc, lam_a, None)
                lam, lam_a = lam_a, lam
            del stages
        ctx.saved = None
        return lam, None, None, None, None


def trajectory(solver, w0, nsteps: int, dt, checkpoint: int = 20):
    """w_T after `nsteps` fixed-dt SSP-RK3 steps; differentiable in w0."""
    return _Trajectory.apply(w0, solver, nsteps, dt, checkpoint)


def density_square_integral(solver, w):
    """J = int rho^2 dV = |K| sum_K sum_j (w_{j,rho}^K)^2 (orthonormal basis)."""
    return solver.dx ** solver.wl["dim"] * (w[0] ** 2).sum()
