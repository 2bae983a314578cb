"""Adjoint of the NSFR right-hand side for PyTorch, and time-integrated
sensitivities with step checkpointing.

`NSFRRhs.apply(U, solver, t)` returns dU/dt through `nsfr_rhs` and
back-propagates through `nsfr_rhs_vjp` (the hand-written discrete adjoint
kernels). `kinetic_energy_gradient` integrates N classical RK4 steps, keeps the
step states U^n as checkpoints, and runs the discrete RK4 adjoint backwards
(`nsfr_rk4_step_vjp` recomputes the stage states of each step from its
checkpoint). All arithmetic runs in the library's kernels; this module only
orders the calls and holds the checkpoints.
"""
import torch


class NSFRRhs(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, solver, t=0.0):
        U = U.contiguous()
        ctx.solver, ctx.t = solver, float(t)
        ctx.save_for_backward(U)
        return solver.rhs(U, t=t)

    @staticmethod
    def backward(ctx, grad):
        (U,) = ctx.saved_tensors
        return ctx.solver.rhs_vjp(U, grad.contiguous(), t=ctx.t), None, None


def rhs(U, solver, t=0.0):
    return NSFRRhs.apply(U, solver, t)


def integrate(solver, U0, dt, nsteps, t0=0.0, checkpoints=False):
    """nsteps RK4 steps from U0 (not modified). dt is a 1-element device tensor.
    Returns U_N, and the list of step states U_0..U_{N-1} if requested."""
    U = U0.clone()
    work = solver.work(3)
    h = float(dt) if solver.cfg.source else 0.0
    ck = []
    for i in range(nsteps):
        if checkpoints:
            ck.append(U.clone())
        solver.rk4_step(U, dt, t0 + i * h, work)
    return (U, ck) if checkpoints else U


def kinetic_energy_gradient(solver, U0, dt, nsteps, t0=0.0):
    """J = sum W J rho |u|^2 / 2 at step N and dJ/dU0 by the discrete adjoint."""
    UN, ck = integrate(solver, U0, dt, nsteps, t0, checkpoints=True)
    lam = solver.empty()
    ke, _ = solver.kinetic_energy(UN, grad=lam)
    work = solver.work(6)
    h = float(dt) if solver.cfg.source else 0.0
    for i in reversed(range(nsteps)):
        solver.rk4_step_vjp(ck[i], dt, lam, t=t0 + i * h, out=lam, work=work)
    return ke, lam
