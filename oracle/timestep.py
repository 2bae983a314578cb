"""Explicit time integration (oracle; test infrastructure only).

Paper: Sec. 7 (opening paragraph) -- a four-stage, fourth-order Runge-Kutta scheme with an
adaptive step from the maximum wave speed and CFL = 0.1. Reading: the classical
RK4 tableau; dt = CFL * dx / lambda_max with dx the mean node spacing
(hi - lo) / (ne (p + 1)) of the first direction.
"""
from .flux import max_wavespeed


def rk4_step(f, U, dt, t):
    """One classical RK4 step of dU/dt = f(U, t)."""
    k1 = f(U, t)
    k2 = f(U + 0.5 * dt * k1, t + 0.5 * dt)
    k3 = f(U + 0.5 * dt * k2, t + 0.5 * dt)
    k4 = f(U + dt * k3, t + dt)
    return U + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def cfl_dt(mesh, U, gamma, cfl=0.1):
    """dt = cfl * dx / max(|u| + c)."""
    dx = (mesh.hi - mesh.lo) / (mesh.ne[0] * mesh.n)
    return cfl * dx / max_wavespeed(U, gamma)
