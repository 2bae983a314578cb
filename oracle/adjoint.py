"""Derivatives of the semi-discrete operator (oracle; test infrastructure).

The paper has no adjoint; these are the reference derivatives the GPU adjoint
is checked against:
  * vjp               lambda^T d(du/dt)/dU by reverse-mode differentiation of
                      the oracle's own rhs (a library primitive applied to the
                      oracle forward);
  * jvp_complex_step  d(du/dt)/dU . w by the complex step Im f(U + i h w) / h,
                      an independent route used to pin vjp;
  * rk4_step_vjp      the discrete adjoint of one classical RK4 step;
  * ke_gradient       gradient of the domain kinetic energy after N RK4 steps
                      with respect to the initial state, by per-step
                      recomputation from stored step states.
"""
import torch


def vjp(scheme, U, lam, t=0.0):
    Ud = U.detach().clone().requires_grad_(True)
    out = scheme.rhs(Ud, t)
    (g,) = torch.autograd.grad(out, Ud, lam)
    return g


def jvp_complex_step(scheme, U, w, t=0.0, h=1e-30):
    Uc = U.to(torch.complex128) + 1j * h * w.to(torch.complex128)
    return scheme.rhs(Uc, t).imag / h


def rk4_step_vjp(scheme, U, dt, t, lam_next):
    Ud = U.detach().clone().requires_grad_(True)
    out = scheme.rk4_step(Ud, dt, t)
    (g,) = torch.autograd.grad(out, Ud, lam_next)
    return g


def kinetic_energy_objective(scheme, U):
    """J_KE = sum over nodes of W J rho |u|^2 / 2."""
    rho = U[0]
    ke = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho
    return (scheme.mesh.WJ * ke).sum()


def ke_gradient(scheme, U0, dt, nsteps, t0=0.0):
    """dJ_KE(U_N)/dU_0 for N classical RK4 steps of fixed dt."""
    states = [U0.detach().clone()]
    U = states[0]
    with torch.no_grad():
        for i in range(nsteps):
            U = scheme.rk4_step(U, dt, t0 + i * dt)
            states.append(U.clone())
    UN = states[-1].clone().requires_grad_(True)
    J = kinetic_energy_objective(scheme, UN)
    (lam,) = torch.autograd.grad(J, UN)
    for i in reversed(range(nsteps)):
        lam = rk4_step_vjp(scheme, states[i], dt, t0 + i * dt, lam)
    return float(J), lam
