"""Conservation, entropy and kinetic-energy diagnostics (oracle; test
infrastructure only).

Paper: Sec. 6.2 (global conservation: 1^T (M_m + K_m) du/dt sums surface
fluxes only), Sec. 6.3 (entropy conservation: v^T (M_m + K_m) du/dt reduces to
surface entropy-potential terms that cancel on a periodic mesh), Sec. 6.3
Lemma (kinetic-energy variables), Sec. 7.3 (entropy change and conservation
reported at round-off).

With du/dt = -A R and (M_m + K_m) read as A^-1, v^T (M_m + K_m) du/dt = -v^T R.
"""
import torch

from .flux import entropy_variables, primitives


def entropy_rate(U, R, gamma):
    """(sum v . R, sum |v . R|) over all nodes and states."""
    v = entropy_variables(U, gamma)
    vr = v * R
    return float(vr.sum()), float(vr.abs().sum())


def conservation(R):
    """sum of R over all nodes, per state."""
    return R.reshape(R.shape[0], -1).sum(1)


def kinetic_energy_variables(U, gamma):
    """v_KE = [-|u|^2 / 2, u, v, w, 0] (Lemma in Sec. 6.3, Eq. kin energy var)."""
    rho, vel, _, _ = primitives(U, gamma)
    q2 = vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2
    return torch.stack([-0.5 * q2, vel[0], vel[1], vel[2], torch.zeros_like(q2)])


def kinetic_energy(mesh, U, gamma):
    """sum over nodes of W J rho |u|^2 / 2."""
    rho, vel, _, _ = primitives(U, gamma)
    return float((mesh.WJ * 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)).sum())
