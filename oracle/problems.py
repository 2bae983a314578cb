"""Manufactured solution of Sec. 7.1 (oracle; test infrastructure only).

Paper: Sec. 7.1 -- density 2 + sin(pi (x + y + z - 2t)) / 10, unit velocity in
every direction, rho e = rho^2, and the printed unsteady source q with
constants c1..c5 (c3 read as (pi/100)(gamma - 1): the printed comma is a
typesetting slip). Also the L2 error of Sec. 7.1 with the W J weights.
"""
import math

import torch


def mms_state(X, t, gamma):
    """Exact conservative state at coordinates X = (x, y, z), shape (5, ...)."""
    s = X[0] + X[1] + X[2] - 2.0 * t
    rho = 2.0 + 0.1 * torch.sin(math.pi * s)
    return torch.stack([rho, rho, rho, rho, rho * rho])


def mms_source(X, t, gamma):
    """Source q(x, t) of Sec. 7.1, shape (5, ...)."""
    pi = math.pi
    c1 = pi / 10.0
    c2 = -pi / 5.0 + pi / 20.0 * (1.0 + 5.0 * gamma)
    c3 = pi / 100.0 * (gamma - 1.0)
    c4 = pi / 20.0 * (-7.0 + 15.0 * gamma)
    c5 = pi / 100.0 * (3.0 * gamma - 2.0)
    s = X[0] + X[1] + X[2] - 2.0 * t
    cs, s2 = torch.cos(pi * s), torch.sin(2.0 * pi * s)
    m = c2 * cs + c3 * s2
    return torch.stack([c1 * cs, m, m, m, c4 * cs + c5 * s2])


def l2_error(mesh, U, Uex):
    """sqrt(sum_m (u_m - u_ex)^T W J_m (u_m - u_ex)) per state (Sec. 7.1)."""
    d = U - Uex
    return torch.sqrt((d * d * mesh.WJ).reshape(U.shape[0], -1).sum(1))
