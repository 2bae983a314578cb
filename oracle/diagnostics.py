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


def ln_mean_branch_counts(mesh, U, gamma):
    """Branch structure the two-point flux meets on a state (collocated LGL
    mesh): for every volume pair of every line and every shared face-node pair,
    whether each of the two logarithmic means of the flux (of the density and
    of beta = rho / (2 p)) takes the series branch (squared relative jump below
    flux.LN_MEAN_SWITCH) or the closed form with its two logarithms.

    Returns {"pairs": total pairs, "series_rho": .., "series_beta": ..,
    "series_both": ..} as counts."""
    from .flux import LN_MEAN_SWITCH
    rho, _, _, beta = primitives(U, gamma)
    n = mesh.n

    def series(x, y):
        f = (x - y) / (x + y)
        return (f * f) < LN_MEAN_SWITCH

    tot = s_r = s_b = s_rb = 0
    for k in range(3):
        rk = rho.movedim(-1 - k, -1)
        bk = beta.movedim(-1 - k, -1)
        ia, ib = torch.triu_indices(n, n, offset=1)
        sr = series(rk[..., ia], rk[..., ib])
        sb = series(bk[..., ia], bk[..., ib])
        # the face pair across the +k face of every element (each shared face once)
        rn = mesh.neighbor(rho, k, 1).movedim(-1 - k, -1)
        bn = mesh.neighbor(beta, k, 1).movedim(-1 - k, -1)
        fr = series(rk[..., n - 1], rn[..., 0])
        fb = series(bk[..., n - 1], bn[..., 0])
        tot += sr.numel() + fr.numel()
        s_r += int(sr.sum()) + int(fr.sum())
        s_b += int(sb.sum()) + int(fb.sum())
        s_rb += int((sr & sb).sum()) + int((fr & fb).sum())
    return {"pairs": tot, "series_rho": s_r, "series_beta": s_b, "series_both": s_rb}
