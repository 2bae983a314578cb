"""Euler fluxes, entropy variables and the entropy-conserving two-point flux
(oracle; test infrastructure only).

Paper: Sec. 2.1 (entropy variables v = U'(u), entropy potential, Tadmor's
shuffle condition, Eq. EC flux; 3D Euler system and its fluxes), Sec. 3.3
(two-point flux choice: Chandrashekar's flux in the variables rho, u and
beta = rho / (2p)) and Sec. 7 opening paragraph (the experiments use Chandrashekar's flux with
Ranocha's pressure fix in volume and surface).

Readings of the paper used here:
  * the entropy is U = -rho s / (gamma - 1) with s = ln p - gamma ln rho, which
    gives v = [(gamma - s)/(gamma - 1) - beta |u|^2, 2 beta u, -2 beta] and
    entropy potential psi^k = rho u_k;
  * "Chandrashekar with Ranocha's pressure fix" (variant 0) uses the
    arithmetic-mean pressure in the momentum flux, and the energy flux is the
    unique completion that satisfies Tadmor's condition:
        f_rho = rho_ln un_avg
        f_m   = u_avg f_rho + p_avg N
        f_E   = f_rho (1 / (2 (gamma-1) beta_ln) + u_a . u_b / 2)
                + (p_a un_b + p_b un_a) / 2
    variant 1 is plain Chandrashekar (pressure rho_avg / (2 beta_avg));
  * the logarithmic mean uses the series of Ismail and Roe when the squared
    relative jump is below 1e-4, and the closed form otherwise.

All two-point fluxes take a direction vector N (not normalised) and are linear
in it. Works for float64 and complex128 tensors (branches use real parts).
"""
import torch

LN_MEAN_SWITCH = 1e-4


def primitives(U, gamma):
    """rho, (u, v, w), p, beta from conservative U = [rho, rho u, rho v, rho w, rho e]
    with rho e = p / (gamma - 1) + rho |u|^2 / 2 (Sec. 2.1)."""
    rho = U[0]
    vel = [U[1] / rho, U[2] / rho, U[3] / rho]
    kin = 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    p = (gamma - 1.0) * (U[4] - kin)
    beta = rho / (2.0 * p)
    return rho, vel, p, beta


def conservative(rho, vel, p, gamma):
    """U from primitives (Sec. 2.1)."""
    rhoe = p / (gamma - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return torch.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2], rhoe])


def physical_flux(U, gamma):
    """Physical Euler flux f_k(U), k = 1..3, shape (3, 5, ...) (Sec. 2.1)."""
    rho, vel, p, _ = primitives(U, gamma)
    rhoe = U[4]
    out = []
    for k in range(3):
        uk = vel[k]
        fk = [rho * uk,
              rho * vel[0] * uk + (p if k == 0 else 0.0 * p),
              rho * vel[1] * uk + (p if k == 1 else 0.0 * p),
              rho * vel[2] * uk + (p if k == 2 else 0.0 * p),
              (rhoe + p) * uk]
        out.append(torch.stack(fk))
    return torch.stack(out)


def entropy_variables(U, gamma):
    """v = dU/du for the entropy U = -rho s / (gamma - 1), s = ln p - gamma ln rho."""
    rho, vel, p, beta = primitives(U, gamma)
    s = torch.log(p) - gamma * torch.log(rho)
    q2 = vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2
    return torch.stack([(gamma - s) / (gamma - 1.0) - beta * q2,
                        2 * beta * vel[0], 2 * beta * vel[1], 2 * beta * vel[2],
                        -2 * beta])


def entropy_function(U, gamma):
    """Mathematical entropy U(u) = -rho s / (gamma - 1)."""
    rho, _, p, _ = primitives(U, gamma)
    s = torch.log(p) - gamma * torch.log(rho)
    return -rho * s / (gamma - 1.0)


def entropy_potential(U, gamma):
    """psi^k = v . f^k - F^k = rho u_k (Eq. entropy pot with flux relationship)."""
    rho, vel, _, _ = primitives(U, gamma)
    return torch.stack([rho * vel[0], rho * vel[1], rho * vel[2]])


def _re(t):
    return t.real if torch.is_complex(t) else t


def ln_mean(a, b):
    """Logarithmic mean (a - b) / (ln a - ln b), with (a + b) / 2 at a = b."""
    s = a + b
    d = a - b
    f = d / s
    u = f * f
    small = _re(u) < LN_MEAN_SWITCH
    series = s / (2.0 * (1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u / 7.0))))
    # evaluate the closed form on harmless stand-ins where the series is used,
    # so that neither branch produces NaN (or NaN derivatives)
    a_s = torch.where(small, torch.full_like(a, 2.0), a)
    b_s = torch.where(small, torch.ones_like(b), b)
    closed = (a_s - b_s) / (torch.log(a_s) - torch.log(b_s))
    return torch.where(small, series, closed)


def ec_flux(Ua, Ub, N, gamma, variant=0):
    """Entropy-conserving, kinetic-energy-preserving two-point flux
    f_s(Ua, Ub) . N for direction vector N = (Nx, Ny, Nz) (Eq. Tadmor shuffle
    quad node; Sec. 3.3). Returns a stacked (5, ...) tensor."""
    ra, va, pa, ba = primitives(Ua, gamma)
    rb, vb, pb, bb = primitives(Ub, gamma)
    rho_ln = ln_mean(ra, rb)
    beta_ln = ln_mean(ba, bb)
    u_avg = [0.5 * (va[k] + vb[k]) for k in range(3)]
    un_a = va[0] * N[0] + va[1] * N[1] + va[2] * N[2]
    un_b = vb[0] * N[0] + vb[1] * N[1] + vb[2] * N[2]
    un_avg = 0.5 * (un_a + un_b)
    f_rho = rho_ln * un_avg
    if variant == 0:
        p_avg = 0.5 * (pa + pb)
        f_m = [u_avg[k] * f_rho + p_avg * N[k] for k in range(3)]
        uaub = va[0] * vb[0] + va[1] * vb[1] + va[2] * vb[2]
        f_E = f_rho * (1.0 / (2.0 * (gamma - 1.0) * beta_ln) + 0.5 * uaub) + 0.5 * (pa * un_b + pb * un_a)
    else:
        p_hat = 0.5 * (ra + rb) / (ba + bb)
        f_m = [u_avg[k] * f_rho + p_hat * N[k] for k in range(3)]
        qa = va[0] ** 2 + va[1] ** 2 + va[2] ** 2
        qb = vb[0] ** 2 + vb[1] ** 2 + vb[2] ** 2
        f_E = (f_rho * (1.0 / (2.0 * (gamma - 1.0) * beta_ln) - 0.25 * (qa + qb))
               + u_avg[0] * f_m[0] + u_avg[1] * f_m[1] + u_avg[2] * f_m[2])
    return torch.stack([f_rho, f_m[0], f_m[1], f_m[2], f_E])


def llf_dissipation(Ua, Ub, N, gamma):
    """Local Lax-Friedrichs term -|N| lambda_max (Ub - Ua) / 2 added to the EC
    surface flux for the manufactured-solution runs (the paper adds an upwind
    dissipation there, read here as LLF on the conservative jumps).
    lambda_max = max over both sides of |u . N/|N|| + sqrt(gamma p / rho).
    Real tensors only. Pinned by a hand-computed pair, antisymmetry, zero jump
    and entropy dissipation (the jump of the entropy variables times this term
    is never positive)."""
    ra, va, pa, _ = primitives(Ua, gamma)
    rb, vb, pb, _ = primitives(Ub, gamma)
    nn = torch.sqrt(N[0] ** 2 + N[1] ** 2 + N[2] ** 2)
    una = (va[0] * N[0] + va[1] * N[1] + va[2] * N[2]) / nn
    unb = (vb[0] * N[0] + vb[1] * N[1] + vb[2] * N[2]) / nn
    lam = torch.maximum(una.abs() + torch.sqrt(gamma * pa / ra), unb.abs() + torch.sqrt(gamma * pb / rb))
    return -0.5 * lam * nn * (Ub - Ua)


def roe_dissipation(Ua, Ub, N, gamma):
    """Entropy-stable Roe-type matrix dissipation on the jump of the entropy
    variables, -|N| R |Lambda| T R^T (v_b - v_a) / 2, added to the EC surface
    flux (Sec. 6.3: Roe's dissipation recast with entropy-variable jumps is
    provably entropy dissipative; Sec. 7.1: the manufactured-solution runs add
    Roe dissipation to the EC flux).

    Reading: R, |Lambda| and T are the eigenvectors, the absolute eigenvalues
    and Barth's eigenvector scaling (R T R^T = du/dv) of the Euler flux
    Jacobian in the direction n = N / |N|, all evaluated at one averaged state
    (rho_ln, arithmetic-mean velocity, p = mean(rho) / (2 mean(beta))).
    Because R T R^T is symmetric positive definite and |Lambda| >= 0, the
    entropy production -(v_b - v_a) . term is never positive.

      waves n -+ a:  r = [1, u -+ a n, h -+ a u.n],  T = rho / (2 gamma)
      entropy wave:  r = [1, u, |u|^2 / 2],          T = (gamma - 1) rho / gamma
      shear waves:   sum_t T r r^T dv with T = p, r = [0, t, u.t], t _|_ n,
                     = p [0, P w, u . P w], P = I - n n^T, w = dv_m + u dv_E
    with h = a^2 / (gamma - 1) + |u|^2 / 2, a = sqrt(gamma p / rho). Real
    tensors only."""
    ra, va, pa, ba = primitives(Ua, gamma)
    rb, vb, pb, bb = primitives(Ub, gamma)
    rho = ln_mean(ra, rb)
    u = [0.5 * (va[k] + vb[k]) for k in range(3)]
    p = 0.5 * (ra + rb) / (ba + bb)
    nn = torch.sqrt(N[0] ** 2 + N[1] ** 2 + N[2] ** 2)
    n = [N[k] / nn for k in range(3)]
    a = torch.sqrt(gamma * p / rho)
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    h = a * a / (gamma - 1.0) + 0.5 * q2
    un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2]
    dv = entropy_variables(Ub, gamma) - entropy_variables(Ua, gamma)
    out = torch.zeros_like(Ua)
    # acoustic waves
    for sgn in (-1.0, 1.0):
        r = [torch.ones_like(rho)] + [u[k] + sgn * a * n[k] for k in range(3)] + [h + sgn * a * un]
        c = sum(r[i] * dv[i] for i in range(5)) * (un + sgn * a).abs() * rho / (2.0 * gamma)
        out = out + torch.stack([c * r[i] for i in range(5)])
    # entropy wave
    r = [torch.ones_like(rho)] + u + [0.5 * q2]
    c = sum(r[i] * dv[i] for i in range(5)) * un.abs() * (gamma - 1.0) * rho / gamma
    out = out + torch.stack([c * r[i] for i in range(5)])
    # shear waves
    w = [dv[1 + k] + u[k] * dv[4] for k in range(3)]
    wn = w[0] * n[0] + w[1] * n[1] + w[2] * n[2]
    Pw = [w[k] - wn * n[k] for k in range(3)]
    c = un.abs() * p
    uPw = u[0] * Pw[0] + u[1] * Pw[1] + u[2] * Pw[2]
    out = out + torch.stack([torch.zeros_like(rho), c * Pw[0], c * Pw[1], c * Pw[2], c * uPw])
    return -0.5 * nn * out


def roe_flux(Ua, Ub, N, gamma):
    """Roe's approximate Riemann solver (Roe 1981), the surface numerical flux
    of the conservative DG scheme the paper compares against (Sec. 7.4):
    N . f* = (f(U_a) + f(U_b)) . N / 2 - |N| |A^| (U_b - U_a) / 2, with A^ the
    flux Jacobian in n = N / |N| at Roe's average (sqrt(rho)-weighted velocity
    and total enthalpy H = (rho e + p) / rho; rho^ = sqrt(rho_a rho_b)), so that
    A^ (U_b - U_a) = (f(U_b) - f(U_a)) . n. |A^| dU is written wave by wave:
      acoustic n -+ c:  strength (dp -+ rho^ c dun) / (2 c^2),
                        r = [1, u -+ c n, H -+ c u.n];
      entropy:          strength drho - dp / c^2, r = [1, u, |u|^2 / 2];
      shear:            rho^ [0, du - dun n, u . du - u.n dun], speed u.n;
    c^2 = (gamma - 1)(H - |u|^2 / 2). No entropy fix (the compared flows are
    subsonic). Real tensors only."""
    ra, va, pa, _ = primitives(Ua, gamma)
    rb, vb, pb, _ = primitives(Ub, gamma)
    nn = torch.sqrt(N[0] ** 2 + N[1] ** 2 + N[2] ** 2)
    n = [N[k] / nn for k in range(3)]
    sa, sb = torch.sqrt(ra), torch.sqrt(rb)
    w = 1.0 / (sa + sb)
    u = [(sa * va[k] + sb * vb[k]) * w for k in range(3)]
    Ha, Hb = (Ua[4] + pa) / ra, (Ub[4] + pb) / rb
    H = (sa * Ha + sb * Hb) * w
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    c = torch.sqrt((gamma - 1.0) * (H - 0.5 * q2))
    rho = sa * sb
    un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2]
    dr, dp = rb - ra, pb - pa
    du = [vb[k] - va[k] for k in range(3)]
    dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2]
    one = torch.ones_like(rho)
    d = torch.zeros_like(Ua)
    for sg in (-1.0, 1.0):
        a = (dp + sg * rho * c * dun) / (2.0 * c * c) * (un + sg * c).abs()
        r = [one] + [u[k] + sg * c * n[k] for k in range(3)] + [H + sg * c * un]
        d = d + torch.stack([a * r[i] for i in range(5)])
    a = (dr - dp / (c * c)) * un.abs()
    d = d + torch.stack([a, a * u[0], a * u[1], a * u[2], a * 0.5 * q2])
    sh = [du[k] - dun * n[k] for k in range(3)]
    b = rho * un.abs()
    d = d + torch.stack([0.0 * b, b * sh[0], b * sh[1], b * sh[2], b * (u[0] * du[0] + u[1] * du[1] + u[2] * du[2]
                                                                      - un * dun)])
    fa, fb = physical_flux(Ua, gamma), physical_flux(Ub, gamma)
    central = 0.5 * sum((fa[k] + fb[k]) * N[k] for k in range(3))
    return central - 0.5 * nn * d


def surface_dissipation(kind, gamma):
    """The dissipation term added to the EC surface flux: None for kind 0 /
    False, local Lax-Friedrichs for kind 1 / True / "llf", the entropy-stable
    Roe-type matrix dissipation for kind 2 / "roe"."""
    if kind is None or kind is False or kind == 0:
        return None
    if kind is True or kind == 1 or kind == "llf":
        return lambda a, b, N: llf_dissipation(a, b, N, gamma)
    if kind == 2 or kind == "roe":
        return lambda a, b, N: roe_dissipation(a, b, N, gamma)
    raise ValueError(f"unknown surface dissipation {kind!r}")


def max_wavespeed(U, gamma):
    """max over nodes of |u| + sqrt(gamma p / rho) (Sec. 7 opening paragraph: adaptive step)."""
    rho, vel, p, _ = primitives(U, gamma)
    speed = torch.sqrt(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2) + torch.sqrt(gamma * p / rho)
    return float(speed.max())
