"""The NSFR right-hand side evaluated in extended precision (oracle; test
infrastructure only).

Purpose: round-off attribution. The smooth low-Mach states of the
Taylor-Green vortex make the residual a small difference of large terms (the
momentum residual is the derivative of a pressure of about 71 that varies by
about 0.3), so two FP64 evaluations of the same definition differ by far more
than eps |R|. This module evaluates the same definitions as the FP64 oracle
with numpy's extended type (x87 80-bit long double on x86-64: 64-bit
significand, unit round-off 5.4e-20), so that both the FP64 oracle and the
GPU can be measured against a result whose own round-off is about 2000 times
smaller.

It is written independently of the FP64 oracle modules (numpy instead of
PyTorch, its own small dense solver) and follows the paper's definitions:
  * LGL nodes, weights, barycentric derivative matrix, S1 = W D - D^T W
    (Sec. 2.2, Eq. SBP);
  * K = c (D^p)^T W D^p and Pi~ = (W + K)^-1 W (Sec. 3.2 Eq. Km, Sec. 4
    Eq. Fr projection);
  * the warped map of Sec. 7 (Eq. warped grid), metric cofactors by the
    conservative curl form on element-local coordinates (Sec. 2.2, Eq. GCL);
  * the residual of Eq. NSFR on collocated LGL nodes: volume two-point flux
    differencing along every line and the shared-face numerical flux
    (Sec. 3.3, Sec. 5), Chandrashekar's flux with Ranocha's pressure fix or
    plain Chandrashekar, optional local Lax-Friedrichs term and manufactured
    source (Sec. 7.1);
  * dU/dt = -Pi~_3 (W J)^-1 Pi~_3^T R (Sec. 4, Eq. weight-adj ESFR mass).

All arrays use the layout of the FP64 oracle: state (5, E, n, n, n) indexed
[s, e, c, b, a] with a the xi index, element e = ex + nx (ey + ny ez).
"""
import math

import numpy as np

LD = np.longdouble
LN_MEAN_SWITCH = 1e-4


def _pi(dt):
    return dt(4) * np.arctan(dt(1))


# ---------------------------------------------------------------- operators

def _legendre(p, x):
    P0, P1 = np.ones_like(x), x.copy()
    for k in range(2, p + 1):
        P0, P1 = P1, ((2 * k - 1) * x * P1 - (k - 1) * P0) / k
    return P1, P0


def _solve(A, B):
    """A^-1 B by Gauss-Jordan elimination with partial pivoting (small n)."""
    A = A.copy()
    X = B.copy()
    n = A.shape[0]
    for k in range(n):
        piv = k + int(np.argmax(np.abs(A[k:, k])))
        if piv != k:
            A[[k, piv]] = A[[piv, k]]
            X[[k, piv]] = X[[piv, k]]
        r = A[k, k]
        A[k] = A[k] / r
        X[k] = X[k] / r
        for i in range(n):
            if i != k:
                f = A[i, k]
                A[i] = A[i] - f * A[k]
                X[i] = X[i] - f * X[k]
    return X


class Ops1D:
    """1D LGL operators of degree p and FR parameter c in the scalar type dt."""

    def __init__(self, p, c=0.0, dt=LD):
        n = p + 1
        self.p, self.n = p, n
        pi = _pi(dt)
        x = -np.cos(pi * np.arange(n, dtype=dt) / dt(p))
        for _ in range(200):   # Newton on p (P_{p-1} - x P_p), derivative -p (p+1) P_p
            Pp, Pm = _legendre(p, x)
            dx = (x * Pp - Pm) / ((p + 1) * Pp)
            x = x - dx
            if float(np.max(np.abs(dx))) < 1e-21:
                break
        x = (x - x[::-1]) / 2
        x[0], x[-1] = -1, 1
        Pp, _ = _legendre(p, x)
        w = dt(2) / (p * (p + 1) * Pp * Pp)
        w = (w + w[::-1]) / 2
        self.x, self.w = x, w
        lam = np.array([dt(1) / np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)], dtype=dt)
        D = np.zeros((n, n), dtype=dt)
        for i in range(n):
            for j in range(n):
                if i != j:
                    D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
            D[i, i] = -sum(D[i, j] for j in range(n) if j != i)
        self.D = D
        W = np.diag(w)
        self.S1 = W @ D - D.T @ W
        Dp = np.eye(n, dtype=dt)
        for _ in range(p):
            Dp = Dp @ D
        K = dt(c) * (Dp.T @ W @ Dp)
        self.Pi = _solve(W + K, W)


# ---------------------------------------------------------------- mesh

def _apply_D(D, F, axis):
    """Apply D along reference direction axis (0 = xi = last dim) of (..., n, n, n)."""
    F = np.moveaxis(F, -1 - axis, -1)
    G = F @ D.T
    return np.moveaxis(G, -1, -1 - axis)


class MeshX:
    """Warped periodic box [lo, hi]^3, ne elements per direction, degree p.

    elements: optional list of global element ids; the mesh terms are then
    computed for those elements only (in the order given), for sampled
    evaluations of large meshes. Element terms are element-local, so a subset
    is computed exactly as on the full mesh."""

    def __init__(self, p, ne, lo=0.0, hi=None, beta=0.0, l=None, dt=LD, elements=None):
        self.dt = dt
        pi = _pi(dt)
        self.p, self.n = p, p + 1
        self.ne = tuple(int(v) for v in ne)
        nx, ny, nz = self.ne
        self.E = nx * ny * nz
        lo = dt(lo)
        hi = 2 * pi if hi is None else dt(hi)
        self.lo, self.hi = lo, hi
        ll = (hi - lo) / (2 * pi) if (l is None or l <= 0) else dt(l)
        ops = Ops1D(p, 0.0, dt)
        self.ops = ops
        e = np.arange(self.E) if elements is None else np.asarray(elements, dtype=np.int64)
        self.ids = e
        self.loc = np.full(self.E, -1, dtype=np.int64)
        self.loc[e] = np.arange(e.size)
        ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
        h = [(hi - lo) / dt(m) for m in self.ne]
        xi = ops.x
        A = lo + h[0] * (ex[:, None, None, None].astype(dt) + (xi[None, None, None, :] + 1) / 2)
        B = lo + h[1] * (ey[:, None, None, None].astype(dt) + (xi[None, None, :, None] + 1) / 2)
        C = lo + h[2] * (ez[:, None, None, None].astype(dt) + (xi[None, :, None, None] + 1) / 2)
        A, B, C = np.broadcast_arrays(A, B, C)
        b = dt(beta)
        X = np.stack([A + b * np.sin(A / ll) * np.sin(B / ll) * np.sin(2 * C / ll),
                      B + b * np.sin(4 * A / ll) * np.sin(B / ll) * np.sin(3 * C / ll),
                      C + b * np.sin(2 * A / ll) * np.sin(5 * B / ll) * np.sin(C / ll)])
        self.X = X
        ctr = np.stack([lo + h[0] * (ex.astype(dt) + dt(0.5)), lo + h[1] * (ey.astype(dt) + dt(0.5)),
                        lo + h[2] * (ez.astype(dt) + dt(0.5))])
        Xl = X - ctr[:, :, None, None, None]
        D = ops.D
        G = [[_apply_D(D, X[m], j) for j in range(3)] for m in range(3)]
        J = (G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1])
             - G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0])
             + G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]))
        self.J = J
        Cm = np.empty((3, 3) + J.shape, dtype=dt)
        for (a, m, q) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
            V = [Xl[q] * G[m][j] for j in range(3)]
            Cm[a, 0] = -(_apply_D(D, V[2], 1) - _apply_D(D, V[1], 2))
            Cm[a, 1] = -(_apply_D(D, V[0], 2) - _apply_D(D, V[2], 0))
            Cm[a, 2] = -(_apply_D(D, V[1], 0) - _apply_D(D, V[0], 1))
        self.C = Cm
        w = ops.w
        self.W3 = (w[None, None, None, :] * w[None, None, :, None] * w[None, :, None, None]) * np.ones_like(J)
        self.WJ = self.W3 * J

    def neighbour_ids(self, ids, axis, side):
        """Global ids of the periodic neighbours of elements ids across face (axis, side)."""
        nx, ny, nz = self.ne
        c = [ids % nx, (ids // nx) % ny, ids // (nx * ny)]
        c[axis] = (c[axis] + side) % self.ne[axis]
        return c[0] + nx * (c[1] + ny * c[2])


# ---------------------------------------------------------------- flux

def primitives(U, gamma):
    rho = U[0]
    u, v, w = U[1] / rho, U[2] / rho, U[3] / rho
    p = (gamma - 1) * (U[4] - (U[1] * u + U[2] * v + U[3] * w) / 2)
    return rho, (u, v, w), p, rho / (2 * p)


def ln_mean(a, b):
    s, d = a + b, a - b
    f = d / s
    u = f * f
    small = u < LN_MEAN_SWITCH
    # series of (a - b) / ln(a / b) in u = ((a - b)/(a + b))^2, carried further
    # than the FP64 switch needs so that it is exact in this precision
    q = 1 + u * (LD(1) / 3 + u * (LD(1) / 5 + u * (LD(1) / 7 + u * (LD(1) / 9 + u * (LD(1) / 11)))))
    series = s / (2 * q)
    a2 = np.where(small, 2, a)
    b2 = np.where(small, 1, b)
    closed = (a2 - b2) / (np.log(a2) - np.log(b2))
    return np.where(small, series, closed)


def ec_flux(Ua, Ub, N, gamma, variant=0):
    ra, va, pa, ba = primitives(Ua, gamma)
    rb, vb, pb, bb = primitives(Ub, gamma)
    una = va[0] * N[0] + va[1] * N[1] + va[2] * N[2]
    unb = vb[0] * N[0] + vb[1] * N[1] + vb[2] * N[2]
    un = (una + unb) / 2
    frho = ln_mean(ra, rb) * un
    bln = ln_mean(ba, bb)
    um = [(va[k] + vb[k]) / 2 for k in range(3)]
    if variant == 0:
        pm = (pa + pb) / 2
        fm = [um[k] * frho + pm * N[k] for k in range(3)]
        fE = frho * (1 / (2 * (gamma - 1) * bln) + (va[0] * vb[0] + va[1] * vb[1] + va[2] * vb[2]) / 2) \
            + (pa * unb + pb * una) / 2
    else:
        ph = (ra + rb) / 2 / (ba + bb)
        fm = [um[k] * frho + ph * N[k] for k in range(3)]
        qa = va[0] ** 2 + va[1] ** 2 + va[2] ** 2
        qb = vb[0] ** 2 + vb[1] ** 2 + vb[2] ** 2
        fE = frho * (1 / (2 * (gamma - 1) * bln) - (qa + qb) / 4) + um[0] * fm[0] + um[1] * fm[1] + um[2] * fm[2]
    return np.stack([frho, fm[0], fm[1], fm[2], fE])


def llf(Ua, Ub, N, gamma):
    ra, va, pa, _ = primitives(Ua, gamma)
    rb, vb, pb, _ = primitives(Ub, gamma)
    nn = np.sqrt(N[0] ** 2 + N[1] ** 2 + N[2] ** 2)
    una = np.abs(va[0] * N[0] + va[1] * N[1] + va[2] * N[2]) / nn
    unb = np.abs(vb[0] * N[0] + vb[1] * N[1] + vb[2] * N[2]) / nn
    lam = np.maximum(una + np.sqrt(gamma * pa / ra), unb + np.sqrt(gamma * pb / rb))
    return -lam * nn * (Ub - Ua) / 2


def _entropy_vars(U, gamma):
    rho, (u, v, w), p, beta = primitives(U, gamma)
    s = np.log(p) - gamma * np.log(rho)
    return np.stack([(gamma - s) / (gamma - 1) - beta * (u * u + v * v + w * w),
                     2 * beta * u, 2 * beta * v, 2 * beta * w, -2 * beta])


def roe(Ua, Ub, N, gamma):
    """Entropy-stable Roe-type matrix dissipation -|N| R |Lambda| T R^T [v] / 2
    at the averaged state (rho_ln, mean velocity, mean(rho) / (2 mean(beta))),
    written out as the rank-one sum over the acoustic and entropy waves plus
    the shear block p |u.n| (I - n n^T) acting on w = [v]_m + u [v]_E."""
    ra, ua, pa, ba = primitives(Ua, gamma)
    rb, ub, pb, bb = primitives(Ub, gamma)
    rho = ln_mean(ra, rb)
    u = [(ua[k] + ub[k]) / 2 for k in range(3)]
    p = (ra + rb) / (2 * (ba + bb))
    nn = np.sqrt(N[0] ** 2 + N[1] ** 2 + N[2] ** 2)
    n = [N[k] / nn for k in range(3)]
    a = np.sqrt(gamma * p / rho)
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    h = a * a / (gamma - 1) + q2 / 2
    un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2]
    dv = _entropy_vars(Ub, gamma) - _entropy_vars(Ua, gamma)
    one = np.ones_like(rho)
    waves = []
    for sg in (-1, 1):
        r = [one, u[0] + sg * a * n[0], u[1] + sg * a * n[1], u[2] + sg * a * n[2], h + sg * a * un]
        waves.append((r, np.abs(un + sg * a) * rho / (2 * gamma)))
    waves.append(([one, u[0], u[1], u[2], q2 / 2], np.abs(un) * (gamma - 1) * rho / gamma))
    D = np.zeros_like(Ua)
    for r, sc in waves:
        proj = sum(r[i] * dv[i] for i in range(5)) * sc
        for i in range(5):
            D[i] = D[i] + proj * r[i]
    w = [dv[1 + k] + u[k] * dv[4] for k in range(3)]
    wn = w[0] * n[0] + w[1] * n[1] + w[2] * n[2]
    Pw = [w[k] - wn * n[k] for k in range(3)]
    sc = np.abs(un) * p
    for k in range(3):
        D[1 + k] = D[1 + k] + sc * Pw[k]
    D[4] = D[4] + sc * (u[0] * Pw[0] + u[1] * Pw[1] + u[2] * Pw[2])
    return -nn * D / 2


def mms_source(X, t, gamma, dt=LD):
    pi = _pi(dt)
    g = dt(gamma)
    c1 = pi / 10
    c2 = -pi / 5 + pi / 20 * (1 + 5 * g)
    c3 = pi / 100 * (g - 1)
    c4 = pi / 20 * (-7 + 15 * g)
    c5 = pi / 100 * (3 * g - 2)
    s = X[0] + X[1] + X[2] - 2 * dt(t)
    cs, s2 = np.cos(pi * s), np.sin(2 * pi * s)
    m = c2 * cs + c3 * s2
    return np.stack([c1 * cs, m, m, m, c4 * cs + c5 * s2])


# ---------------------------------------------------------------- residual

class SchemeX:
    """Residual and right-hand side in the scalar type dt (default long double).

    elements: optional list of global element ids at which to evaluate (a
    sample of a large mesh); outputs then have shape (5, len(elements), n, n, n)
    in that order. Inputs are always full state arrays (5, E, n, n, n)."""

    def __init__(self, p, ne, lo=0.0, hi=None, beta=0.0, l=None, gamma=1.4, c=0.0, variant=0,
                 dissipation=False, source=False, dt=LD, elements=None):
        self.dt = dt
        ne = tuple(int(v) for v in ne)
        E = ne[0] * ne[1] * ne[2]
        self.target = np.arange(E) if elements is None else np.asarray(elements, dtype=np.int64)
        probe = MeshX(1, ne, lo, hi, 0.0, l, dt, elements=self.target[:1])
        need = [self.target]
        for k in range(3):
            for side in (-1, 1):
                need.append(probe.neighbour_ids(self.target, k, side))
        ids = np.unique(np.concatenate(need)) if elements is not None else None
        self.mesh = MeshX(p, ne, lo, hi, beta, l, dt, elements=ids)
        self.p, self.n = p, p + 1
        self.gamma = dt(gamma)
        self.variant = variant
        self.dissipation, self.source = int(dissipation), bool(source)
        self.Pi = Ops1D(p, c, dt).Pi
        self.tloc = self.mesh.loc[self.target]

    def _lines(self, F, k):
        return np.moveaxis(F, -1 - k, -1)

    def _back(self, F, k):
        return np.moveaxis(F, -1, -1 - k)

    def residual(self, U, t=0.0):
        """Pre-mass residual R = R_vol + R_surf (- W J q) at the target elements."""
        dt, m, g = self.dt, self.mesh, self.gamma
        U = np.asarray(U).astype(dt)
        n = self.n
        T, TL = self.target, self.tloc
        UT = U[:, T]
        S1, w = m.ops.S1, m.ops.w
        wperp = (w[:, None] * w[None, :])[:, :, None]
        R = np.zeros_like(UT)
        for k in range(3):
            Uk = self._lines(UT, k)
            Ck = self._lines(m.C[:, k][:, TL], k)
            N = [(Ck[i][..., :, None] + Ck[i][..., None, :]) / 2 for i in range(3)]
            F = ec_flux(Uk[..., :, None], Uk[..., None, :], N, g, self.variant)
            Rk = np.einsum("ij,...ij->...i", S1, F) * wperp
            R = R + self._back(Rk, k)
        Wf = w[:, None] * w[None, :]
        for k in range(3):
            Rk = np.zeros_like(self._lines(UT, k))
            for side in (-1, 1):
                ao, an = (n - 1, 0) if side > 0 else (0, n - 1)
                nb = m.neighbour_ids(T, k, side)
                Uo = self._lines(UT, k)[..., ao]
                Ub = self._lines(U[:, nb], k)[..., an]
                Co = self._lines(m.C[:, k][:, TL], k)[..., ao]
                Cb = self._lines(m.C[:, k][:, m.loc[nb]], k)[..., an]
                N = [side * (Co[i] + Cb[i]) / 2 for i in range(3)]
                fs = ec_flux(Uo, Ub, N, g, self.variant)
                if self.dissipation == 1:
                    fs = fs + llf(Uo, Ub, N, g)
                elif self.dissipation == 2:
                    fs = fs + roe(Uo, Ub, N, g)
                Rk[..., ao] = Rk[..., ao] + Wf * fs
            R = R + self._back(Rk, k)
        if self.source:
            R = R - m.WJ[TL] * mms_source(m.X[:, TL], t, self.gamma, dt)
        return R

    def apply_inverse_mass(self, R):
        """Pi~_3 (W J)^-1 Pi~_3^T at the target elements, applied direction by
        direction (the tensor product of the 1D projections)."""
        P = self.Pi
        y = R
        for k in range(3):
            y = self._back(self._lines(y, k) @ P, k)        # Pi~^T along k
        y = y / self.mesh.WJ[self.tloc]
        for k in range(3):
            y = self._back(self._lines(y, k) @ P.T, k)      # Pi~ along k
        return y

    def rhs(self, U, t=0.0):
        return -self.apply_inverse_mass(self.residual(U, t))

    def rk4_step(self, U, dt, t=0.0):
        """One classical RK4 step (full meshes only): the four-stage,
        fourth-order scheme of Sec. 7 (opening paragraph)."""
        if self.target.size != self.mesh.E:
            raise ValueError("rk4_step needs the full mesh")
        U = np.asarray(U).astype(self.dt)
        h = self.dt(dt)
        k1 = self.rhs(U, t)
        k2 = self.rhs(U + h / 2 * k1, t + dt / 2)
        k3 = self.rhs(U + h / 2 * k2, t + dt / 2)
        k4 = self.rhs(U + h * k3, t + dt)
        return U + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
