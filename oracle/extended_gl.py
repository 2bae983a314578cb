"""NSFR on Gauss-Legendre and overintegrated quadrature, evaluated in extended
precision (oracle; test infrastructure only).

The round-off reference for the uncollocated scheme, as oracle.extended is for
the collocated one: numpy's long double (64-bit significand), a coding of its
own (numpy, its own Gauss-Legendre rule and dense solver), independent of the
PyTorch oracle in oracle.gl. It follows the same definitions:
  * Sec. 7 (opening paragraph): solution stored as values at the n = p + 1
    LGL nodes, volume rule Gauss-Legendre with q = n + overintegration points
    per direction, surface rule the same 1D rule in the tangential directions;
  * Sec. 3.3: entropy projection v^ = Pi v(chi u) with the reference-space L2
    projection Pi = M^-1 chi^T W, entropy-projected states u~ = u(chi v^) at
    the volume and face points, the hybridised operator of Eq. skew-symm
    qtilde oper (volume-volume block W Dq - Dq^T W per direction,
    surface-volume blocks t_L, t_R at the two ends of every line), the surface
    numerical flux with N = (C_L n_L - C_R n_R) / 2 and optional dissipation;
  * Sec. 4: dU/dt = -Pi~_3 (W J)^-1 Pi~_3^T R with Pi~ = (M + K)^-1 chi^T W
    (Eq. weight-adj ESFR mass, Eq. Fr projection at the quadrature points);
  * metric terms: the degree-p grid and its conservative-curl cofactors at the
    LGL nodes (oracle.extended.MeshX), evaluated as polynomials at the
    quadrature points; J the determinant of the interpolated grid derivative.

Layout as in the other oracles: state (5, E, n, n, n) indexed [s, e, c, b, a]
with a the xi index."""
import numpy as np

from .extended import (LD, MeshX, Ops1D, _entropy_vars, _legendre, _pi, _solve, ec_flux, llf, mms_source, primitives,
                       roe)


def gauss_legendre_x(q, dt=LD):
    """Gauss-Legendre nodes and weights on [-1, 1] in type dt: roots of P_q by
    Newton from the Chebyshev-like guesses cos(pi (i + 3/4) / (q + 1/2)),
    weights 2 / ((1 - x^2) P_q'(x)^2), P_q' = q (x P_q - P_{q-1}) / (x^2 - 1)."""
    pi = _pi(dt)
    x = -np.cos(pi * (np.arange(q, dtype=dt) + dt(0.75)) / (dt(q) + dt(0.5)))
    for _ in range(200):
        P, Pm = _legendre(q, x)
        dP = q * (x * P - Pm) / (x * x - 1)
        dx = P / dP
        x = x - dx
        if float(np.max(np.abs(dx))) < 1e-21:
            break
    x = (x - x[::-1]) / 2
    P, Pm = _legendre(q, x)
    dP = q * (x * P - Pm) / (x * x - 1)
    w = dt(2) / ((1 - x * x) * dP * dP)
    return x, (w + w[::-1]) / 2


def lagrange_matrix(nodes, pts):
    """L[i, j] = l_j(pts[i]) for the Lagrange basis on nodes (product form)."""
    n = nodes.size
    L = np.ones((pts.size, n), dtype=nodes.dtype)
    for j in range(n):
        for k in range(n):
            if k != j:
                L[:, j] = L[:, j] * (pts - nodes[k]) / (nodes[j] - nodes[k])
    return L


def lagrange_derivative(nodes):
    """Dq[i, j] = l_j'(nodes[i]) (barycentric form)."""
    n = nodes.size
    lam = np.array([1 / np.prod([nodes[j] - nodes[k] for k in range(n) if k != j]) for j in range(n)],
                   dtype=nodes.dtype)
    D = np.zeros((n, n), dtype=nodes.dtype)
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (nodes[i] - nodes[j])
        D[i, i] = -sum(D[i, j] for j in range(n) if j != i)
    return D


class GLOps1DX:
    """1D operators of the uncollocated scheme in type dt."""

    def __init__(self, p, q, c=0.0, dt=LD):
        base = Ops1D(p, 0.0, dt)
        self.p, self.n, self.q = p, p + 1, q
        self.x = base.x
        self.xq, self.wq = gauss_legendre_x(q, dt)
        self.chi = lagrange_matrix(self.x, self.xq)                  # q x n
        W = np.diag(self.wq)
        M = self.chi.T @ W @ self.chi
        self.Pi = _solve(M, self.chi.T @ W)                         # n x q
        Dp = np.eye(self.n, dtype=dt)
        for _ in range(p):
            Dp = Dp @ base.D
        K = dt(c) * (Dp.T @ M @ Dp)
        self.PiT = _solve(M + K, self.chi.T @ W)
        Dq = lagrange_derivative(self.xq)
        self.Sq = W @ Dq - Dq.T @ W
        T = lagrange_matrix(self.xq, np.array([-1, 1], dtype=dt))
        self.tL, self.tR = T[0], T[1]


def _along(A, F, axis):
    """Apply the matrix A along reference direction axis (0 = xi = last dim)."""
    G = np.moveaxis(F, -1 - axis, -1) @ A.T
    return np.moveaxis(G, -1, -1 - axis)


def _tensor(A, F):
    return _along(A, _along(A, _along(A, F, 0), 1), 2)


def _slab(F, k, side):
    """Face slab (..., t2, t1) of nodal values on face (k, side)."""
    idx = -1 if side > 0 else 0
    return F[..., idx] if k == 0 else (F[..., idx, :] if k == 1 else F[..., idx, :, :])


def _slab_interp(A, S):
    return np.einsum("ij,kl,...lj->...ki", A, A, S)


def conservative_from_entropy(V, gamma):
    beta = -V[4] / 2
    u, v, w = V[1] / (2 * beta), V[2] / (2 * beta), V[3] / (2 * beta)
    q2 = u * u + v * v + w * w
    s = gamma - (gamma - 1) * (V[0] + beta * q2)
    p = np.exp((s + gamma * np.log(2 * beta)) / (1 - gamma))
    rho = 2 * beta * p
    return np.stack([rho, rho * u, rho * v, rho * w, p / (gamma - 1) + rho * q2 / 2])


class GLSchemeX:
    """Residual and right-hand side of the uncollocated scheme in type dt.

    elements: optional global element ids at which to evaluate (a sample of a
    large mesh); outputs then have shape (5, len(elements), n, n, n)."""

    def __init__(self, p, ne, lo=0.0, hi=None, beta=0.0, l=None, gamma=1.4, c=0.0, variant=0,
                 dissipation=0, source=False, overint=0, dt=LD, elements=None):
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
        m = MeshX(p, ne, lo, hi, beta, l, dt, elements=ids)
        self.mesh = m
        self.p, self.n = p, p + 1
        self.ops = o = GLOps1DX(p, p + 1 + int(overint), c, dt)
        self.gamma = dt(gamma)
        self.variant, self.dissipation, self.source = variant, int(dissipation), bool(source)
        chi = o.chi
        self.Cq = _tensor(chi, m.C)                                       # (3 comp, 3 dir, E', q, q, q)
        G = [[_tensor(chi, _along(m.ops.D, m.X[a], j)) for j in range(3)] for a in range(3)]
        Jq = (G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1])
              - G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0])
              + G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]))
        wq = o.wq
        self.WJq = (wq[None, None, None, :] * wq[None, None, :, None] * wq[None, :, None, None]) * Jq
        self.Xq = _tensor(chi, m.X)
        self.Cf = {(k, s): _slab_interp(chi, _slab(m.C[:, k], k, s)) for k in range(3) for s in (-1, 1)}
        self.tloc = m.loc[self.target]

    def _project(self, U):
        """v^ and the entropy-projected states at the volume and face points,
        for every element the mesh holds."""
        o, g = self.ops, self.gamma
        vq = _entropy_vars(_tensor(o.chi, U), g)
        vhat = _tensor(o.Pi, vq)
        uv = conservative_from_entropy(_tensor(o.chi, vhat), g)
        uf = {(k, s): conservative_from_entropy(_slab_interp(o.chi, _slab(vhat, k, s)), g)
              for k in range(3) for s in (-1, 1)}
        return vhat, uv, uf

    def projected_entropy_variables(self, U):
        U = np.asarray(U).astype(self.dt)[:, self.mesh.ids]
        return self._project(U)[0][:, self.tloc]

    def _two_point(self, a, b, N):
        return ec_flux(a, b, N, self.gamma, self.variant)

    def residual(self, U, t=0.0):
        """Pre-mass residual R (in solution coefficients) at the target elements."""
        m, o, g = self.mesh, self.ops, self.gamma
        U = np.asarray(U).astype(self.dt)[:, m.ids]
        _, uv, uf = self._project(U)
        TL = self.tloc
        uv = uv[:, TL]
        wq = o.wq
        wperp = wq[:, None] * wq[None, :]
        Rv = np.zeros_like(uv)
        Rf = {}
        for k in range(3):
            uk = np.moveaxis(uv, -1 - k, -1)
            Ck = np.moveaxis(self.Cq[:, k][:, TL], -1 - k, -1)
            N = [(Ck[i][..., :, None] + Ck[i][..., None, :]) / 2 for i in range(3)]
            F = self._two_point(uk[..., :, None], uk[..., None, :], N)
            Rk = np.einsum("ij,...ij->...i", o.Sq, F) * wperp[..., None]
            for s, tv in ((1, o.tR), (-1, o.tL)):
                ufs = uf[(k, s)][:, TL][..., None]
                Cfs = self.Cf[(k, s)][:, TL][..., None]
                N = [(Ck[i] + Cfs[i]) / 2 for i in range(3)]
                F = self._two_point(uk, ufs, N)
                Rk = Rk + s * tv * F * wperp[..., None]
                # surface-volume block of the face rows: -s t . F, plus the
                # numerical flux with the neighbour's face point
                nb = m.loc[m.neighbour_ids(self.target, k, s)]
                ub = uf[(k, -s)][:, nb]
                Cb = self.Cf[(k, -s)][:, nb]
                Co = self.Cf[(k, s)][:, TL]
                Ns = [s * (Co[i] + Cb[i]) / 2 for i in range(3)]
                uo = uf[(k, s)][:, TL]
                fs = self._two_point(uo, ub, Ns)
                if self.dissipation == 1:
                    fs = fs + llf(uo, ub, Ns, g)
                elif self.dissipation == 2:
                    fs = fs + roe(uo, ub, Ns, g)
                Rf[(k, s)] = (fs - s * np.einsum("a,...a->...", tv, F)) * wperp
            Rv = Rv + np.moveaxis(Rk, -1, -1 - k)
        if self.source:
            Rv = Rv - self.WJq[TL] * mms_source(self.Xq[:, TL], t, g, self.dt)
        R = _tensor(o.chi.T, Rv)
        for (k, s), S in Rf.items():
            add = np.einsum("ji,lk,...lj->...ki", o.chi, o.chi, S)
            idx = -1 if s > 0 else 0
            if k == 0:
                R[..., idx] += add
            elif k == 1:
                R[..., idx, :] += add
            else:
                R[..., idx, :, :] += add
        return R

    def apply_inverse_mass(self, R):
        P = self.ops.PiT
        y = _tensor(P.T, R)
        y = y / self.WJq[self.tloc]
        return _tensor(P, y)

    def rhs(self, U, t=0.0):
        return -self.apply_inverse_mass(self.residual(U, t))


# ---------------------------------------------------------------------------
# Conservative strong DG on the same rule (Sec. 3.1 Eq. cons DG strong) with
# Roe's flux (Sec. 7.4): the baseline of the paper's cost comparison
# ---------------------------------------------------------------------------

def physical_flux(U, gamma):
    """f_k(U), shape (3, 5, ...)."""
    rho, vel, p, _ = primitives(U, gamma)
    out = []
    for k in range(3):
        f = [U[0] * vel[k], U[1] * vel[k], U[2] * vel[k], U[3] * vel[k], (U[4] + p) * vel[k]]
        f[1 + k] = f[1 + k] + p
        out.append(np.stack(f))
    return np.stack(out)


def roe_flux(Ua, Ub, N, gamma):
    """Roe's flux N . f* = (f_a + f_b) . N / 2 - |N| |A^| (U_b - U_a) / 2 with
    |A^| dU written as the sum over the acoustic, entropy and shear waves at
    Roe's sqrt(rho)-weighted average."""
    ra, va, pa, _ = primitives(Ua, gamma)
    rb, vb, pb, _ = primitives(Ub, gamma)
    nn = np.sqrt(N[0] ** 2 + N[1] ** 2 + N[2] ** 2)
    n = [N[k] / nn for k in range(3)]
    sa, sb = np.sqrt(ra), np.sqrt(rb)
    u = [(sa * va[k] + sb * vb[k]) / (sa + sb) for k in range(3)]
    H = (sa * (Ua[4] + pa) / ra + sb * (Ub[4] + pb) / rb) / (sa + sb)
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    c2 = (gamma - 1) * (H - q2 / 2)
    c = np.sqrt(c2)
    rho = sa * sb
    un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2]
    du = [vb[k] - va[k] for k in range(3)]
    dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2]
    dp = pb - pa
    one = np.ones_like(rho)
    waves = []
    for sg in (-1, 1):
        waves.append(((dp + sg * rho * c * dun) / (2 * c2) * np.abs(un + sg * c),
                      [one, u[0] + sg * c * n[0], u[1] + sg * c * n[1], u[2] + sg * c * n[2], H + sg * c * un]))
    waves.append(((rb - ra - dp / c2) * np.abs(un), [one, u[0], u[1], u[2], q2 / 2]))
    D = np.zeros_like(Ua)
    for a, r in waves:
        for i in range(5):
            D[i] = D[i] + a * r[i]
    b = rho * np.abs(un)
    for k in range(3):
        D[1 + k] = D[1 + k] + b * (du[k] - dun * n[k])
    D[4] = D[4] + b * (u[0] * du[0] + u[1] * du[1] + u[2] * du[2] - un * dun)
    fa, fb = physical_flux(Ua, gamma), physical_flux(Ub, gamma)
    return sum((fa[k] + fb[k]) * N[k] for k in range(3)) / 2 - nn * D / 2


class DGSchemeX(GLSchemeX):
    """Conservative strong DG with Roe's flux on the Gauss-Legendre rule, in
    type dt (same mesh, operators, sampling and mass inverse as GLSchemeX)."""

    def __init__(self, p, ne, lo=0.0, hi=None, beta=0.0, l=None, gamma=1.4, c=0.0, source=False, overint=0,
                 dt=LD, elements=None):
        super().__init__(p, ne, lo=lo, hi=hi, beta=beta, l=l, gamma=gamma, c=c, source=source, overint=overint,
                         dt=dt, elements=elements)
        self.Dq = lagrange_derivative(self.ops.xq)

    def residual(self, U, t=0.0):
        m, o, g = self.mesh, self.ops, self.gamma
        U = np.asarray(U).astype(self.dt)[:, m.ids]
        TL = self.tloc
        UT = U[:, TL]
        F = physical_flux(_tensor(o.chi, UT), g)
        wq = o.wq
        wperp = wq[:, None] * wq[None, :]
        uf = {(k, s): _slab_interp(o.chi, _slab(U, k, s)) for k in range(3) for s in (-1, 1)}
        Rv = np.zeros_like(F[0])
        Rf = {}
        for k in range(3):
            Ck = self.Cq[:, k][:, TL]
            fr = sum(Ck[mm][None] * F[mm] for mm in range(3))
            Fk = np.moveaxis(fr, -1 - k, -1)
            Rk = (Fk @ self.Dq.T) * wq * wperp[..., None]
            Rv = Rv + np.moveaxis(Rk, -1, -1 - k)
            for s, tv in ((1, o.tR), (-1, o.tL)):
                nb = m.loc[m.neighbour_ids(self.target, k, s)]
                Co = self.Cf[(k, s)][:, TL]
                Cb = self.Cf[(k, -s)][:, nb]
                Ns = [s * (Co[i] + Cb[i]) / 2 for i in range(3)]
                fs = roe_flux(uf[(k, s)][:, TL], uf[(k, -s)][:, nb], Ns, g)
                Rf[(k, s)] = (fs - s * np.einsum("a,...a->...", tv, Fk)) * wperp
        if self.source:
            Rv = Rv - self.WJq[TL] * mms_source(self.Xq[:, TL], t, g, self.dt)
        R = _tensor(o.chi.T, Rv)
        for (k, s), S in Rf.items():
            add = np.einsum("ji,lk,...lj->...ki", o.chi, o.chi, S)
            idx = -1 if s > 0 else 0
            if k == 0:
                R[..., idx] += add
            elif k == 1:
                R[..., idx, :] += add
            else:
                R[..., idx, :, :] += add
        return R
