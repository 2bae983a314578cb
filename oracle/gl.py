"""NSFR with an uncollocated volume and surface quadrature (oracle; test
infrastructure only).

Paper: Sec. 3.3 (Eq. NSFR with the hybridised operator of Eq. skew-symm qtilde
oper, the reference two-point flux built from the entropy-projected
conservative variables, and the entropy projection itself), Sec. 4 (Eq. Fr
projection and Eq. weight-adj ESFR mass with the basis evaluated at the
quadrature nodes), Sec. 5 (sum-factorised evaluation: the volume-volume block
acts along lines, the surface-volume blocks couple every volume node of a line
with the two face nodes at the line's ends), Sec. 6.3 (the entropy-projected
variables make the hybrid term reduce to surface entropy potentials) and
Sec. 7 (opening paragraph: Gauss-Legendre (GL) quadrature, the solution
stored in a Lagrange basis on LGL nodes, overintegration = extra quadrature
nodes per direction).

Setting. Solution basis chi: Lagrange polynomials of degree p on the n = p+1
LGL nodes (coefficients = nodal values at the LGL nodes). Volume quadrature:
Nq points per direction (Gauss-Legendre with Nq = n + overintegration, or the
LGL nodes themselves, which gives back the collocated scheme); surface
quadrature: the same 1D rule in the two tangential directions. Flux basis phi:
Lagrange polynomials on the volume quadrature nodes, so that its
differentiation matrix Dq and its values at the element ends tL, tR define
the hybrid operator.

Readings of the paper used here:
  * the L2 projection of the entropy variables is the reference-space
    projection Pi = M^-1 chi^T W (M = chi^T W chi), applied per direction;
  * the metric cofactors are the conservative-curl cofactors of the degree-p
    grid (as on LGL nodes) evaluated as polynomials at the volume and face
    quadrature nodes, and J is the determinant of the grid polynomial's
    derivative there; this keeps the discrete GCL and phi_f C_v = C_f exact;
  * the surface numerical flux at a face quadrature node uses
    N = (C_L n_L - C_R n_R) / 2 and the entropy-projected states of the two
    elements at that node.

The residual returned is the pre-mass vector R (in solution coefficients) with
(M_m + K_m) du/dt + R = 0. Two independent evaluations: ``residual`` (line-wise)
and ``residual_definition`` (dense hybridised operator, small meshes).
"""
import itertools
import math

import torch

from . import flux as fx
from .mesh import Mesh, apply_D
from .operators import (diff_matrix, gauss_legendre, kron3, lagrange_eval, lgl_nodes_weights)

f64 = torch.float64


class GLOperators1D:
    """1D operators of the uncollocated scheme.

    Attributes
    ----------
    x          LGL solution nodes (n)
    xq, wq     volume quadrature nodes and weights (Nq)
    chi        Nq x n: solution basis at the quadrature nodes
    Dq         Nq x Nq: flux-basis differentiation on the quadrature nodes
    Sq         Wq Dq - Dq^T Wq: 1D volume-volume block of (Q~ - Q~^T)
    tL, tR     flux basis at xi = -1, +1 (length Nq)
    M          chi^T Wq chi, the 1D mass of the solution basis
    Pi         M^-1 chi^T Wq: L2 projection onto the solution basis
    D          LGL strong differentiation (n x n); Dp = D^p
    K          c (D^p)^T M (D^p)  (Eq. Km in 1D)
    PiT        (M + K)^-1 chi^T Wq: the ESFR projection of Eq. Fr projection
    """

    def __init__(self, p, c=0.0, quad="gl", overint=0):
        self.p, self.n, self.c = p, p + 1, float(c)
        self.x, self.w = lgl_nodes_weights(p)
        if quad == "gl":
            self.xq, self.wq = gauss_legendre(self.n + int(overint))
        elif quad == "lgl":
            if overint:
                raise ValueError("overintegration is defined for the GL rule")
            self.xq, self.wq = self.x.clone(), self.w.clone()
        else:
            raise ValueError(quad)
        self.quad, self.overint = quad, int(overint)
        self.nq = self.xq.numel()
        self.chi = lagrange_eval(self.x, self.xq)
        self.Wq = torch.diag(self.wq)
        self.Dq = diff_matrix(self.xq)
        self.Sq = self.Wq @ self.Dq - self.Dq.T @ self.Wq
        ends = torch.tensor([-1.0, 1.0], dtype=f64)
        T = lagrange_eval(self.xq, ends)
        self.tL, self.tR = T[0].clone(), T[1].clone()
        self.M = self.chi.T @ self.Wq @ self.chi
        self.Pi = torch.linalg.solve(self.M, self.chi.T @ self.Wq)
        self.D = diff_matrix(self.x)
        self.Dp = torch.linalg.matrix_power(self.D, p)
        self.K = self.c * self.Dp.T @ self.M @ self.Dp
        self.PiT = torch.linalg.solve(self.M + self.K, self.chi.T @ self.Wq)


def apply_1d(A, F, axis):
    """Apply the (m x n) matrix A along one reference direction of (..., n, n, n):
    axis 0 = xi (last dim), 1 = eta, 2 = zeta; that dim becomes m."""
    if axis == 0:
        return torch.einsum("ij,...cbj->...cbi", A, F)
    if axis == 1:
        return torch.einsum("ij,...cja->...cia", A, F)
    return torch.einsum("ij,...jba->...iba", A, F)


def apply_3(Ax, Ay, Az, F):
    """Tensor-product operator Az (x) Ay (x) Ax on (..., nz, ny, nx), one direction
    at a time (sum factorisation, Eq. sum-factorization)."""
    return apply_1d(Az, apply_1d(Ay, apply_1d(Ax, F, 0), 1), 2)


def face_slab(F, k, side):
    """The (..., n, n) slab of nodal coefficients on the face (k, side): on the
    LGL basis the solution at xi_k = +-1 is the end node's coefficient."""
    n = F.shape[-1]
    idx = n - 1 if side > 0 else 0
    if k == 0:
        return F[..., :, :, idx]
    if k == 1:
        return F[..., :, idx, :]
    return F[..., idx, :, :]


def slab_interp(A, S):
    """Interpolate a face slab (..., t2, t1) with A in both tangential directions."""
    return torch.einsum("ij,kl,...lj->...ki", A, A, S)


def slab_interp_T(A, S):
    return torch.einsum("ji,lk,...lj->...ki", A, A, S)


def _line_last(F, k):
    return F.movedim(-1 - k, -1)


def _line_back(F, k):
    return F.movedim(-1, -1 - k)


def conservative_from_entropy(V, gamma):
    """Inverse of the entropy-variable map of Sec. 2.1 (U = -rho s / (gamma - 1)):
    beta = -v5 / 2, u = v_{2..4} / (2 beta), s = gamma - (gamma - 1)(v1 + beta |u|^2),
    ln p = (s + gamma ln(2 beta)) / (1 - gamma), rho = 2 beta p."""
    beta = -0.5 * V[4]
    vel = [V[1] / (2 * beta), V[2] / (2 * beta), V[3] / (2 * beta)]
    q2 = vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2
    s = gamma - (gamma - 1.0) * (V[0] + beta * q2)
    p = torch.exp((s + gamma * torch.log(2 * beta)) / (1.0 - gamma))
    rho = 2 * beta * p
    return fx.conservative(rho, vel, p, gamma)


class GLMesh:
    """Metric terms of the warped mesh at the quadrature nodes.

    Builds the LGL mesh of oracle.mesh (grid of degree p at the LGL nodes,
    conservative-curl cofactors there) and evaluates the polynomials at the
    volume quadrature nodes (Cq, Jq) and at the face quadrature nodes
    (Cf[k][side]: the column k of the cofactor matrix on the faces normal to k)."""

    def __init__(self, p, ne, ops, lo=0.0, hi=2 * math.pi, beta=0.0, l=None):
        self.base = Mesh(p, ne, lo, hi, beta, l)
        b = self.base
        self.p, self.n, self.nq, self.E, self.ne = p, p + 1, ops.nq, b.E, b.ne
        self.lo, self.hi = b.lo, b.hi
        chi = ops.chi
        self.X = b.X
        self.Xq = apply_3(chi, chi, chi, b.X)
        self.Cq = apply_3(chi, chi, chi, b.C)                 # (3 comp, 3 dir, E, nq, nq, nq)
        G = [[apply_3(chi, chi, chi, apply_D(b.ops.D, b.X[m], j)) for j in range(3)] for m in range(3)]
        self.Jq = (G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1])
                   - G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0])
                   + G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]))
        wq = ops.wq
        self.W3q = (wq[None, None, :] * wq[None, :, None] * wq[:, None, None]).expand_as(self.Jq[0])
        self.WJq = self.W3q * self.Jq
        self.Cf = [{s: slab_interp(chi, face_slab(b.C[:, k], k, s)) for s in (-1, 1)} for k in range(3)]

    def neighbor(self, F, axis, side, trailing=2):
        """Field of the periodic neighbour across face (axis, side) for arrays
        (..., E, <trailing dims>): neighbor(F, 0, +1)[e] = F[e + 1 in x]."""
        shp = F.shape
        ed = F.dim() - trailing - 1
        nx, ny, nz = self.ne
        G = F.reshape(*shp[:ed], nz, ny, nx, *shp[ed + 1:])
        G = torch.roll(G, shifts=-side, dims=ed + (2 - axis))
        return G.reshape(shp)


def entropy_projection(ops, U, gamma):
    """Entropy-projected variables (Sec. 3.3): interpolate u to the volume
    quadrature nodes, evaluate v there, project onto the solution basis (v^),
    interpolate v^ to the volume and face quadrature nodes and map back.
    Returns (v^, u~ at volume nodes, {(k, side): u~ at face nodes})."""
    chi, Pi = ops.chi, ops.Pi
    uq = apply_3(chi, chi, chi, U)
    vq = fx.entropy_variables(uq, gamma)
    vhat = apply_3(Pi, Pi, Pi, vq)
    vv = apply_3(chi, chi, chi, vhat)
    uv = conservative_from_entropy(vv, gamma)
    uf = {}
    for k in range(3):
        for s in (-1, 1):
            uf[(k, s)] = conservative_from_entropy(slab_interp(chi, face_slab(vhat, k, s)), gamma)
    return vhat, uv, uf


def _scatter_slab(R, k, side, S):
    n = R.shape[-1]
    idx = n - 1 if side > 0 else 0
    if k == 0:
        R[..., :, :, idx] += S
    elif k == 1:
        R[..., :, idx, :] += S
    else:
        R[..., idx, :, :] += S


def surface_fluxes(gm, ops, uf, gamma, two_point, dissipation=None):
    """n^r . f* at the face quadrature nodes of every face (k, side), with the
    neighbour's entropy-projected state across the face."""
    out = {}
    for k in range(3):
        for s in (-1, 1):
            ub = gm.neighbor(uf[(k, -s)], k, s)
            Cb = gm.neighbor(gm.Cf[k][-s], k, s)
            Co = gm.Cf[k][s]
            N = [s * 0.5 * (Co[i] + Cb[i]) for i in range(3)]
            f = two_point(uf[(k, s)], ub, N)
            if dissipation is not None:
                f = f + dissipation(uf[(k, s)], ub, N)
            out[(k, s)] = f
    return out


def residual(gm, ops, U, gamma, variant=0, dissipation=False, two_point=None):
    """Pre-mass residual R in solution coefficients, line-wise form:
    R = chi_v^T R_v + sum_f chi_f^T R_f with, per direction k,
      R_v[a] += sum_b Sq[a, b] w_perp F(u~_a, u~_b)
                + w_perp (tR[a] F(u~_a, u~_fR) - tL[a] F(u~_a, u~_fL)),
      R_fR   -= w_perp sum_a tR[a] F(u~_fR, u~_a),
      R_fL   += w_perp sum_a tL[a] F(u~_fL, u~_a),
    F(x, y) = f_s(x, y) . (C(x) + C(y)) / 2 with column k of C, and
      R_f    += w_perp n^r . f*   (the surface term of Eq. NSFR)."""
    tp = two_point or (lambda a, b, N: fx.ec_flux(a, b, N, gamma, variant))
    diss = fx.surface_dissipation(dissipation, gamma)
    _, uv, uf = entropy_projection(ops, U, gamma)
    wq = ops.wq
    wperp = wq[:, None] * wq[None, :]                 # tangential weights (t2, t1)
    Rv = torch.zeros_like(uv)
    Rf = {key: torch.zeros_like(val) for key, val in uf.items()}
    for k in range(3):
        uk = _line_last(uv, k)                        # (5, E, t2, t1, a)
        Ck = _line_last(gm.Cq[:, k], k)               # (3, E, t2, t1, a)
        Na = [0.5 * (Ck[i][..., :, None] + Ck[i][..., None, :]) for i in range(3)]
        F = tp(uk[..., :, None], uk[..., None, :], Na)
        Rk = torch.einsum("ij,...ij->...i", ops.Sq, F) * wperp[..., None]
        for s, t in ((1, ops.tR), (-1, ops.tL)):
            ufs = uf[(k, s)][..., None]               # (5, E, t2, t1, 1)
            Cfs = gm.Cf[k][s][..., None]
            N = [0.5 * (Ck[i] + Cfs[i]) for i in range(3)]
            Fvf = tp(uk, ufs, N)                       # F(u~_a, u~_f)
            Rk = Rk + s * t * Fvf * wperp[..., None]
            Ffv = tp(ufs, uk, N)                       # F(u~_f, u~_a)
            Rf[(k, s)] = Rf[(k, s)] - s * torch.einsum("a,...a->...", t, Ffv) * wperp
        Rv = Rv + _line_back(Rk, k)
    fst = surface_fluxes(gm, ops, uf, gamma, tp, diss)
    chi = ops.chi
    R = apply_3(chi.T, chi.T, chi.T, Rv)
    for (k, s), fs in fst.items():
        _scatter_slab(R, k, s, slab_interp_T(chi, Rf[(k, s)] + wperp * fs))
    return R


# ---------------------------------------------------------------------------
# Definition form: the dense hybridised operator
# ---------------------------------------------------------------------------

def _face_points(nq):
    """Face quadrature points as (k, side, [(volume index along k's line,
    tangential (t1, t2))]) in the order t2 slow, t1 fast."""
    faces = []
    for k in range(3):
        for side in (-1, 1):
            faces.append((k, side, [(t1, t2) for t2 in range(nq) for t1 in range(nq)]))
    return faces


def _vol_index(nq, k, a, t1, t2):
    """Volume quadrature node index (xi fastest) of position a on the k-line with
    tangential indices (t1, t2) in increasing direction order."""
    if k == 0:
        i, j, l = a, t1, t2
    elif k == 1:
        i, j, l = t1, a, t2
    else:
        i, j, l = t1, t2, a
    return i + nq * j + nq * nq * l


def hybrid_operators(ops):
    """Dense Q~_k - Q~_k^T (Eq. skew-symm qtilde oper), k = 1..3, of size
    (Nq^3 + 6 Nq^2)^2: volume-volume block Wq3 Dq_k - Dq_k^T Wq3, volume-face
    block phi(xi_f)^T W_f diag(n^r_f), face-volume block its negative
    transpose, face-face block 0. Also returns the face-point weights."""
    nq = ops.nq
    I = torch.eye(nq, dtype=f64)
    Dk = [kron3(I, I, ops.Dq), kron3(I, ops.Dq, I), kron3(ops.Dq, I, I)]
    W3 = torch.diag(kron3(ops.Wq, ops.Wq, ops.Wq).diagonal())
    faces = _face_points(nq)
    Nv = nq ** 3
    Nt = Nv + sum(len(f[2]) for f in faces)
    Qs = []
    for k in range(3):
        Q = torch.zeros(Nt, Nt, dtype=f64)
        Q[:Nv, :Nv] = W3 @ Dk[k] - Dk[k].T @ W3
        col = Nv
        for (kf, side, pts) in faces:
            t = ops.tR if side > 0 else ops.tL
            for (t1, t2) in pts:
                if kf == k:
                    wf = float(ops.wq[t1] * ops.wq[t2])
                    for a in range(nq):
                        v = _vol_index(nq, kf, a, t1, t2)
                        Q[v, col] += float(t[a]) * wf * side     # phi(xi_f)^T W_f n_f
                        Q[col, v] -= float(t[a]) * wf * side     # -W_f n_f phi(xi_f)
                col += 1
        Qs.append(Q)
    return Qs, faces


def chi_face(ops, k, side):
    """Dense Nq^2 x n^3 matrix: the solution basis at the face quadrature points of
    face (k, side), points ordered t2 slow, t1 fast."""
    n = ops.n
    e = torch.zeros(1, n, dtype=f64)
    e[0, n - 1 if side > 0 else 0] = 1.0
    chi = ops.chi
    if k == 0:
        return kron3(chi, chi, e)
    if k == 1:
        return kron3(chi, e, chi)
    return kron3(e, chi, chi)


def residual_definition(gm, ops, U, gamma, variant=0, dissipation=False, two_point=None):
    """Pre-mass residual from the dense hybridised form of Eq. NSFR:
    R = [chi_v^T chi_f^T][(Q~ - Q~^T) o F^r] 1 + sum_f chi_f^T W_f n^r . f*,
    with every state, cofactor and projection formed by dense matrices. Small
    meshes only (memory grows as E (Nq^3 + 6 Nq^2)^2)."""
    tp = two_point or (lambda a, b, N: fx.ec_flux(a, b, N, gamma, variant))
    diss = fx.surface_dissipation(dissipation, gamma)
    n, nq, E = ops.n, ops.nq, gm.E
    chi3 = kron3(ops.chi, ops.chi, ops.chi)            # Nq^3 x n^3
    Pi3 = kron3(ops.Pi, ops.Pi, ops.Pi)                # n^3 x Nq^3
    Uf = U.reshape(5, E, n ** 3)
    vq = fx.entropy_variables(torch.einsum("qi,sei->seq", chi3, Uf), gamma)
    vhat = torch.einsum("iq,seq->sei", Pi3, vq)
    Qs, faces = hybrid_operators(ops)
    Xf = [chi_face(ops, k, s) for (k, s, _) in faces]
    chit = torch.cat([chi3] + Xf)                      # (Nt, n^3): [chi_v; chi_f]
    ut = conservative_from_entropy(torch.einsum("ti,sei->set", chit, vhat), gamma)
    Cn = gm.base.C.reshape(3, 3, E, n ** 3)
    H = torch.zeros(5, E, chit.shape[0], dtype=U.dtype)
    for k in range(3):
        Ct = torch.einsum("ti,cei->cet", chit, Cn[:, k])
        N = [0.5 * (Ct[i][:, :, None] + Ct[i][:, None, :]) for i in range(3)]
        F = tp(ut[:, :, :, None], ut[:, :, None, :], N)
        H = H + torch.einsum("ij,seij->sei", Qs[k], F)
    R = torch.einsum("ti,set->sei", chit, H)
    # surface term with the neighbour's face state and cofactor (dense per face)
    nv = nq ** 3
    off = nv
    for (k, s, pts), X in zip(faces, Xf):
        m = len(pts)
        uo = ut[:, :, off:off + m]
        Co = torch.einsum("ti,cei->cet", X, Cn[:, k])
        # neighbour across (k, s): its face (k, -s), same point order
        Xn = chi_face(ops, k, -s)
        vn = gm.neighbor(vhat, k, s, trailing=1)
        ub = conservative_from_entropy(torch.einsum("ti,sei->set", Xn, vn), gamma)
        Cb = torch.einsum("ti,cei->cet", Xn, gm.neighbor(Cn[:, k], k, s, trailing=1))
        N = [s * 0.5 * (Co[i] + Cb[i]) for i in range(3)]
        f = tp(uo, ub, N)
        if diss is not None:
            f = f + diss(uo, ub, N)
        wf = torch.tensor([float(ops.wq[t1] * ops.wq[t2]) for (t1, t2) in pts], dtype=f64)
        R = R + torch.einsum("ti,set->sei", X, f * wf)
        off += m
    return R.reshape_as(U)


# ---------------------------------------------------------------------------
# Mass inverses
# ---------------------------------------------------------------------------

def wa_apply(gm, ops, R):
    """A R with A = Pi~3 (Wq J)^-1 Pi~3^T (Eq. weight-adj ESFR mass with the
    basis at the quadrature nodes), sum-factorised."""
    P = ops.PiT
    y = apply_3(P.T, P.T, P.T, R)
    y = y / gm.WJq
    return apply_3(P, P, P, y)


def modified_mass(gm, ops):
    """Dense M_m + K_m per element: M_m = chi_v^T Wq J chi_v and K_m of Eq. Km."""
    n, p, E = ops.n, ops.p, gm.E
    chi3 = kron3(ops.chi, ops.chi, ops.chi)
    WJ = gm.WJq.reshape(E, -1)
    Mm = torch.einsum("qi,eq,qj->eij", chi3, WJ, chi3)
    I = torch.eye(n, dtype=f64)
    MK = Mm.clone()
    for s, v, w in itertools.product((0, p), repeat=3):
        if s + v + w == 0:
            continue
        csvw = ops.c ** ((s + v + w) / p)
        Dsvw = kron3(ops.Dp if w else I, ops.Dp if v else I, ops.Dp if s else I)
        MK = MK + csvw * Dsvw.T @ Mm @ Dsvw
    return MK


def exact_apply(gm, ops, R):
    MK = modified_mass(gm, ops)
    E, Nv = gm.E, ops.n ** 3
    L = torch.linalg.cholesky(MK)
    X = torch.cholesky_solve(R.reshape(5, E, Nv).permute(1, 2, 0), L)
    return X.permute(2, 0, 1).reshape_as(R)


class GLScheme:
    """du/dt = -A R for the uncollocated NSFR scheme (weight-adjusted or exact
    inverse of the FR-modified mass)."""

    def __init__(self, p, ne, lo=0.0, hi=2 * math.pi, beta=0.0, l=None, gamma=1.4, c=0.0, variant=0,
                 dissipation=False, quad="gl", overint=0, mass="wa", source=False):
        self.ops = GLOperators1D(p, c, quad, overint)
        self.mesh = GLMesh(p, ne, self.ops, lo, hi, beta, l)
        self.p, self.gamma, self.c = p, float(gamma), float(c)
        self.variant, self.dissipation, self.mass, self.source = variant, dissipation, mass, bool(source)

    @property
    def X(self):
        return self.mesh.X

    def residual(self, U, t=0.0, definition=False):
        f = residual_definition if definition else residual
        R = f(self.mesh, self.ops, U, self.gamma, self.variant, self.dissipation)
        if self.source:
            from .problems import mms_source
            chi = self.ops.chi
            q = mms_source(self.mesh.Xq, t, self.gamma)
            R = R - apply_3(chi.T, chi.T, chi.T, self.mesh.WJq * q)
        return R

    def rhs(self, U, t=0.0, definition=False):
        R = self.residual(U, t, definition)
        if self.mass == "wa":
            return -wa_apply(self.mesh, self.ops, R)
        return -exact_apply(self.mesh, self.ops, R)

    def projected_entropy_variables(self, U):
        return entropy_projection(self.ops, U, self.gamma)[0]
