"""Conservative DG in strong form on Gauss-Legendre (optionally overintegrated)
quadrature: the baseline scheme the paper compares NSFR against (oracle; test
infrastructure only).

Paper: Sec. 3.1 (Eq. variational weak DG, and after discrete integration by
parts, Eq. cons DG strong, with M_m = chi^T W J chi), Sec. 7.4 (the
comparison: the same GL quadrature and curvilinear TGV, Roe's surface
numerical flux for DG, an overintegrated DG variant), Sec. 4 (the mass
inverse approximated in weight-adjusted form for every scheme).

Eq. cons DG strong, written out for one element:

    R = chi_v^T W sum_k Dphi_k f^r_k
        + sum_f sum_fk chi(xi_fk)^T W_fk [n^r . f^{*,r} - n^r . phi(xi_fk) f^r]

  * u at the volume points is the interpolated solution chi u^ (no entropy
    projection), f^r_k = sum_m C_mk f_m(u) the contravariant flux with the
    cofactors evaluated at the points (the same metric terms as oracle.gl);
  * the flux basis phi is Lagrange on the volume quadrature points
    (collocated, so its projection is the identity), Dphi_k its derivative
    along k, and n^r . phi(xi_fk) f^r = +-(t_R or t_L) . (f^r_k on the line);
  * n^r . f^{*,r} = N . f*(u_own, u_nb) at the face point with
    N = (C_L n_L - C_R n_R) / 2 (reading shared with oracle.gl) and u the
    interpolated face states of the two elements; f* is Roe's flux
    (`flux.roe_flux`) by default.

Readings:
  * "overintegrated by 2(p+1)" (Sec. 7.4) is read as a rule of 2(p+1) points
    per direction (overint = p + 1);
  * the DG mass inverse is the same weight-adjusted form Pi~ (W J)^-1 Pi~^T
    as NSFR's (c = 0 gives DG; the paper notes the cost is the same for c_+).

Two evaluations: ``residual`` (line-wise) and ``residual_definition``
(dense matrices, small meshes). The residual returned is R with
(M_m + K_m) du/dt + R = 0."""
import math

import torch

from . import flux as fx
from .gl import (GLMesh, GLOperators1D, _scatter_slab, apply_3, face_slab, kron3, slab_interp, slab_interp_T,
                 wa_apply, _face_points, chi_face)

f64 = torch.float64


def contravariant_flux(Cq, F, k):
    """f^r_k = sum_m C[m, k] f_m at every point: Cq (3 comp, 3 dir, ...),
    F (3, 5, ...) the physical flux."""
    return sum(Cq[m, k][None] * F[m] for m in range(3))


def _surface(gm, uf, gamma, numflux):
    out = {}
    for k in range(3):
        for s in (-1, 1):
            ub = gm.neighbor(uf[(k, -s)], k, s)
            Cb = gm.neighbor(gm.Cf[k][-s], k, s)
            Co = gm.Cf[k][s]
            N = [s * 0.5 * (Co[i] + Cb[i]) for i in range(3)]
            out[(k, s)] = numflux(uf[(k, s)], ub, N)
    return out


def residual(gm, ops, U, gamma, numflux=None):
    """Pre-mass residual of Eq. cons DG strong, line-wise (sum factorised)."""
    nf = numflux or (lambda a, b, N: fx.roe_flux(a, b, N, gamma))
    chi = ops.chi
    uq = apply_3(chi, chi, chi, U)
    F = fx.physical_flux(uq, gamma)                         # (3, 5, E, q, q, q)
    wq = ops.wq
    wperp = wq[:, None] * wq[None, :]
    Rv = torch.zeros_like(uq)
    Rf = {}
    for k in range(3):
        Fk = contravariant_flux(gm.Cq, F, k).movedim(-1 - k, -1)        # (5, E, t2, t1, a)
        Rk = torch.einsum("ab,...b->...a", ops.Dq, Fk) * wq * wperp[..., None]
        Rv = Rv + Rk.movedim(-1, -1 - k)
        for s, t in ((1, ops.tR), (-1, ops.tL)):
            Rf[(k, s)] = -s * torch.einsum("a,...a->...", t, Fk) * wperp
    uf = {(k, s): slab_interp(chi, face_slab(U, k, s)) for k in range(3) for s in (-1, 1)}
    fst = _surface(gm, uf, gamma, nf)
    R = apply_3(chi.T, chi.T, chi.T, Rv)
    for (k, s), fs in fst.items():
        _scatter_slab(R, k, s, slab_interp_T(chi, Rf[(k, s)] + wperp * fs))
    return R


def residual_definition(gm, ops, U, gamma, numflux=None):
    """Eq. cons DG strong with dense operators per element: the volume term
    chi_v^T W3 (D_k (x) phi) f^r_k with 3D Kronecker differentiation matrices,
    the surface term with the dense face interpolation chi_f and the flux basis
    phi evaluated at the face points (Kronecker of t with identities)."""
    nf = numflux or (lambda a, b, N: fx.roe_flux(a, b, N, gamma))
    n, nq, E = ops.n, ops.nq, gm.E
    I = torch.eye(nq, dtype=f64)
    Dk = [kron3(I, I, ops.Dq), kron3(I, ops.Dq, I), kron3(ops.Dq, I, I)]
    W3 = kron3(ops.Wq, ops.Wq, ops.Wq).diagonal()
    chi3 = kron3(ops.chi, ops.chi, ops.chi)
    Uf = U.reshape(5, E, n ** 3)
    uq = torch.einsum("qi,sei->seq", chi3, Uf)
    F = fx.physical_flux(uq, gamma)                         # (3, 5, E, q^3)
    Cq = gm.Cq.reshape(3, 3, E, nq ** 3)
    R = torch.zeros(5, E, n ** 3, dtype=U.dtype)
    for k in range(3):
        fr = sum(Cq[m, k][None] * F[m] for m in range(3))   # (5, E, q^3)
        R = R + torch.einsum("qi,q,qr,ser->sei", chi3, W3, Dk[k], fr)
    Cn = gm.base.C.reshape(3, 3, E, n ** 3)
    for (k, s, pts) in _face_points(nq):
        X = chi_face(ops, k, s)                             # (q^2, n^3)
        Xn = chi_face(ops, k, -s)
        t = ops.tR if s > 0 else ops.tL
        # phi at the face points: t along k, identity in the tangential directions
        e = [I, I, I]
        e[k] = t[None, :]
        Phi = kron3(e[2], e[1], e[0])                       # (q^2, q^3)
        fr = sum(Cq[m, k][None] * F[m] for m in range(3))
        uo = torch.einsum("ti,sei->set", X, Uf)
        ub = torch.einsum("ti,sei->set", Xn, gm.neighbor(Uf, k, s, trailing=1))
        Co = torch.einsum("ti,cei->cet", X, Cn[:, k])
        Cb = torch.einsum("ti,cei->cet", Xn, gm.neighbor(Cn[:, k], k, s, trailing=1))
        N = [s * 0.5 * (Co[i] + Cb[i]) for i in range(3)]
        wf = torch.tensor([float(ops.wq[t1] * ops.wq[t2]) for (t1, t2) in pts], dtype=f64)
        jump = nf(uo, ub, N) - s * torch.einsum("tq,seq->set", Phi, fr)
        R = R + torch.einsum("ti,set->sei", X, jump * wf)
    return R.reshape_as(U)


class DGScheme:
    """du/dt = -A R for conservative strong DG on the GL rule (weight-adjusted
    inverse of the (FR-modified) mass, c = 0 for DG)."""

    def __init__(self, p, ne, lo=0.0, hi=2 * math.pi, beta=0.0, l=None, gamma=1.4, c=0.0, quad="gl", overint=0,
                 source=False, numflux=None):
        self.ops = GLOperators1D(p, c, quad, overint)
        self.mesh = GLMesh(p, ne, self.ops, lo, hi, beta, l)
        self.p, self.gamma, self.c = p, float(gamma), float(c)
        self.source = bool(source)
        self.numflux = numflux

    @property
    def X(self):
        return self.mesh.X

    def residual(self, U, t=0.0, definition=False):
        f = residual_definition if definition else residual
        R = f(self.mesh, self.ops, U, self.gamma, self.numflux)
        if self.source:
            from .problems import mms_source
            chi = self.ops.chi
            q = mms_source(self.mesh.Xq, t, self.gamma)
            R = R - apply_3(chi.T, chi.T, chi.T, self.mesh.WJq * q)
        return R

    def rhs(self, U, t=0.0, definition=False):
        return -wa_apply(self.mesh, self.ops, self.residual(U, t, definition))
