"""Inverse of the FR-modified mass matrix (oracle; test infrastructure).

Paper: Sec. 3.2, Eq. Km (ESFR correction operator K_m built from the
derivative operators D^s with s in {0, p} and c_(s,v,w) = c^((s+v+w)/p));
Sec. 4, Eq. weight-adj ESFR mass:
    (M_m + K_m)^-1  ~=  Pi~(xi) (W J_m)^-1 Pi~(xi)^T,
    Pi~ = Pi~_xi (x) Pi~_eta (x) Pi~_zeta,  Pi~_1D = (M + K)^-1 chi^T W.

Both the weight-adjusted approximation (dense tensor-product operator, as
printed) and the exact dense inverse are provided.
"""
import itertools

import torch

from .operators import Operators1D, kron3


def wa_apply(mesh, c, R):
    """A R with A = Pi3 diag(1/(W J)) Pi3^T, per element and state (Eq.
    weight-adj ESFR mass). R has shape (S, E, n, n, n)."""
    ops = Operators1D(mesh.p, c)
    P3 = kron3(ops.Pi, ops.Pi, ops.Pi).to(R.dtype)
    S, E = R.shape[0], R.shape[1]
    Nv = mesh.n ** 3
    Rf = R.reshape(S, E, Nv)
    y = torch.einsum("ji,sej->sei", P3, Rf)           # Pi3^T R
    y = y * mesh.invWJ.reshape(E, Nv)                 # (W J)^-1
    z = torch.einsum("ij,sej->sei", P3, y)            # Pi3 (.)
    return z.reshape_as(R)


def modified_mass(mesh, c):
    """Dense M_m + K_m for every element, shape (E, Nv, Nv) (Eq. Km with the
    collocated LGL basis, so M_m = diag(W J))."""
    ops = Operators1D(mesh.p, c)
    n, p = mesh.n, mesh.p
    I = torch.eye(n, dtype=torch.float64)
    Nv = n ** 3
    Mm = torch.diag_embed(mesh.WJ.reshape(mesh.E, Nv))
    MK = Mm.clone()
    for s, v, w in itertools.product((0, p), repeat=3):
        if s + v + w == 0:
            continue
        order = (s + v + w) / p
        csvw = c ** order
        Dx = ops.Dp if s else I
        Dy = ops.Dp if v else I
        Dz = ops.Dp if w else I
        Dsvw = kron3(Dz, Dy, Dx)
        MK = MK + csvw * Dsvw.T @ Mm @ Dsvw
    return MK


def exact_apply(mesh, c, R):
    """(M_m + K_m)^-1 R with the dense modified mass (Cholesky solve)."""
    MK = modified_mass(mesh, c)
    S, E = R.shape[0], R.shape[1]
    Nv = mesh.n ** 3
    L = torch.linalg.cholesky(MK).to(R.dtype)
    Rf = R.reshape(S, E, Nv).permute(1, 2, 0)         # (E, Nv, S)
    X = torch.cholesky_solve(Rf, L)
    return X.permute(2, 0, 1).reshape_as(R)
