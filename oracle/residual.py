"""NSFR spatial residual on collocated LGL nodes (oracle; test infrastructure).

Paper: Sec. 3.3, Eq. NSFR with the hybridised skew-symmetric operator of
Eq. skew-symm qtilde oper and the metric-split reference two-point flux
(F^r)_ij = f_s(u_i, u_j) . (C_i + C_j) / 2; Sec. 5 (sum-factorised evaluation
of the Hadamard product: on a tensor-product element the volume-volume block
in direction k is nonzero only between nodes on the same k-line).

The residual returned here is the pre-mass vector R with
    (M_m + K_m) du/dt + R = 0,   R = R_vol + R_surf,
where R_vol = [chi_v^T chi_f^T][(Q~ - Q~^T) o F^r] 1 and
R_surf = sum_f sum_k chi(xi_fk)^T W_fk n^r . f*.

Two independent evaluations are provided:
  * ``residual``            line-wise (sum-factorised) form, all elements at once;
  * ``residual_definition`` the literal dense hybridised form, for small meshes.

Readings used: the solution, volume quadrature and surface quadrature all sit
on the LGL nodes, so chi_v = I, the face basis is node extraction and the
entropy projection returns the nodal state itself; the numerical flux at a
face node uses the direction N = (C_L n_L - C_R n_R) / 2 built from the metric
columns of the two elements at the shared node (n = reference outward normal).
"""
import torch

from . import flux as fx


def _line_last(F, k):
    """Move reference direction k (0 = xi) of (..., n, n, n) to the last dim."""
    return F.movedim(-1 - k, -1)


def _line_back(F, k):
    return F.movedim(-1, -1 - k)


def volume_residual(mesh, U, gamma, two_point):
    """R_vol[abc] = sum_k sum_{a'} S1[a, a'] w_perp f_s(U_a, U_a'; (C_k(a) + C_k(a'))/2)
    along every k-line (the volume-volume block of Eq. NSFR in sum-factorised
    form). U has shape (5, E, n, n, n)."""
    S1, w = mesh.ops.S1, mesh.ops.w
    wperp = (w[:, None] * w[None, :])[:, :, None]  # over the two other directions
    R = torch.zeros_like(U)
    for k in range(3):
        Uk = _line_last(U, k)
        Ck = _line_last(mesh.C[:, k], k)
        Ua, Ub = Uk[..., :, None], Uk[..., None, :]
        N = [0.5 * (Ck[i][..., :, None] + Ck[i][..., None, :]) for i in range(3)]
        F = two_point(Ua, Ub, N)  # (5, E, ., ., n, n)
        Rk = torch.einsum("ij,...ij->...i", S1.to(F.dtype), F) * wperp
        R = R + _line_back(Rk, k)
    return R


def face_flux(mesh, U, k, side, gamma, two_point, dissipation=None):
    """Numerical flux n^r . f* at the face nodes of every element on the face
    normal to direction k on the given side (+1 or -1). Returns (5, E, n, n)
    with the two tangential indices in their natural order."""
    n = mesh.n
    a_own = n - 1 if side > 0 else 0
    a_nbr = 0 if side > 0 else n - 1
    Un = mesh.neighbor(U, k, side)
    Cn = mesh.neighbor(mesh.C[:, k], k, side)
    Uo = _line_last(U, k)[..., a_own]
    Ub = _line_last(Un, k)[..., a_nbr]
    Co = _line_last(mesh.C[:, k], k)[..., a_own]
    Cb = _line_last(Cn, k)[..., a_nbr]
    N = [side * 0.5 * (Co[i] + Cb[i]) for i in range(3)]
    fstar = two_point(Uo, Ub, N)
    if dissipation is not None:
        fstar = fstar + dissipation(Uo, Ub, N)
    return fstar


def surface_residual(mesh, U, gamma, two_point, dissipation=None):
    """R_surf: + W_f n^r . f* added at every face node (Eq. NSFR, last term)."""
    w = mesh.ops.w
    Wf = w[:, None] * w[None, :]
    R = torch.zeros_like(U)
    n = mesh.n
    for k in range(3):
        Rk = torch.zeros_like(_line_last(U, k))
        for side in (-1, 1):
            fs = face_flux(mesh, U, k, side, gamma, two_point, dissipation)
            idx = n - 1 if side > 0 else 0
            Rk[..., idx] = Rk[..., idx] + Wf * fs
        R = R + _line_back(Rk, k)
    return R


def ec_two_point(gamma, variant):
    return lambda Ua, Ub, N: fx.ec_flux(Ua, Ub, N, gamma, variant)


def residual(mesh, U, gamma, variant=0, dissipation=False, two_point=None):
    """Pre-mass NSFR residual R = R_vol + R_surf (line-wise form)."""
    tp = two_point or ec_two_point(gamma, variant)
    diss = fx.surface_dissipation(dissipation, gamma)
    return volume_residual(mesh, U, gamma, tp) + surface_residual(mesh, U, gamma, tp, diss)


# ---------------------------------------------------------------------------
# Definition form: the dense hybridised operator of Eq. skew-symm qtilde oper
# ---------------------------------------------------------------------------

def _faces(n):
    """Faces as (k, side); face node lists as volume node indices a + n b + n^2 c."""
    faces = []
    for k in range(3):
        for side in (-1, 1):
            idx_line = n - 1 if side > 0 else 0
            nodes = []
            for t2 in range(n):
                for t1 in range(n):
                    if k == 0:
                        a, b, c = idx_line, t1, t2
                    elif k == 1:
                        a, b, c = t1, idx_line, t2
                    else:
                        a, b, c = t1, t2, idx_line
                    nodes.append(a + n * b + n * n * c)
            faces.append((k, side, nodes))
    return faces


def hybrid_operators(ops):
    """Dense Q~_k - Q~_k^T, k = 1..3, of size (N_v + N_fp)^2 for the LGL
    element, together with the face-to-volume node map and the face weights.

    Volume-volume block: W3 D_k - D_k^T W3 (D_k the 3D strong derivative);
    volume-face block: phi(xi_f)^T W_f diag(n^r_f); face-volume block: minus
    its transpose; face-face block: 0."""
    from .operators import kron3
    n = ops.n
    I = torch.eye(n, dtype=torch.float64)
    Dk = [kron3(I, I, ops.D), kron3(I, ops.D, I), kron3(ops.D, I, I)]
    W3 = torch.diag(kron3(ops.W, ops.W, ops.W).diagonal())
    faces = _faces(n)
    Nv = n ** 3
    Nfp = sum(len(f[2]) for f in faces)
    Nt = Nv + Nfp
    fmap = []
    wf = []
    for (k, side, nodes) in faces:
        fmap += nodes
        wf += [float(ops.w[t1] * ops.w[t2]) for t2 in range(n) for t1 in range(n)]
    fmap = torch.tensor(fmap)
    wf = torch.tensor(wf, dtype=torch.float64)
    Qs = []
    for k in range(3):
        Q = torch.zeros(Nt, Nt, dtype=torch.float64)
        Q[:Nv, :Nv] = W3 @ Dk[k] - Dk[k].T @ W3
        col = Nv
        for (kf, side, nodes) in faces:
            for q, vnode in enumerate(nodes):
                if kf == k:
                    val = wf[col - Nv] * side
                    Q[vnode, col] += val   # phi(xi_f)^T W_f n_f
                    Q[col, vnode] -= val   # -W_f n_f phi(xi_f)
                col += 1
        Qs.append(Q)
    return Qs, fmap, wf, faces


def residual_definition(mesh, U, gamma, variant=0, dissipation=False, two_point=None):
    """Pre-mass residual from the literal dense form of Eq. NSFR:
    R = [chi_v^T chi_f^T][(Q~ - Q~^T) o F^r] 1 + sum_f chi_f^T W_f n^r . f*.
    Memory grows as E (N_v + N_fp)^2: small meshes only."""
    tp = two_point or ec_two_point(gamma, variant)
    diss = fx.surface_dissipation(dissipation, gamma)
    ops = mesh.ops
    n = mesh.n
    Nv = n ** 3
    E = mesh.E
    Qs, fmap, wf, faces = hybrid_operators(ops)
    sel = torch.cat([torch.arange(Nv), fmap])  # total node -> volume node
    Uv = U.reshape(5, E, Nv)
    Ut = Uv[:, :, sel]
    H = torch.zeros(5, E, sel.numel(), dtype=U.dtype)
    for k in range(3):
        Ct = mesh.C[:, k].reshape(3, E, Nv)[:, :, sel]
        N = [0.5 * (Ct[i][:, :, None] + Ct[i][:, None, :]) for i in range(3)]
        F = tp(Ut[:, :, :, None], Ut[:, :, None, :], N)  # (5, E, Nt, Nt)
        H = H + torch.einsum("ij,seij->sei", Qs[k].to(F.dtype), F)
    R = H[:, :, :Nv].clone()
    R.index_add_(2, fmap, H[:, :, Nv:])
    # surface numerical flux term
    col = 0
    for (k, side, nodes) in faces:
        fs = face_flux(mesh, U, k, side, gamma, tp, diss)  # (5, E, n, n), tangential (t2, t1)
        fs = fs.reshape(5, E, n * n)
        R.index_add_(2, torch.tensor(nodes), fs * wf[col:col + n * n])
        col += n * n
    return R.reshape_as(U)
