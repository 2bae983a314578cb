"""Warped periodic hexahedral mesh and metric terms (oracle; test infrastructure).

Paper: Sec. 2.2 (mapping, covariant/contravariant bases, Jacobian J, metric
cofactor matrix C with C^T = J (J^Omega)^-1, discrete GCL, Eq. GCL) and Sec. 7
(nonsymmetric warped map, Eq. warped grid).

Layout: a nodal field on the mesh is a tensor of shape (E, n, n, n) indexed
[e, c, b, a] with a the xi index (fastest), element e = ex + nx (ey + ny ez).

Readings of the paper used here:
  * the grid is of the solution degree p, with its nodes at the LGL solution
    nodes (the paper defers the exact construction to another report);
  * C is built with the conservative curl form of Kopriva (cited in Sec. 2.2),
    differentiating element-local coordinates X - X_center;
  * the warp's l defaults to (hi - lo) / (2 pi), as printed in Eq. warped grid,
    which keeps the map periodic on the box.
"""
import math

import torch

from .operators import Operators1D

f64 = torch.float64


def warp_map(a, b, c, beta, l):
    """Eq. warped grid: nonsymmetric sinusoidal warp of reference-uniform points."""
    x = a + beta * torch.sin(a / l) * torch.sin(b / l) * torch.sin(2 * c / l)
    y = b + beta * torch.sin(4 * a / l) * torch.sin(b / l) * torch.sin(3 * c / l)
    z = c + beta * torch.sin(2 * a / l) * torch.sin(5 * b / l) * torch.sin(c / l)
    return x, y, z


def apply_D(D, F, axis):
    """Apply the 1D operator D along one reference direction of (..., n, n, n).

    axis 0 = xi (last tensor dim), 1 = eta, 2 = zeta.
    """
    if axis == 0:
        return torch.einsum("ij,...cbj->...cbi", D, F)
    if axis == 1:
        return torch.einsum("ij,...cja->...cia", D, F)
    return torch.einsum("ij,...jba->...iba", D, F)


class Mesh:
    """Structured periodic box [lo, hi]^3 split into ne[0] x ne[1] x ne[2]
    hexahedra of degree p, with the optional warp of Eq. warped grid."""

    def __init__(self, p, ne, lo=0.0, hi=2 * math.pi, beta=0.0, l=None):
        self.p, self.n = p, p + 1
        self.ne = tuple(int(v) for v in ne)
        self.E = self.ne[0] * self.ne[1] * self.ne[2]
        self.lo, self.hi = float(lo), float(hi)
        self.beta = float(beta)
        self.l = (self.hi - self.lo) / (2 * math.pi) if (l is None or l <= 0) else float(l)
        self.ops = Operators1D(p, 0.0)
        n, (nx, ny, nz) = self.n, self.ne
        h = [(self.hi - self.lo) / m for m in self.ne]
        self.h = h
        xi = self.ops.x
        ez, ey, ex = torch.meshgrid(torch.arange(nz), torch.arange(ny), torch.arange(nx), indexing="ij")
        ex, ey, ez = (t.reshape(-1).to(f64) for t in (ex, ey, ez))
        # reference-uniform coordinates of every node, shape (E, n, n, n)
        A = self.lo + h[0] * (ex[:, None, None, None] + (xi[None, None, None, :] + 1) / 2)
        Bc = self.lo + h[1] * (ey[:, None, None, None] + (xi[None, None, :, None] + 1) / 2)
        Cc = self.lo + h[2] * (ez[:, None, None, None] + (xi[None, :, None, None] + 1) / 2)
        A, Bc, Cc = torch.broadcast_tensors(A, Bc, Cc)
        X = torch.stack(warp_map(A, Bc, Cc, self.beta, self.l))  # (3, E, n, n, n)
        self.X = X
        # element centres (image of the un-warped centre is not needed: any
        # per-element constant works; use the un-warped centre)
        ctr = torch.stack([self.lo + h[0] * (ex + 0.5), self.lo + h[1] * (ey + 0.5), self.lo + h[2] * (ez + 0.5)])
        self.center = ctr
        self._metrics()

    def _metrics(self):
        D = self.ops.D
        X = self.X
        Xl = X - self.center[:, :, None, None, None]
        # G[m][j] = d X_m / d xi_j
        G = [[apply_D(D, X[m], j) for j in range(3)] for m in range(3)]
        self.G = G
        J = (G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1])
             - G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0])
             + G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]))
        self.J = J
        # conservative curl form: for (n, m, l) cyclic, with V_j = Xl_l * G[m][j],
        # C[n][i] = -(curl_xi V)_i
        C = [[None] * 3 for _ in range(3)]
        for (nn, mm, ll) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
            V = [Xl[ll] * G[mm][j] for j in range(3)]
            C[nn][0] = -(apply_D(D, V[2], 1) - apply_D(D, V[1], 2))
            C[nn][1] = -(apply_D(D, V[0], 2) - apply_D(D, V[2], 0))
            C[nn][2] = -(apply_D(D, V[1], 0) - apply_D(D, V[0], 1))
        # C tensor: (3 components n, 3 reference directions i, E, n, n, n)
        self.C = torch.stack([torch.stack(row) for row in C])
        w = self.ops.w
        W3 = w[None, None, None, :] * w[None, None, :, None] * w[None, :, None, None]
        self.W3 = W3.expand_as(J)
        self.WJ = self.W3 * J
        self.invWJ = 1.0 / self.WJ

    def grid_shape(self):
        """Element grid (nz, ny, nx) so that E reshapes to it (x fastest)."""
        return (self.ne[2], self.ne[1], self.ne[0])

    def neighbor(self, F, axis, side):
        """Field of the periodic neighbour across face (axis, side): element-wise
        gather, so neighbour(F, 0, +1)[e] = F[e + 1 in x, periodic]."""
        shp = F.shape
        lead = shp[:-4]
        G = F.reshape(*lead, *self.grid_shape(), *shp[-3:])
        dim = len(lead) + (2 - axis)
        G = torch.roll(G, shifts=-side, dims=dim)
        return G.reshape(shp)
