"""1D reference operators on Legendre-Gauss-Lobatto (LGL) nodes (oracle; test
infrastructure only).

Paper: Sec. 2.2 (tensor-product basis, SBP property Eq. SBP), Sec. 3.2 (ESFR
correction operator, Eq. Km), Sec. 4 (ESFR projection, Eq. Fr projection) and
Sec. 7.2 (c_HU makes the modified mass equal to the LGL collocated mass).

The solution is a nodal Lagrange basis collocated on the p+1 LGL nodes, so the
basis evaluated at the volume quadrature nodes is the identity and the 1D mass
matrix is the diagonal weight matrix W.
"""
import math

import torch

f64 = torch.float64


def legendre(p, x):
    """Legendre polynomials P_p(x) and P_{p-1}(x) by the three-term recurrence."""
    P0 = torch.ones_like(x)
    if p == 0:
        return P0, torch.zeros_like(x)
    P1 = x.clone()
    for k in range(2, p + 1):
        P0, P1 = P1, ((2 * k - 1) * x * P1 - (k - 1) * P0) / k
    return P1, P0


def lgl_nodes_weights(p):
    """LGL nodes (roots of (1-x^2) P_p'(x)) and weights 2 / (p(p+1) P_p(x_i)^2).

    Newton's method on q(x) = (1-x^2) P_p'(x) = p (P_{p-1} - x P_p), whose
    derivative is -p(p+1) P_p by Legendre's equation; started from the
    Chebyshev-Lobatto points. The result is symmetrised about 0.
    """
    if p < 1:
        raise ValueError("p >= 1 required")
    x = -torch.cos(math.pi * torch.arange(p + 1, dtype=f64) / p)
    for _ in range(100):
        Pp, Pm = legendre(p, x)
        dx = (x * Pp - Pm) / ((p + 1) * Pp)
        x = x - dx
        if float(dx.abs().max()) < 1e-17:
            break
    x = 0.5 * (x - x.flip(0))
    x[0], x[-1] = -1.0, 1.0
    Pp, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * Pp**2)
    w = 0.5 * (w + w.flip(0))
    return x, w


def barycentric_weights(x):
    """lambda_j = 1 / prod_{k != j} (x_j - x_k)."""
    n = x.numel()
    lam = torch.empty(n, dtype=f64)
    for j in range(n):
        prod = 1.0
        for k in range(n):
            if k != j:
                prod *= float(x[j] - x[k])
        lam[j] = 1.0 / prod
    return lam


def diff_matrix(x):
    """Strong-form derivative D_ij = l_j'(x_i) of the Lagrange basis on nodes x.

    Off-diagonal entries from the barycentric form, diagonal by the
    row-sum-zero property (the derivative of the constant 1 vanishes).
    """
    n = x.numel()
    lam = barycentric_weights(x)
    D = torch.zeros(n, n, dtype=f64)
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -sum(D[i, j] for j in range(n) if j != i)
    return D


class Operators1D:
    """All 1D operators of degree p with FR parameter c (Eq. Km convention).

    Attributes
    ----------
    x, w   LGL nodes and weights (volume quadrature = solution nodes)
    D      strong-form differentiation matrix, D = M^-1 S with M = W
    S1     W D - D^T W: the 1D volume-volume block of (Q~ - Q~^T), Eq. skew-symm
    B      diag(-1, 0, ..., 0, 1): boundary operator, W D + D^T W = B (Eq. SBP)
    Dp     D^p, the p-th derivative operator used in the ESFR correction
    K      1D ESFR correction operator c (D^p)^T W (D^p), Eq. Km with J = 1
    Pi     ESFR projection (M + K)^-1 chi^T W with chi = I, Eq. Fr projection
    """

    def __init__(self, p, c=0.0):
        self.p, self.n, self.c = p, p + 1, float(c)
        self.x, self.w = lgl_nodes_weights(p)
        self.W = torch.diag(self.w)
        self.D = diff_matrix(self.x)
        self.S1 = self.W @ self.D - self.D.T @ self.W
        self.B = torch.zeros(self.n, self.n, dtype=f64)
        self.B[0, 0], self.B[-1, -1] = -1.0, 1.0
        self.Dp = torch.linalg.matrix_power(self.D, p)
        self.K = self.c * self.Dp.T @ self.W @ self.Dp
        self.MK = self.W + self.K
        self.Pi = torch.linalg.solve(self.MK, self.W)


def c_hu(p):
    """FR parameter c_HU (Eq. Km convention) for which the modified 1D mass on
    LGL nodes equals the exactly integrated Lagrange mass (Sec. 7.2).

    Derived from the requirement M_exact + c (D^p)^T W D^p = W_LGL, where
    M_exact is the exactly integrated mass of the LGL Lagrange basis, computed
    here with a (p+2)-point Gauss-Legendre rule (exact for degree 2p). The
    difference W_LGL - M_exact is rank one, proportional to d d^T with
    d = p! lambda, so c follows from any one entry.
    """
    ops = Operators1D(p, 0.0)
    M = exact_lagrange_mass(ops.x)
    K1 = ops.Dp.T @ ops.W @ ops.Dp
    diff = ops.W - M
    i = int(torch.argmax(K1.abs()))
    return float(diff.flatten()[i] / K1.flatten()[i])


def gauss_legendre(m):
    """m-point Gauss-Legendre rule (eigenvalues of the Jacobi matrix)."""
    k = torch.arange(1, m, dtype=f64)
    b = k / torch.sqrt(4 * k * k - 1)
    T = torch.diag(b, 1) + torch.diag(b, -1)
    x, V = torch.linalg.eigh(T)
    w = 2 * V[0, :] ** 2
    return x, w


def lagrange_eval(xnodes, xeval):
    """Matrix L_ij = l_j(xeval_i) of the Lagrange basis on xnodes."""
    n = xnodes.numel()
    L = torch.ones(xeval.numel(), n, dtype=f64)
    for j in range(n):
        for k in range(n):
            if k != j:
                L[:, j] *= (xeval - xnodes[k]) / (xnodes[j] - xnodes[k])
    return L


def exact_lagrange_mass(x):
    """Exactly integrated mass matrix int l_i l_j of the Lagrange basis on x."""
    n = x.numel()
    xg, wg = gauss_legendre(n + 1)
    L = lagrange_eval(x, xg)
    return L.T @ torch.diag(wg) @ L


def kron3(Az, Ay, Ax):
    """3D tensor-product operator for node index a + n b + n^2 c (xi fastest)."""
    return torch.kron(Az, torch.kron(Ay, Ax))
