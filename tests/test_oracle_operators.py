"""Pins for the oracle's 1D/3D reference operators (CPU only).

Each check is independent of how the oracle builds the operator: closed forms,
exactness on polynomials, the SBP identity (Sec. 2.2, Eq. SBP; Sec. 3.3,
Eq. SBP Qtilde), the p-th derivative of a Lagrange polynomial, the rank-one
structure of the ESFR correction (Eq. Km) and of the FR projection (Eq. Fr
projection), and the c_HU special case of Sec. 7.2.
"""
import json
import math
import os

import pytest
import torch

from oracle import operators as op
from oracle.residual import hybrid_operators, _faces

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _ev(s):
    return float(eval(s, {"sqrt": math.sqrt}))


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_lgl_closed_forms(p):
    g = json.load(open(os.path.join(GOLD, "lgl_closed_forms.json")))["rules"][str(p)]
    x, w = op.lgl_nodes_weights(p)
    xr = torch.tensor([_ev(s) for s in g["x"]], dtype=torch.float64)
    wr = torch.tensor([_ev(s) for s in g["w"]], dtype=torch.float64)
    assert torch.allclose(x, xr, atol=1e-15, rtol=0)
    assert torch.allclose(w, wr, atol=1e-15, rtol=0)
    assert abs(float(w.sum()) - 2.0) < 1e-15


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 8])
def test_lgl_integrates_degree_2p_minus_1(p):
    x, w = op.lgl_nodes_weights(p)
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(float((w * x**k).sum()) - exact) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_D_exact_on_polynomials(p):
    ops = op.Operators1D(p)
    for k in range(p + 1):
        f = ops.x**k
        df = k * ops.x ** (k - 1) if k else torch.zeros_like(ops.x)
        assert torch.allclose(ops.D @ f, df, atol=1e-12, rtol=0)
    assert float((ops.D @ torch.ones(p + 1, dtype=torch.float64)).abs().max()) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_sbp_1d(p):
    ops = op.Operators1D(p)
    assert torch.allclose(ops.W @ ops.D + ops.D.T @ ops.W, ops.B, atol=1e-14, rtol=0)
    assert torch.allclose(ops.S1, -ops.S1.T, atol=0, rtol=0)


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_Dp_rows_are_p_factorial_lambda(p):
    """The p-th derivative of l_j is the constant p! * (leading coefficient)."""
    ops = op.Operators1D(p)
    lam = op.barycentric_weights(ops.x)
    d = math.factorial(p) * lam
    rel = (ops.Dp - d[None, :]).abs().max() / d.abs().max()
    assert float(rel) < 1e-11


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_K_rank_one(p):
    """Eq. Km in 1D on LGL: K = c (D^p)^T W D^p = 2 c d d^T (sum of weights is 2)."""
    c = 1.7e-3
    ops = op.Operators1D(p, c)
    d = math.factorial(p) * op.barycentric_weights(ops.x)
    K = 2 * c * torch.outer(d, d)
    assert float((ops.K - K).abs().max() / K.abs().max()) < 1e-11


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_c_hu_special_case(p):
    """Sec. 7.2: with c_HU the modified mass of the exactly integrated Lagrange
    basis equals the LGL collocated mass. Closed form: W_LGL - M_exact is rank
    one, E_p lambda lambda^T, with E_p the LGL quadrature error of x^(2p), so
    c_HU = E_p / (2 (p!)^2)."""
    x, w = op.lgl_nodes_weights(p)
    lam = op.barycentric_weights(x)
    Ep = float((w * x ** (2 * p)).sum()) - 2.0 / (2 * p + 1)
    M = op.exact_lagrange_mass(x)
    assert torch.allclose(torch.diag(w) - M, Ep * torch.outer(lam, lam), atol=1e-14 * float(lam.abs().max()) ** 2, rtol=1e-12)
    chu = op.c_hu(p)
    assert abs(chu - Ep / (2 * math.factorial(p) ** 2)) < 1e-13 * abs(chu)
    ops = op.Operators1D(p, chu)
    assert torch.allclose(M + ops.K, torch.diag(w), atol=1e-14, rtol=0)


def test_gauss_legendre_rule():
    for m in range(2, 8):
        x, w = op.gauss_legendre(m)
        for k in range(2 * m):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(float((w * x**k).sum()) - exact) < 1e-14


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("c", [0.0, 1e-3, 0.37])
def test_projection_closed_form(p, c):
    """Eq. Fr projection with chi = I: Pi = (W + 2c d d^T)^-1 W, which by
    Sherman-Morrison is I - alpha W^-1 d d^T, alpha = 2c / (1 + 2c d^T W^-1 d).
    At c = 0 it is the identity."""
    ops = op.Operators1D(p, c)
    d = math.factorial(p) * op.barycentric_weights(ops.x)
    mu = float((d * d / ops.w).sum())
    alpha = 2 * c / (1 + 2 * c * mu)
    Pi = torch.eye(p + 1, dtype=torch.float64) - alpha * torch.outer(d / ops.w, d)
    # the solve is conditioned like 1 + 2 c mu
    assert torch.allclose(ops.Pi, Pi, atol=1e-14 * (1 + 2 * c * mu), rtol=0)
    if c == 0.0:
        assert torch.equal(ops.Pi, torch.eye(p + 1, dtype=torch.float64))


@pytest.mark.parametrize("p", [2, 3])
def test_3d_modified_mass_is_tensor_product(p):
    """Eq. Km summed over (s,v,w) in {0,p}^3 with c_(s,v,w) = c^((s+v+w)/p), on
    the reference element (J = 1), equals the Kronecker product of the 1D
    modified masses W + K."""
    import itertools
    c = 0.013
    ops = op.Operators1D(p, c)
    n = p + 1
    I = torch.eye(n, dtype=torch.float64)
    W3 = op.kron3(ops.W, ops.W, ops.W)
    MK = W3.clone()
    for s, v, w in itertools.product((0, p), repeat=3):
        if s + v + w == 0:
            continue
        D3 = op.kron3(ops.Dp if w else I, ops.Dp if v else I, ops.Dp if s else I)
        MK += c ** ((s + v + w) / p) * D3.T @ W3 @ D3
    ref = op.kron3(ops.MK, ops.MK, ops.MK)
    assert float((MK - ref).abs().max() / ref.abs().max()) < 1e-12


@pytest.mark.parametrize("p", [2, 3, 4])
def test_hybrid_operator_sbp(p):
    """Eq. SBP Qtilde: the volume block Q_k = W3 D_k satisfies
    Q_k + Q_k^T = E^T W_f diag(n_k) E (3D SBP on the face quadrature), and the
    assembled hybrid Q~ - Q~^T is skew-symmetric."""
    ops = op.Operators1D(p)
    n = p + 1
    Qs, fmap, wf, faces = hybrid_operators(ops)
    I = torch.eye(n, dtype=torch.float64)
    Dk = [op.kron3(I, I, ops.D), op.kron3(I, ops.D, I), op.kron3(ops.D, I, I)]
    W3 = op.kron3(ops.W, ops.W, ops.W)
    Nv = n**3
    for k in range(3):
        Q = W3 @ Dk[k]
        B = torch.zeros(Nv, Nv, dtype=torch.float64)
        col = 0
        for (kf, side, nodes) in faces:
            for q, node in enumerate(nodes):
                if kf == k:
                    B[node, node] += side * wf[col + q]
            col += len(nodes)
        assert torch.allclose(Q + Q.T, B, atol=1e-13, rtol=0)
        assert torch.equal(Qs[k], -Qs[k].T)
        # volume rows of the hybrid operator sum to zero (constant preservation);
        # face rows sum to -W_f n_k
        rows = Qs[k].sum(1)
        assert float(rows[:Nv].abs().max()) < 1e-13
        expect, col = [], 0
        for (kf, side, nodes) in faces:
            expect += [-side * float(wf[col + q]) if kf == k else 0.0 for q in range(len(nodes))]
            col += len(nodes)
        assert torch.allclose(rows[Nv:], torch.tensor(expect, dtype=torch.float64), atol=1e-14, rtol=0)


def test_face_lists_cover_boundary():
    for n in (3, 4):
        faces = _faces(n)
        assert len(faces) == 6
        assert all(len(f[2]) == n * n for f in faces)
