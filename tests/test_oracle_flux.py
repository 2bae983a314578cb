"""Pins for the oracle's fluxes (CPU only).

Checks that do not reuse the oracle's formulas: Tadmor's shuffle condition
(Sec. 2.1, Eq. EC flux / Eq. Tadmor shuffle quad node) against the entropy
variables and potential, consistency with the physical Euler flux of Sec. 2.1,
exact symmetry, linearity in the direction vector, the entropy variables as the
gradient of the entropy (checked by complex step), the potential identity
psi = v . f - F, and the logarithmic mean against 50-digit arithmetic.
"""
import math

import mpmath
import pytest
import torch
from hypothesis import given, settings, strategies as st

from oracle import flux as fx

G = 1.4


def rand_states(n, seed, spread=0.5):
    g = torch.Generator().manual_seed(seed)
    r = lambda: torch.rand(n, generator=g, dtype=torch.float64)  # noqa: E731
    rho = 0.5 + spread * 2 * r()
    vel = [2 * r() - 1 for _ in range(3)]
    p = 0.3 + spread * 3 * r()
    return fx.conservative(rho, vel, p, G)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("spread", [1e-6, 1e-3, 0.5])
def test_tadmor_shuffle(variant, spread):
    Ua = rand_states(4000, 1, 0.5)
    # neighbour state: every primitive perturbed by a relative amount ~ spread
    rho, vel, p, _ = fx.primitives(Ua, G)
    gg = torch.Generator().manual_seed(2)
    j = lambda: 1 + spread * (2 * torch.rand(4000, generator=gg, dtype=torch.float64) - 1)  # noqa: E731
    Ub = fx.conservative(rho * j(), [v * j() for v in vel], p * j(), G)
    g = torch.Generator().manual_seed(3)
    N = [torch.randn(4000, generator=g, dtype=torch.float64) for _ in range(3)]
    F = fx.ec_flux(Ua, Ub, N, G, variant)
    dv = fx.entropy_variables(Ua, G) - fx.entropy_variables(Ub, G)
    dpsi = fx.entropy_potential(Ua, G) - fx.entropy_potential(Ub, G)
    lhs = (dv * F).sum(0)
    rhs = sum(dpsi[k] * N[k] for k in range(3))
    # round-off scale of the two sides before cancellation of the jumps
    va, vb = fx.entropy_variables(Ua, G), fx.entropy_variables(Ub, G)
    pa, pb = fx.entropy_potential(Ua, G), fx.entropy_potential(Ub, G)
    scale = ((va.abs() + vb.abs()) * F.abs()).sum(0) + sum((pa[k].abs() + pb[k].abs()) * N[k].abs() for k in range(3))
    assert float(((lhs - rhs).abs() / scale).max()) < 1e-14


@pytest.mark.parametrize("variant", [0, 1])
def test_consistency(variant):
    U = rand_states(1000, 4)
    g = torch.Generator().manual_seed(5)
    N = [torch.randn(1000, generator=g, dtype=torch.float64) for _ in range(3)]
    F = fx.ec_flux(U, U, N, G, variant)
    f = fx.physical_flux(U, G)
    ref = sum(f[k] * N[k] for k in range(3))
    assert float(((F - ref).abs() / (ref.abs() + 1)).max()) < 4e-15


@pytest.mark.parametrize("variant", [0, 1])
def test_symmetry_bitwise_and_linear_in_N(variant):
    Ua, Ub = rand_states(1000, 6), rand_states(1000, 7)
    g = torch.Generator().manual_seed(8)
    N1 = [torch.randn(1000, generator=g, dtype=torch.float64) for _ in range(3)]
    N2 = [torch.randn(1000, generator=g, dtype=torch.float64) for _ in range(3)]
    assert torch.equal(fx.ec_flux(Ua, Ub, N1, G, variant), fx.ec_flux(Ub, Ua, N1, G, variant))
    a, b = 0.7, -1.9
    lhs = fx.ec_flux(Ua, Ub, [a * x + b * y for x, y in zip(N1, N2)], G, variant)
    rhs = a * fx.ec_flux(Ua, Ub, N1, G, variant) + b * fx.ec_flux(Ua, Ub, N2, G, variant)
    assert float(((lhs - rhs).abs() / (rhs.abs() + 1)).max()) < 1e-13
    # negating N negates the flux exactly (used for the two sides of a face)
    assert torch.equal(fx.ec_flux(Ua, Ub, [-x for x in N1], G, variant), -fx.ec_flux(Ua, Ub, N1, G, variant))


@settings(max_examples=300, deadline=None)
@given(a=st.floats(1e-3, 1e3), r=st.floats(-0.3, 0.3))
def test_ln_mean_against_high_precision(a, r):
    b = a * math.exp(r)
    mpmath.mp.dps = 50
    A, B = mpmath.mpf(a), mpmath.mpf(b)
    ref = (A + B) / 2 if A == B else (A - B) / (mpmath.log(A) - mpmath.log(B))
    got = float(fx.ln_mean(torch.tensor([a], dtype=torch.float64), torch.tensor([b], dtype=torch.float64))[0])
    # closed-form branch: rounding of ln a, ln b is amplified by 1 / |ln a - ln b|
    la, lb = math.log(a), math.log(b)
    amp = (abs(la) + abs(lb)) / abs(la - lb) if la != lb else 0.0
    assert abs(got - float(ref)) <= (2e-15 + 4e-16 * amp) * float(ref)


def test_entropy_variables_are_gradient_of_entropy():
    U = rand_states(200, 9)
    v = fx.entropy_variables(U, G)
    h = 1e-30
    for s in range(5):
        e = torch.zeros_like(U)
        e[s] = 1.0
        d = fx.entropy_function(U.to(torch.complex128) + 1j * h * e, G).imag / h
        assert torch.allclose(d, v[s], rtol=1e-13, atol=1e-13)


def test_entropy_potential_identity():
    """psi^k = v . f^k - F^k with entropy flux F^k = U u_k."""
    U = rand_states(300, 10)
    v = fx.entropy_variables(U, G)
    f = fx.physical_flux(U, G)
    Uent = fx.entropy_function(U, G)
    rho, vel, _, _ = fx.primitives(U, G)
    psi = fx.entropy_potential(U, G)
    for k in range(3):
        ref = (v * f[k]).sum(0) - Uent * vel[k]
        assert torch.allclose(psi[k], ref, rtol=1e-12, atol=1e-12)


def test_kinetic_energy_preserving_structure():
    """Chandrashekar-type flux: momentum flux = u_avg * mass flux + pressure N."""
    Ua, Ub = rand_states(500, 11), rand_states(500, 12)
    N = [torch.ones(500, dtype=torch.float64), torch.zeros(500, dtype=torch.float64), torch.zeros(500, dtype=torch.float64)]
    F = fx.ec_flux(Ua, Ub, N, G, 0)
    _, va, pa, _ = fx.primitives(Ua, G)
    _, vb, pb, _ = fx.primitives(Ub, G)
    assert torch.allclose(F[2], 0.5 * (va[1] + vb[1]) * F[0], rtol=1e-14, atol=1e-14)
    assert torch.allclose(F[1] - 0.5 * (va[0] + vb[0]) * F[0], 0.5 * (pa + pb), rtol=1e-13, atol=1e-13)


def test_llf_dissipation_properties():
    Ua, Ub = rand_states(300, 13), rand_states(300, 14)
    g = torch.Generator().manual_seed(15)
    N = [torch.randn(300, generator=g, dtype=torch.float64) for _ in range(3)]
    d1 = fx.llf_dissipation(Ua, Ub, N, G)
    d2 = fx.llf_dissipation(Ub, Ua, [-x for x in N], G)
    assert torch.allclose(d1, -d2, rtol=0, atol=0)
    assert float(fx.llf_dissipation(Ua, Ua, N, G).abs().max()) == 0.0


def test_llf_dissipation_hand_computed_pair():
    # Ua: rho 1, u (0.5, 0, 0), p 1; Ub: rho 1.2, at rest, p 0.8; N = (2, 0, 0).
    # Wave speeds: 0.5 + sqrt(1.4) on the left, sqrt(1.4 * 0.8 / 1.2) on the
    # right; the left one is larger. Conservative jump Ub - Ua:
    # (0.2, -0.5, 0, 0, 2.0 - 2.625).
    one = lambda v: torch.tensor([v], dtype=torch.float64)  # noqa: E731
    Ua = fx.conservative(one(1.0), [one(0.5), one(0.0), one(0.0)], one(1.0), G)
    Ub = fx.conservative(one(1.2), [one(0.0), one(0.0), one(0.0)], one(0.8), G)
    N = [one(2.0), one(0.0), one(0.0)]
    lam = 0.5 + math.sqrt(1.4)
    jump = [0.2, -0.5, 0.0, 0.0, -0.625]
    d = fx.llf_dissipation(Ua, Ub, N, G)[:, 0]
    for s in range(5):
        assert abs(float(d[s]) - (-0.5 * 2.0 * lam * jump[s])) < 1e-14


def test_llf_dissipation_is_entropy_dissipative():
    Ua, Ub = rand_states(500, 16), rand_states(500, 17)
    g = torch.Generator().manual_seed(18)
    N = [torch.randn(500, generator=g, dtype=torch.float64) for _ in range(3)]
    d = fx.llf_dissipation(Ua, Ub, N, G)
    dv = fx.entropy_variables(Ub, G) - fx.entropy_variables(Ua, G)
    assert float((dv * d).sum(0).max()) <= 0.0


# ---- entropy-stable Roe-type matrix dissipation (Sec. 6.3, Sec. 7.1)

def _flux_jacobian_abs(U, n):
    """|A| = V |Lambda| V^-1 of the physical flux Jacobian A = d(f . n)/du at one
    state, by automatic differentiation of the physical flux and an
    eigendecomposition (independent of the dissipation's formulas)."""
    def fn(u):
        f = fx.physical_flux(u[:, None], G)[:, :, 0]
        return n[0] * f[0] + n[1] * f[1] + n[2] * f[2]
    A = torch.autograd.functional.jacobian(fn, U)
    lam, V = torch.linalg.eig(A)
    return (V @ torch.diag(lam.real.abs().to(V.dtype)) @ torch.linalg.inv(V)).real


def test_roe_dissipation_is_roe_to_first_order():
    """For a small jump du the term is -|N| |A| du / 2 to first order: R |Lambda|
    T R^T times dv = (du/dv)^-1 du reproduces |A| only if R and Lambda are the
    eigenpairs of the flux Jacobian and R T R^T = du/dv (Barth's scaling)."""
    g = torch.Generator().manual_seed(21)
    U = rand_states(6, 22)
    for j in range(6):
        u0 = U[:, j].clone()
        N = [float(torch.randn(1, generator=g, dtype=torch.float64)) for _ in range(3)]
        nn = math.sqrt(sum(x * x for x in N))
        du = torch.randn(5, generator=g, dtype=torch.float64)
        eps = 1e-7
        d = fx.roe_dissipation(u0[:, None], (u0 + eps * du)[:, None], [torch.tensor([x]) for x in N], G)[:, 0] / eps
        ref = -0.5 * nn * _flux_jacobian_abs(u0, [x / nn for x in N]) @ du
        assert float((d - ref).abs().max()) < 1e-5 * float(ref.abs().max()), (d, ref)


def test_roe_dissipation_is_entropy_dissipative_and_antisymmetric():
    Ua, Ub = rand_states(800, 23), rand_states(800, 24)
    g = torch.Generator().manual_seed(25)
    N = [torch.randn(800, generator=g, dtype=torch.float64) for _ in range(3)]
    d = fx.roe_dissipation(Ua, Ub, N, G)
    dv = fx.entropy_variables(Ub, G) - fx.entropy_variables(Ua, G)
    assert float((dv * d).sum(0).max()) <= 0.0
    d2 = fx.roe_dissipation(Ub, Ua, [-x for x in N], G)
    assert float((d + d2).abs().max()) < 1e-13 * float(d.abs().max())
    assert float(fx.roe_dissipation(Ua, Ua, N, G).abs().max()) == 0.0


def test_roe_dissipation_two_codings_agree():
    """The extended module's numpy coding, run in FP64, against this one."""
    import numpy as np
    from oracle import extended as X
    Ua, Ub = rand_states(400, 26), rand_states(400, 27)
    g = torch.Generator().manual_seed(28)
    N = [torch.randn(400, generator=g, dtype=torch.float64) for _ in range(3)]
    d = fx.roe_dissipation(Ua, Ub, N, G).numpy()
    x = X.roe(Ua.numpy(), Ub.numpy(), [t.numpy() for t in N], np.float64(G))
    assert np.max(np.abs(d - x)) < 1e-13 * np.max(np.abs(d))
