"""Pins for the oracle's derivatives (CPU only).

The reverse-mode VJP of the oracle is checked against independent routes:
the complex-step JVP (dot-product test and the full Jacobian of a tiny mesh),
central finite differences, and for the RK4 discrete adjoint the complex step
through a whole step and a finite difference of the kinetic-energy objective.
"""
import pytest
import torch

import oracle
from oracle import adjoint as adj
from paper_2312_07725_amd import inputs


def scheme(p=2, ne=(2, 1, 2), c=0.0, variant=0):
    return oracle.Scheme(p, ne, beta=0.2, c=c, variant=variant)


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("c", [0.0, 1e-3])
@pytest.mark.parametrize("variant", [0, 1])
def test_vjp_dot_product_with_complex_step(p, c, variant):
    s = scheme(p, (2, 2, 1), c, variant)
    U = inputs.perturbed_state(s.X, seed=5)
    lam = inputs.normal_like(U.shape, 6)
    g = adj.vjp(s, U, lam)
    for seed in (7, 8):
        w = inputs.normal_like(U.shape, seed)
        Jw = adj.jvp_complex_step(s, U, w)
        lhs, rhs = float((lam * Jw).sum()), float((g * w).sum())
        scale = float((lam * Jw).abs().sum())
        assert abs(lhs - rhs) < 1e-12 * scale


def test_vjp_equals_transposed_complex_step_jacobian():
    s = scheme(2, (2, 1, 1), 1e-3)
    U = inputs.perturbed_state(s.X, seed=9)
    lam = inputs.normal_like(U.shape, 10)
    g = adj.vjp(s, U, lam)
    nd = U.numel()
    gref = torch.zeros(nd, dtype=torch.float64)
    lamf = lam.reshape(-1)
    for j in range(nd):
        e = torch.zeros(nd, dtype=torch.float64)
        e[j] = 1.0
        col = adj.jvp_complex_step(s, U, e.reshape(U.shape)).reshape(-1)
        gref[j] = (lamf * col).sum()
    assert float((g.reshape(-1) - gref).abs().max()) < 1e-12 * float(gref.abs().max())


def test_complex_step_matches_finite_difference():
    s = scheme(2, (2, 2, 1))
    U = inputs.perturbed_state(s.X, seed=11)
    w = inputs.normal_like(U.shape, 12) * 1e-3
    Jw = adj.jvp_complex_step(s, U, w)
    h = 1e-5
    fd = (s.rhs(U + h * w) - s.rhs(U - h * w)) / (2 * h)
    assert float((Jw - fd).abs().max()) < 1e-7 * float(Jw.abs().max())


def test_rk4_step_vjp_dot_product():
    s = scheme(2, (2, 2, 1), 1e-3)
    U = inputs.perturbed_state(s.X, seed=13)
    dt = 0.01
    lam = inputs.normal_like(U.shape, 14)
    w = inputs.normal_like(U.shape, 15)
    g = adj.rk4_step_vjp(s, U, dt, 0.0, lam)
    Uc = U.to(torch.complex128) + 1j * 1e-30 * w
    Jw = s.rk4_step(Uc, dt).imag / 1e-30
    lhs, rhs = float((lam * Jw).sum()), float((g * w).sum())
    assert abs(lhs - rhs) < 1e-12 * float((lam * Jw).abs().sum())


def test_ke_gradient_against_finite_difference():
    s = oracle.Scheme(2, (2, 2, 2), beta=0.2)
    U0 = inputs.tgv_state(s.X)
    dt, n = 0.02, 3
    J0, g = adj.ke_gradient(s, U0, dt, n)
    d = inputs.normal_like(U0.shape, 16) * U0.abs()
    h = 1e-6

    def J(U):
        for i in range(n):
            U = s.rk4_step(U, dt, i * dt)
        return float(adj.kinetic_energy_objective(s, U))

    fd = (J(U0 + h * d) - J(U0 - h * d)) / (2 * h)
    an = float((g * d).sum())
    assert abs(fd - an) < 1e-7 * abs(an)
