"""Pins for the conservative strong-DG oracle (oracle.dg) and Roe's flux
(CPU only).

What the paper and the mathematics fix:
  * Roe's flux is consistent (f*(u, u) = f(u) . N), antisymmetric under
    (a, b, N) -> (b, a, -N), and has Roe's property A^ (u_b - u_a) =
    (f_b - f_a) . n: for supersonic states (all wave speeds of one sign) it is
    exactly the upwind flux; for a small jump its dissipation is |A(u)| du
    with |A| from a numerical eigendecomposition of the flux Jacobian;
  * the line-wise residual equals the dense form of Eq. cons DG strong;
  * on a Cartesian mesh with the LGL rule and the central flux, strong DG is
    NSFR with the central two-point flux (Sec. 3.3: with a central two-point
    flux the flux-differencing form is the strong conservative form);
  * free-stream preservation (Sec. 6.1) and conservation (Sec. 6.2) on the
    warped mesh, with and without overintegration;
  * the long-double coding (oracle.extended_gl.DGSchemeX) agrees in FP64 and
    conserves at long-double round-off;
  * order p + 1 on the manufactured solution (Sec. 7.1) with Roe's flux.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import dg, gl
from oracle import flux as fx
from oracle.operators import c_hu
from paper_2312_07725_amd import inputs
from test_oracle_flux import _flux_jacobian_abs

G = 1.4


def _rand_states(m, seed):
    g = torch.Generator().manual_seed(seed)
    r = 0.5 + torch.rand(m, generator=g, dtype=torch.float64)
    vel = [torch.randn(m, generator=g, dtype=torch.float64) * 0.5 for _ in range(3)]
    p = 0.4 + torch.rand(m, generator=g, dtype=torch.float64)
    return fx.conservative(r, vel, p, G)


def test_roe_flux_consistency_and_antisymmetry():
    Ua, Ub = _rand_states(500, 1), _rand_states(500, 2)
    g = torch.Generator().manual_seed(3)
    N = [torch.randn(500, generator=g, dtype=torch.float64) for _ in range(3)]
    f = fx.physical_flux(Ua, G)
    assert torch.allclose(fx.roe_flux(Ua, Ua, N, G), sum(f[k] * N[k] for k in range(3)), atol=1e-14, rtol=1e-14)
    a = fx.roe_flux(Ua, Ub, N, G)
    b = fx.roe_flux(Ub, Ua, [-x for x in N], G)
    assert float((a + b).abs().max()) < 1e-13 * float(a.abs().max())


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_roe_flux_is_upwind_for_supersonic_states(sign):
    """Roe's property: with every wave speed of one sign, |A^| = +-A^ and the
    flux is the upwind physical flux exactly (to rounding). This holds only if
    the averages, eigenvectors and wave strengths are all right."""
    g = torch.Generator().manual_seed(4)
    m = 200
    n = torch.nn.functional.normalize(torch.randn(3, m, generator=g, dtype=torch.float64), dim=0)
    r = 0.8 + 0.4 * torch.rand(m, generator=g, dtype=torch.float64)
    p = 0.7 + 0.3 * torch.rand(m, generator=g, dtype=torch.float64)
    c = torch.sqrt(G * p / r)
    vel = [sign * 3.0 * c * n[k] + 0.1 * torch.randn(m, generator=g, dtype=torch.float64) for k in range(3)]
    Ua = fx.conservative(r, vel, p, G)
    Ub = fx.conservative(r * 1.05, [v * 1.02 for v in vel], p * 0.97, G)
    N = [2.0 * n[k] for k in range(3)]
    up = Ua if sign > 0 else Ub
    f = fx.physical_flux(up, G)
    ref = sum(f[k] * N[k] for k in range(3))
    got = fx.roe_flux(Ua, Ub, N, G)
    assert float((got - ref).abs().max()) < 1e-13 * float(ref.abs().max())


def test_roe_flux_small_jump_is_abs_jacobian():
    g = torch.Generator().manual_seed(5)
    U = _rand_states(4, 6)
    for j in range(4):
        u0 = U[:, j].clone()
        N = [float(torch.randn(1, generator=g, dtype=torch.float64)) for _ in range(3)]
        nn = math.sqrt(sum(x * x for x in N))
        du = torch.randn(5, generator=g, dtype=torch.float64)
        eps = 1e-7
        Nt = [torch.tensor([x], dtype=torch.float64) for x in N]
        f0 = fx.physical_flux(u0[:, None], G)
        f1 = fx.physical_flux((u0 + eps * du)[:, None], G)
        central = 0.5 * sum((f0[k] + f1[k]) * N[k] for k in range(3))[:, 0]
        d = (fx.roe_flux(u0[:, None], (u0 + eps * du)[:, None], Nt, G)[:, 0] - central) / eps
        ref = -0.5 * nn * _flux_jacobian_abs(u0, [x / nn for x in N]) @ du
        assert float((d - ref).abs().max()) < 1e-5 * float(ref.abs().max())


@pytest.mark.parametrize("p,overint", [(2, 0), (2, 3), (3, 1), (4, 0)])
def test_linewise_equals_definition(p, overint):
    s = dg.DGScheme(p, (2, 1, 2), beta=0.2, overint=overint)
    U = inputs.perturbed_state(s.X, seed=7)
    R1 = dg.residual(s.mesh, s.ops, U, G)
    R2 = dg.residual_definition(s.mesh, s.ops, U, G)
    assert float((R1 - R2).abs().max()) < 1e-13 * float(R2.abs().max())


@pytest.mark.parametrize("p", [2, 3])
def test_central_flux_reduces_to_nsfr_on_cartesian_lgl(p):
    def central(a, b, N):
        fa, fb = fx.physical_flux(a, G), fx.physical_flux(b, G)
        return 0.5 * sum((fa[k] + fb[k]) * N[k] for k in range(3))
    s = dg.DGScheme(p, (2, 2, 1), beta=0.0, quad="lgl")
    U = inputs.perturbed_state(s.X, seed=3)
    Rd = dg.residual(s.mesh, s.ops, U, G, numflux=central)
    Rn = gl.residual(s.mesh, s.ops, U, G, two_point=central)
    assert float((Rd - Rn).abs().max()) < 1e-13 * float(Rn.abs().max())


@pytest.mark.parametrize("p,overint", [(2, 0), (3, 4), (5, 1)])
def test_free_stream_and_conservation(p, overint):
    s = dg.DGScheme(p, (2, 2, 3), beta=0.2, overint=overint)
    Uc = inputs.constant_state(s.mesh.base.J.shape)
    R = s.residual(Uc)
    scale = (float(fx.physical_flux(Uc, G).abs().max()) * float(s.mesh.Cq.abs().max())
             * float(s.ops.Dq.abs().max()))
    assert float(R.abs().max()) < 1e-13 * scale
    U = inputs.perturbed_state(s.X, seed=p)
    R = s.residual(U)
    tot = R.reshape(5, -1).sum(1)
    mag = R.abs().reshape(5, -1).sum(1)
    assert bool((tot.abs() <= 1e-13 * mag).all())


@pytest.mark.parametrize("p,overint", [(2, 0), (3, 4)])
def test_extended_dg_agrees_and_conserves(p, overint):
    from oracle import extended_gl as XG
    c = c_hu(p)
    s = dg.DGScheme(p, (2, 3, 2), beta=0.2, overint=overint, c=c, source=True)
    x = XG.DGSchemeX(p, (2, 3, 2), beta=0.2, overint=overint, c=c, source=True, dt=np.float64)
    U = inputs.perturbed_state(s.X, seed=4)
    a = s.rhs(U, 0.2).numpy()
    assert np.max(np.abs(a - x.rhs(U.numpy(), 0.2))) < 1e-13 * np.max(np.abs(a))
    xl = XG.DGSchemeX(p, (2, 3, 2), beta=0.2, overint=overint)
    R = xl.residual(U.numpy())
    assert np.all(np.abs(R.reshape(5, -1).sum(1)) <= 1e-17 * np.abs(R).reshape(5, -1).sum(1))
    ids = [0, 5, 11]
    xs = XG.DGSchemeX(p, (2, 3, 2), beta=0.2, overint=overint, elements=ids)
    assert np.max(np.abs(xs.residual(U.numpy()) - R[:, ids])) == 0.0


def test_mms_order_of_accuracy_dg():
    """Sec. 7.1 with conservative DG and Roe's flux on the GL rule: order p + 1
    for p = 2 (c = 0, slightly warped periodic mesh, t_f = 0.5)."""
    p, tf = 2, 0.5
    errs = []
    for ne in (3, 6):
        s = dg.DGScheme(p, (ne, ne, ne), lo=-1.0, hi=1.0, beta=0.002, source=True)
        U = inputs.mms_initial_state(s.X, G)
        dx = 2.0 / (ne * (p + 1))
        nsteps = int(math.ceil(tf / (0.3 * dx / 3.0)))
        dt = tf / nsteps
        t = 0.0
        for _ in range(nsteps):
            U = oracle.timestep.rk4_step(s.rhs, U, dt, t)
            t += dt
        err = oracle.problems.l2_error(s.mesh.base, U, oracle.problems.mms_state(s.X, tf, G))
        errs.append(float(err[0]))
    rate = math.log2(errs[0] / errs[1])
    assert rate > p + 0.7, (errs, rate)
