"""GPU discrete adjoint against the oracle's reverse-mode derivatives, plus
properties that hold at any size (dot-product / finite-difference checks of
the GPU adjoint against the GPU forward)."""
import pytest
import torch

import oracle
from oracle import adjoint as oadj
from gpu_helpers import assert_parity, cuda, make_pair, state
from paper_2312_07725_amd import adjoint, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("c", ["0", "chu"])
@pytest.mark.parametrize("flux", [0, 1])
def test_vjp_parity(p, c, flux, lib):
    cval = 0.0 if c == "0" else oracle.operators.c_hu(p)
    g, o = make_pair(p, (3, 2, 2), beta=0.2, c=cval, flux=flux)
    U = state(o, "rough", seed=p)
    lam = inputs.normal_like(U.shape, 100 + p)
    ref = oadj.vjp(o, U, lam)
    got = g.rhs_vjp(cuda(U), cuda(lam))
    assert_parity(got, ref, 1e-12, f"vjp p={p} c={c} flux={flux}")


def test_vjp_tgv_branch_mix(lib):
    """TGV state (series branch of the log means) on a single element and a
    ragged mesh."""
    for ne in ((1, 1, 1), (2, 3, 1)):
        g, o = make_pair(3, ne, beta=0.2, c=1e-3)
        U = state(o, "tgv")
        lam = inputs.normal_like(U.shape, 7)
        assert_parity(g.rhs_vjp(cuda(U), cuda(lam)), oadj.vjp(o, U, lam), 1e-12, f"vjp tgv {ne}")


def test_autograd_function(lib):
    g, o = make_pair(2, (2, 2, 2), beta=0.2)
    U = cuda(state(o, "rough", seed=1)).requires_grad_(True)
    lam = cuda(inputs.normal_like(U.shape, 2))
    out = adjoint.rhs(U, g)
    (out * lam).sum().backward()
    ref = oadj.vjp(o, U.detach().cpu(), lam.cpu())
    assert_parity(U.grad, ref, 1e-12, "autograd")


def test_vjp_dot_product_full_size(lib):
    """24^3 warped TGV, p = 4: <lam, J w> by a central difference of the GPU
    rhs equals <J^T lam, w> from the GPU adjoint."""
    from paper_2312_07725_amd.nsfr import NSFR
    g = NSFR(4, 24, beta=0.2)
    U = cuda(inputs.tgv_state(g.node_coords().cpu()))
    lam = cuda(inputs.normal_like(U.shape, 1))
    w = cuda(inputs.normal_like(U.shape, 2)) * U.abs()
    gt = g.rhs_vjp(U, lam)
    h = 1e-7
    fd = ((g.rhs(U + h * w) - g.rhs(U - h * w)) * lam).sum() / (2 * h)
    an = (gt * w).sum()
    assert abs(float(fd - an)) < 1e-6 * abs(float(an))


def test_vjp_parity_full_size_24(lib):
    """Adjoint workload, 24^3 warped TGV, p = 4, c = c_HU, every element: the
    GPU VJP against the oracle's reverse-mode VJP of its own rhs, with a random
    lambda (no cancellation in the result, so the plain 1e-12 bar)."""
    from paper_2312_07725_amd.nsfr import NSFR
    c = oracle.operators.c_hu(4)
    g = NSFR(4, 24, beta=0.2, c=c)
    o = oracle.Scheme(4, (24, 24, 24), beta=0.2, c=c)
    U = inputs.tgv_state(o.X)
    lam = inputs.normal_like(U.shape, 1)
    got = g.rhs_vjp(cuda(U), cuda(lam))
    assert_parity(got, oadj.vjp(o, U, lam), 1e-12, "vjp 24^3 p=4")


@pytest.mark.parametrize("c", ["0", "chu"])
def test_rk4_step_vjp_parity(c, lib):
    p = 3
    cval = 0.0 if c == "0" else oracle.operators.c_hu(p)
    g, o = make_pair(p, (2, 2, 3), beta=0.2, c=cval)
    U = state(o, "tgv")
    dt = o.dt(U, 0.1)
    lam = inputs.normal_like(U.shape, 11)
    ref = oadj.rk4_step_vjp(o, U, dt, 0.0, lam)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    got = g.rk4_step_vjp(cuda(U), dtd, cuda(lam))
    assert_parity(got, ref, 1e-12, "rk4 step vjp")
    # in-place form (lam aliases lam_next)
    lam_g = cuda(lam)
    g.rk4_step_vjp(cuda(U), dtd, lam_g, out=lam_g)
    assert_parity(lam_g, ref, 1e-12, "rk4 step vjp in place")


def test_ke_gradient_small_against_oracle(lib):
    p = 2
    g, o = make_pair(p, (2, 2, 2), beta=0.2)
    U0 = state(o, "tgv")
    dt, n = 0.02, 5
    J0, gref = oadj.ke_gradient(o, U0, dt, n)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    ke, lam = adjoint.kinetic_energy_gradient(g, cuda(U0), dtd, n)
    assert abs(float(ke) - J0) < 1e-12 * abs(J0)
    assert_parity(lam, gref, 1e-11, "dJ/dU0")


def test_ke_gradient_fifty_steps_24(lib):
    """Adjoint workload: 24^3 warped TGV, p = 4, gradient of the kinetic
    energy after 50 RK4 steps (dt frozen at step 0) with step checkpoints,
    checked by a central finite difference of the GPU forward along a random
    direction."""
    from paper_2312_07725_amd.nsfr import NSFR
    g = NSFR(4, 24, beta=0.2)
    U0 = cuda(inputs.tgv_state(g.node_coords().cpu()))
    dtd = g.cfl_dt(U0, 0.1)
    n = 50
    ke, lam = adjoint.kinetic_energy_gradient(g, U0, dtd, n)
    d = cuda(inputs.normal_like(U0.shape, 2)) * U0.abs()
    h = 1e-6

    def J(U):
        UN = adjoint.integrate(g, U, dtd, n)
        return float(g.kinetic_energy(UN)[0])

    fd = (J(U0 + h * d) - J(U0 - h * d)) / (2 * h)
    an = float((lam * d).sum())
    assert abs(fd - an) < 1e-6 * abs(an), (fd, an)
