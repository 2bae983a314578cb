"""GPU parity of the forward path against the CPU oracle (element by element).

Tolerance: every entry differs from the oracle's by at most 1e-12 times the
state's round-off scale, the largest over the mesh of the sum of the
magnitudes of the terms the residual adds at a node (and of |A| applied to it
for dU/dt). For rough states the plain max-normalised error
is checked at 1e-12 as well. For smooth Mach-0.1 states max |R| is up to 1e5
times smaller than the terms that cancel in it (the TGV density residual is
pure truncation error), so normalising by it would measure the conditioning
of the cancellation, not the arithmetic. Cases span p = 2..5,
ragged element counts (so the last workgroup is partial), the single-element
periodic mesh, both two-point flux variants, c = 0 and c = c_HU (weight-
adjusted inverse with the rank-one FR projection), the dissipative surface
flux with the manufactured source, and the full 16^3 TGV meshes.
"""
import math

import pytest
import torch

import oracle
from gpu_helpers import assert_parity, assert_parity_scaled, cuda, make_pair, state, G

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_geometry(p, lib):
    g, o = make_pair(p, (2, 3, 2), beta=0.2)
    X = g.node_coords()
    C, J = g.geometry()
    torch.cuda.synchronize()
    assert_parity(X.reshape(3, -1), o.mesh.X.reshape(3, -1), 1e-14, "coords")
    assert_parity(J.reshape(1, -1), o.mesh.J.reshape(1, -1), 1e-13, "J")
    # normalised by the largest metric entry: some entries vanish identically
    # on coarse meshes and carry only round-off on either side
    err = float((C.cpu() - o.mesh.C).abs().max() / o.mesh.C.abs().max())
    assert err < 1e-12, err


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("kind", ["tgv", "rough"])
@pytest.mark.parametrize("flux", [0, 1])
def test_residual_small(p, kind, flux, lib):
    g, o = make_pair(p, (3, 2, 4), beta=0.2, flux=flux)
    U = state(o, kind, seed=p)
    R = g.residual(cuda(U))
    assert_parity_scaled(R, o.residual(U), o.residual_scale(U), TOL, f"residual p={p} {kind} flux={flux}")
    if kind == "rough":
        assert_parity(R, o.residual(U), TOL, f"residual p={p} {kind} flux={flux}")


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("c", ["0", "chu"])
def test_rhs_small(p, c, lib):
    cval = 0.0 if c == "0" else oracle.operators.c_hu(p)
    g, o = make_pair(p, (2, 3, 2), beta=0.2, c=cval)
    U = state(o, "rough", seed=10 + p)
    assert_parity(g.rhs(cuda(U)), o.rhs(U), TOL, f"rhs p={p} c={c}")
    Ut = state(o, "tgv")
    assert_parity_scaled(g.rhs(cuda(Ut)), o.rhs(Ut), o.rhs_scale(Ut), TOL, f"rhs tgv p={p} c={c}")


@pytest.mark.parametrize("p", [2, 3])
def test_single_element_periodic(p, lib):
    g, o = make_pair(p, (1, 1, 1), beta=0.2, c=oracle.operators.c_hu(p))
    U = state(o, "rough", seed=3)
    assert_parity(g.rhs(cuda(U)), o.rhs(U), TOL, "1 element")


@pytest.mark.parametrize("p", [2, 4])
def test_mms_source_and_dissipation(p, lib):
    g, o = make_pair(p, (3, 2, 2), beta=0.02, lo=-1.0, hi=1.0, diss=1, source=1, c=oracle.operators.c_hu(p))
    U = state(o, "mms")
    t = 0.37
    assert_parity_scaled(g.residual(cuda(U), t=t), o.residual(U, t), o.residual_scale(U, t), TOL, "mms residual")
    assert_parity_scaled(g.rhs(cuda(U), t=t), o.rhs(U, t), o.rhs_scale(U, t), TOL, "mms rhs")


@pytest.mark.parametrize("p", [3, 4, 5])
def test_full_size_tgv_16(p, lib):
    """16^3 warped TGV (beta = 1/5), c = c_HU, in the launch configuration the
    benchmark times (default tile)."""
    g, o = make_pair(p, 16, beta=0.2, c=oracle.operators.c_hu(p))
    U = state(o, "tgv")
    got = g.rhs(cuda(U))
    e = assert_parity_scaled(got, o.rhs(U), o.rhs_scale(U), TOL, f"16^3 p={p} rhs")
    print(f"16^3 p={p}: scaled errors {e.tolist()}")
    R = g.residual(cuda(U))
    assert_parity_scaled(R, o.residual(U), o.residual_scale(U), TOL, f"16^3 p={p} residual")


def test_tiles_and_determinism(lib):
    p = 3
    from paper_2312_07725_amd.nsfr import NSFR
    ref = None
    o = oracle.Scheme(p, (3, 5, 2), beta=0.2, c=1e-3)
    U = cuda(state(o, "rough", seed=5))
    for tile in (1, 2, 3, 4, 5, 7):
        g = NSFR(p, (3, 5, 2), beta=0.2, c=1e-3, tile=tile)
        out = g.rhs(U)
        again = g.rhs(U)
        torch.cuda.synchronize()
        assert torch.equal(out, again)
        if ref is None:
            ref = out
        assert torch.equal(out, ref), f"tile {tile} changes the result"


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_invariants_on_gpu(p, lib):
    """Sec. 5: free-stream preservation, global conservation and entropy
    conservation of the GPU residual on the warped periodic mesh."""
    g, o = make_pair(p, (3, 3, 2), beta=0.2)
    Uc = state(o, "const")
    Rc = g.residual(cuda(Uc))
    f = oracle.flux.physical_flux(Uc, G)
    scale = float(f.abs().max() * o.mesh.C.abs().max() * o.mesh.ops.S1.abs().max())
    assert float(Rc.abs().max()) < 1e-13 * scale
    U = state(o, "tgv")
    d = g.diagnostics(cuda(U)).cpu()
    assert abs(float(d[0])) < 1e-13 * float(d[1])      # entropy
    R = g.residual(cuda(U)).cpu()
    mag = R.abs().reshape(5, -1).sum(1)
    assert bool((d[2:7].abs() <= 1e-13 * mag).all())   # conservation
    assert abs(float(d[7]) - float(R.abs().max())) == 0.0


def test_wavespeed_cfl_and_kinetic_energy(lib):
    g, o = make_pair(3, (2, 3, 4), beta=0.2)
    U = state(o, "tgv")
    lam = float(g.max_wavespeed(cuda(U)))
    assert abs(lam - o.max_wavespeed(U)) < 1e-14 * lam
    dt = float(g.cfl_dt(cuda(U), 0.1))
    assert abs(dt - o.dt(U, 0.1)) < 1e-14 * dt
    grad = g.empty()
    ke, _ = g.kinetic_energy(cuda(U), grad=grad)
    from oracle import adjoint as adj
    Ud = U.clone().requires_grad_(True)
    J = adj.kinetic_energy_objective(o, Ud)
    (gref,) = torch.autograd.grad(J, Ud)
    assert abs(float(ke) - float(J)) < 1e-13 * abs(float(J))
    assert_parity(grad, gref, 1e-13, "dJ/dU")


def test_check_state(lib):
    g, o = make_pair(2, (2, 2, 2), beta=0.0)
    U = state(o, "tgv")
    assert g.check_state(cuda(U)) == 0
    Ub = U.clone()
    Ub[0, 1, 0, 0, 0] = -1.0
    Ub[4, 3, 1, 1, 1] = 0.0
    assert g.check_state(cuda(Ub)) == 2


def test_rejects_bad_tensors(lib):
    g, o = make_pair(2, (2, 2, 2))
    U = cuda(state(o, "tgv"))
    with pytest.raises(TypeError):
        g.rhs(U.float())
    with pytest.raises(ValueError):
        g.rhs(U[:, :4].contiguous())
    from paper_2312_07725_amd.nsfr import NSFRError
    with pytest.raises(NSFRError):
        g.rhs(U, out=U)   # aliasing is rejected by the library
