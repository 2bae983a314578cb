"""GPU RK4 against the oracle, HIP-graph replay, and entropy along long runs.

Trajectory parity: after K steps the increment U_K - U_0 of the GPU must match
that of the extended-precision RK4 trajectory under the criterion of
oracle.parity (per state, max-normalised error of the increment at most
max(1e-12, 2 x the FP64 oracle trajectory's own error)). Comparing increments
rather than states keeps the bar relative to what the steps compute."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_ext, cuda, make_ext, make_pair, state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("beta", [0.1, 0.2])
@pytest.mark.parametrize("c", ["0", "chu"])
def test_rk4_ten_steps_tgv_4cubed(beta, c, lib):
    """TGV, 4^3 warped elements, p = 3, 1 rhs + 10 RK4 steps (CFL 0.1)."""
    p = 3
    cval = 0.0 if c == "0" else oracle.operators.c_hu(p)
    g, o = make_pair(p, 4, beta=beta, c=cval)
    xs = make_ext(p, 4, beta=beta, c=cval)
    x64 = make_ext(p, 4, beta=beta, c=cval, dt=np.float64)
    U0 = state(o, "tgv")
    assert_ext(g.rhs(cuda(U0)), xs.rhs(U0.numpy()), [o.rhs(U0), x64.rhs(U0.numpy())], "rhs")
    dt = o.dt(U0, 0.1)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    Ug = cuda(U0)
    Uo = U0.clone()
    Ux = U0.numpy().astype(np.longdouble)
    U6 = U0.numpy()
    work = g.work(3)
    for i in range(10):
        g.rk4_step(Ug, dtd, i * dt, work)
        Uo = o.rk4_step(Uo, dt, i * dt)
        Ux = xs.rk4_step(Ux, dt, i * dt)
        U6 = x64.rk4_step(U6, dt, i * dt)
    U0x = U0.numpy().astype(np.longdouble)
    assert_ext(Ug.cpu().numpy().astype(np.longdouble) - U0x, Ux - U0x,
               [Uo.numpy().astype(np.longdouble) - U0x, U6.astype(np.longdouble) - U0x], "10 steps, increment")


def test_rk4_mms_time_dependent_source(lib):
    p = 3
    kw = dict(beta=0.02, lo=-1.0, hi=1.0, diss=1, source=1, c=oracle.operators.c_hu(p))
    g, o = make_pair(p, (3, 3, 2), **kw)
    xs = make_ext(p, (3, 3, 2), **kw)
    x64 = make_ext(p, (3, 3, 2), dt=np.float64, **kw)
    U0 = state(o, "mms")
    dt = 0.004
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    Ug, Uo = cuda(U0), U0.clone()
    Ux = U0.numpy().astype(np.longdouble)
    U6 = U0.numpy()
    for i in range(5):
        g.rk4_step(Ug, dtd, 0.1 + i * dt)
        Uo = o.rk4_step(Uo, dt, 0.1 + i * dt)
        Ux = xs.rk4_step(Ux, dt, 0.1 + i * dt)
        U6 = x64.rk4_step(U6, dt, 0.1 + i * dt)
    U0x = U0.numpy().astype(np.longdouble)
    assert_ext(Ug.cpu().numpy().astype(np.longdouble) - U0x, Ux - U0x,
               [Uo.numpy().astype(np.longdouble) - U0x, U6.astype(np.longdouble) - U0x], "mms 5 steps, increment")


def test_graph_replay_equals_steps(lib):
    p = 4
    g, o = make_pair(p, (3, 2, 3), beta=0.02, c=oracle.operators.c_hu(p), diss=1, source=1, lo=-1.0, hi=1.0)
    U0 = cuda(state(o, "mms"))
    dtd = torch.tensor([0.003], dtype=torch.float64, device="cuda")
    A = U0.clone()
    work = g.work(3)
    for i in range(7):
        g.rk4_step(A, dtd, 0.2 + i * 0.003, work)
    B = U0.clone()
    t = torch.tensor([0.2], dtype=torch.float64, device="cuda")
    work2 = g.work(3)
    g.rk4_run(B, dtd, t, 3, work2)
    torch.cuda.synchronize()
    g.rk4_run(B, dtd, t, 4, work2)   # replays the same graph with eager work in between
    torch.cuda.synchronize()
    assert abs(float(t) - (0.2 + 7 * 0.003)) < 1e-15
    assert torch.equal(A, B)


@pytest.mark.parametrize("p", [3, 4])
def test_hundred_steps_entropy_16(p, lib):
    """16^3 warped TGV, 100 RK4 steps: the semi-discrete entropy rate stays at
    round-off at every step (paper Sec. 7.3 reports O(1e-13))."""
    from paper_2312_07725_amd import inputs
    g, o = make_pair(p, 16, beta=0.2, c=oracle.operators.c_hu(p))
    U = cuda(inputs.tgv_state(g.node_coords().cpu()))
    dtd = g.cfl_dt(U, 0.1)
    work = g.work(3)
    worst = 0.0
    for i in range(100):
        g.rk4_step(U, dtd, 0.0, work)
        if i % 10 == 9:
            d = g.diagnostics(U).cpu()
            worst = max(worst, abs(float(d[0])) / float(d[1]))
    assert worst < 1e-13
    assert g.check_state(U) == 0
