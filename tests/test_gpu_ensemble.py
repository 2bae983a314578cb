"""Ensembles of independent flows of differing degree and size in one launch
per RK stage: every flow must equal its own single-flow GPU run (the kernel
body and the per-element arithmetic are the same, so the result is bitwise
identical) and the oracle (criterion of oracle.parity against the
extended-precision evaluation)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_ext, cuda, make_ext
from paper_2312_07725_amd import inputs

pytestmark = pytest.mark.gpu


def flows_small():
    # (p, ne, mach, c, flux)
    return [(5, (2, 1, 2), 0.1, "chu", 0), (2, (3, 2, 2), 0.3, "0", 0), (3, (2, 3, 1), 0.05, "chu", 1),
            (4, (1, 2, 2), 0.2, "0", 1), (3, (1, 1, 1), 0.1, "0", 0), (2, (4, 1, 1), 0.15, "chu", 0)]


def build(flows, beta=0.2):
    from paper_2312_07725_amd.nsfr import Ensemble, NSFR, make_config
    cfgs, singles, orcs, states = [], [], [], []
    for (p, ne, mach, c, flux) in flows:
        cv = oracle.operators.c_hu(p) if c == "chu" else 0.0
        cfgs.append(make_config(p, ne, beta=beta, c=cv, flux=flux))
        singles.append(NSFR(p, ne, beta=beta, c=cv, flux=flux))
        o = oracle.Scheme(p, ne, beta=beta, c=cv, variant=flux)
        orcs.append(o)
        states.append(inputs.tgv_state(o.X, 1.4, mach))
    ens = Ensemble(cfgs)
    U = ens.empty()
    for i, s in enumerate(states):
        ens.flow_view(U, i).copy_(s)
    return ens, singles, orcs, states, U


def test_ensemble_rhs(lib):
    ens, singles, orcs, states, U = build(flows_small())
    out = ens.rhs(U)
    torch.cuda.synchronize()
    for i, (g, o, s) in enumerate(zip(singles, orcs, states)):
        single = g.rhs(cuda(s))
        assert torch.equal(ens.flow_view(out, i), single), f"flow {i} differs from its single-flow run"
        p, ne, mach, c, flux = flows_small()[i]
        cv = oracle.operators.c_hu(p) if c == "chu" else 0.0
        xs = make_ext(p, ne, beta=0.2, c=cv, flux=flux)
        x64 = make_ext(p, ne, beta=0.2, c=cv, flux=flux, dt=np.float64)
        assert_ext(ens.flow_view(out, i), xs.rhs(s.numpy()), [o.rhs(s), x64.rhs(s.numpy())], f"flow {i}")


def test_ensemble_rk4_step_and_graph(lib):
    ens, singles, orcs, states, U = build(flows_small())
    dts = torch.tensor([o.dt(s, 0.1) for o, s in zip(orcs, states)], dtype=torch.float64, device="cuda")
    A = U.clone()
    for _ in range(3):
        ens.rk4_step(A, dts)
    B = U.clone()
    ens.rk4_run(B, dts, 2)
    torch.cuda.synchronize()
    ens.rk4_run(B, dts, 1)
    torch.cuda.synchronize()
    assert torch.equal(A, B)
    for i, (g, s) in enumerate(zip(singles, states)):
        Ug = cuda(s)
        for _ in range(3):
            g.rk4_step(Ug, dts[i:i + 1].contiguous())
        assert torch.equal(ens.flow_view(A, i), Ug), f"flow {i}"


def test_ensemble_tiles(lib):
    ens, singles, orcs, states, U = build(flows_small())
    ref = ens.rhs(U).clone()
    for p, epb in ((2, 3), (3, 1), (4, 1), (5, 1)):
        ens.set_tile(p, epb)
        assert torch.equal(ens.rhs(U), ref)


def test_ensemble_64_flows(lib):
    """The ensemble workload: 64 warped TGV flows, 6^3-12^3 elements, p drawn
    from {2, 3, 4, 5}, Mach 0.05-0.3 (seed 0), c = c_HU(p); one RK4 step from
    the graph equals the single-flow runs; the ensemble rhs of every flow is
    compared with the oracle at 8 sampled elements per flow (seeded, including
    the flow's first and last element)."""
    from paper_2312_07725_amd.nsfr import Ensemble, NSFR, make_config
    draws = inputs.ensemble_draws(64, seed=0)
    cfgs = [make_config(p, ne, beta=0.2, c=oracle.operators.c_hu(p)) for (ne, p, m) in draws]
    ens = Ensemble(cfgs)
    U = ens.empty()
    singles = []
    for i, (ne, p, mach) in enumerate(draws):
        g = NSFR(p, ne, beta=0.2, c=oracle.operators.c_hu(p))
        X = g.node_coords().cpu()
        ens.flow_view(U, i).copy_(inputs.tgv_state(X, 1.4, mach))
        singles.append(g)
    dts = torch.empty(64, dtype=torch.float64, device="cuda")
    for i, g in enumerate(singles):
        g.cfl_dt(ens.flow_view(U, i).contiguous(), 0.1, out=dts[i:i + 1])
    U0 = U.clone()
    ens.rk4_run(U, dts, 1)
    torch.cuda.synchronize()
    for i, g in enumerate(singles):
        Ug = ens.flow_view(U0, i).contiguous().clone()
        g.rk4_step(Ug, dts[i:i + 1].contiguous())
        assert torch.equal(ens.flow_view(U, i), Ug), f"flow {i}"
    out = ens.rhs(U0).cpu()
    U0c = U0.cpu()
    rng = np.random.default_rng(0)
    for i, (ne, p, mach) in enumerate(draws):
        E = ne ** 3
        els = np.unique(np.concatenate([[0, E - 1], rng.choice(E, 6, replace=False)]))
        c = oracle.operators.c_hu(p)
        Ui = ens.flow_view(U0c, i).numpy()
        xs = make_ext(p, ne, beta=0.2, c=c, elements=els)
        x64 = make_ext(p, ne, beta=0.2, c=c, elements=els, dt=np.float64)
        assert_ext(ens.flow_view(out, i)[:, els], xs.rhs(Ui), x64.rhs(Ui), f"flow {i} (ne={ne}, p={p}, M={mach:.3f})")
