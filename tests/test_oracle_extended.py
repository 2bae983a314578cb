"""Pins for the extended-precision evaluation of the oracle (CPU only).

The extended module is a second, independent coding of the oracle's
definitions (numpy, its own solver) run in x87 long double. It is pinned by:
  * LGL closed forms to long-double accuracy (tests/golden/lgl_closed_forms.json);
  * the same code in plain FP64 agreeing with the PyTorch FP64 oracle on
    rough states (two codings of one definition);
  * free-stream preservation, global conservation and entropy conservation of
    its residual at long-double round-off (Sec. 6.1-6.3), a thousand times
    below what FP64 reaches, which shows that its extra digits are real;
  * the weight-adjusted inverse in its rank-one closed form (Sec. 4);
  * sampled-element evaluation equal to the full-mesh evaluation.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import extended as X
from paper_2312_07725_amd import inputs

LD = np.longdouble
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _ld(s):
    """Evaluate a closed form such as 'sqrt(3/7)' with 40-digit mpmath and
    round it to long double."""
    import re
    import mpmath
    mpmath.mp.dps = 40
    v = eval(re.sub(r"(\d+)", r"mpf(\1)", s), {"sqrt": mpmath.sqrt, "mpf": mpmath.mpf}, {})
    return LD(mpmath.nstr(v, 30))


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_lgl_long_double_closed_forms(p):
    g = json.load(open(os.path.join(GOLD, "lgl_closed_forms.json")))["rules"][str(p)]
    ops = X.Ops1D(p)
    xr = np.array([_ld(s) for s in g["x"]], dtype=LD)
    wr = np.array([_ld(s) for s in g["w"]], dtype=LD)
    assert np.max(np.abs(ops.x - xr)) < LD(1e-18)
    assert np.max(np.abs(ops.w - wr)) < LD(1e-18)


@pytest.mark.parametrize("p", [2, 3, 5])
def test_fp64_coding_agrees_with_oracle(p):
    c = oracle.operators.c_hu(p)
    for variant in (0, 1):
        o = oracle.Scheme(p, (2, 3, 2), beta=0.2, c=c, variant=variant)
        x = X.SchemeX(p, (2, 3, 2), beta=0.2, c=c, variant=variant, dt=np.float64)
        U = inputs.perturbed_state(o.X, seed=p)
        R = o.rhs(U).numpy()
        d = np.abs(x.rhs(U.numpy()) - R).reshape(5, -1).max(1) / np.abs(R).reshape(5, -1).max(1)
        assert np.all(d < 1e-13), d


@pytest.mark.parametrize("p", [2, 3, 4])
def test_extended_invariants(p):
    x = X.SchemeX(p, (3, 2, 2), beta=0.2)
    Uc = inputs.constant_state((5, 3 * 2 * 2, p + 1, p + 1, p + 1)[1:]).numpy()
    Rc = x.residual(Uc)
    scale = float(np.max(np.abs(x.mesh.C))) * 3.0     # |f| ~ 3 for this constant state, |S1| ~ 1
    assert float(np.max(np.abs(Rc))) < 1e-17 * scale
    U = inputs.tgv_state(torch.tensor(X.MeshX(p, (3, 2, 2), beta=0.2, dt=np.float64).X)).numpy()
    R = x.residual(U)
    rho, vel, pr, beta = X.primitives(U.astype(LD), x.gamma)
    s = np.log(pr) - x.gamma * np.log(rho)
    q2 = vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2
    v = np.stack([(x.gamma - s) / (x.gamma - 1) - beta * q2, 2 * beta * vel[0], 2 * beta * vel[1],
                  2 * beta * vel[2], -2 * beta])
    vr = v * R
    assert abs(float(vr.sum())) < 1e-16 * float(np.abs(vr).sum())                    # entropy
    tot = R.reshape(5, -1).sum(1)
    mag = np.abs(R).reshape(5, -1).sum(1)
    assert np.all(np.abs(tot) < 1e-16 * mag)                                          # conservation


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_extended_projection_rank_one(p):
    """Pi~ = I - alpha W^-1 d d^T with d = p! lambda, alpha = 2c / (1 + 2c d^T W^-1 d)
    (Sec. 4 with the rank-one K of Eq. Km)."""
    c = 1e-3
    ops = X.Ops1D(p, c)
    x = ops.x
    n = p + 1
    lam = np.array([LD(1) / np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)], dtype=LD)
    d = LD(math.factorial(p)) * lam
    mu = np.sum(d * d / ops.w)
    alpha = 2 * LD(c) / (1 + 2 * LD(c) * mu)
    Pi = np.eye(n, dtype=LD) - alpha * np.outer(d / ops.w, d)
    # the dense solve of W + K loses digits in proportion to its condition
    # number, about 1 + 2 c mu (4.5e3 at p = 5)
    cond = 1 + 2 * LD(c) * mu
    assert np.max(np.abs(ops.Pi - Pi)) < 8 * np.finfo(LD).eps * cond * np.max(np.abs(Pi))


def test_extended_is_closer_than_fp64_on_smooth_state():
    """On the smoke workload the FP64 oracle and the FP64 coding of the
    extended module differ from each other by about as much as each differs
    from the long-double result, and the long-double result changes by orders
    of magnitude less when its metric terms are rounded to FP64: the
    discrepancy is FP64 round-off, not a difference of definitions."""
    c = oracle.operators.c_hu(3)
    o = oracle.Scheme(3, (2, 3, 2), beta=0.2, c=c)
    U = inputs.tgv_state(o.X)
    xs = X.SchemeX(3, (2, 3, 2), beta=0.2, c=c)
    ext = xs.rhs(U.numpy())
    m = np.abs(ext).reshape(5, -1).max(1)
    e64 = (np.abs(o.rhs(U).numpy() - ext).reshape(5, -1).max(1) / m).astype(float)
    xs.mesh.C = xs.mesh.C.astype(np.float64).astype(LD)
    eC = (np.abs(xs.rhs(U.numpy()) - ext).reshape(5, -1).max(1) / m).astype(float)
    assert np.all(eC < 0.1 * np.maximum(e64, 1e-14)), (eC, e64)
    assert e64[1] > 1e-12   # the momentum residual is ill-conditioned in FP64


def test_sampled_elements_equal_full_mesh():
    c = oracle.operators.c_hu(4)
    ne = (3, 2, 4)
    full = X.SchemeX(4, ne, beta=0.2, c=c)
    U = inputs.tgv_state(torch.tensor(full.mesh.X.astype(np.float64))).numpy()
    R = full.rhs(U)
    els = [0, 5, 23, 11]
    sub = X.SchemeX(4, ne, beta=0.2, c=c, elements=els).rhs(U)
    assert np.array_equal(sub, R[:, els])
