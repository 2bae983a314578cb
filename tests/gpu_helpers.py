"""Shared helpers of the GPU parity tests: build a GPU solver and the oracle
(FP64 and extended precision) with the same configuration, and compare arrays
element by element with the criterion of oracle.parity."""
import math

import numpy as np
import torch

import oracle
from oracle import extended, parity
from paper_2312_07725_amd import inputs

TWO_PI = 2 * math.pi
G = 1.4


def make_pair(p, ne, beta=0.2, c=0.0, flux=0, diss=0, source=0, lo=0.0, hi=TWO_PI, tile=0):
    from paper_2312_07725_amd.nsfr import NSFR
    if isinstance(ne, int):
        ne = (ne, ne, ne)
    g = NSFR(p, ne, lo=lo, hi=hi, beta=beta, gamma=G, c=c, flux=flux, diss=diss, source=source, tile=tile)
    o = oracle.Scheme(p, ne, lo=lo, hi=hi, beta=beta, gamma=G, c=c, variant=flux, dissipation=int(diss),
                      source=bool(source))
    return g, o


def make_ext(p, ne, beta=0.2, c=0.0, flux=0, diss=0, source=0, lo=0.0, hi=TWO_PI, elements=None,
             dt=np.longdouble):
    """The oracle's definitions in extended precision (dt=np.float64: the same
    code in plain FP64), optionally at sampled elements only."""
    if isinstance(ne, int):
        ne = (ne, ne, ne)
    return extended.SchemeX(p, ne, lo=lo, hi=hi, beta=beta, gamma=G, c=c, variant=flux, dissipation=int(diss),
                            source=bool(source), dt=dt, elements=elements)


def assert_ext(got, ext, ref64, what="", tol=1e-12, factor=2.0):
    """The parity criterion of oracle.parity: per state, the GPU's
    max-normalised error against the extended-precision result is at most
    max(tol, factor x the FP64 oracle's own error). Returns the errors."""
    ok, eg, e64, bound = parity.check(got, ext, ref64, tol, factor)
    msg = f"{what}: {parity.describe(eg, e64, bound)}"
    print(msg)
    assert ok, msg
    return eg, e64


def state(o, kind, seed=0, mach=0.1):
    if kind == "tgv":
        return inputs.tgv_state(o.X, G, mach)
    if kind == "rough":
        return inputs.perturbed_state(o.X, seed)
    if kind == "mms":
        return inputs.mms_initial_state(o.X, G)
    if kind == "const":
        return inputs.constant_state(o.X.shape[1:])
    raise ValueError(kind)


def rel_err(got, ref):
    """Per-state max |got - ref| / max |ref| (element-by-element difference,
    normalised by the state's magnitude)."""
    got = got.detach().double().cpu()
    ref = ref.detach().double().cpu()
    S = ref.shape[0]
    d = (got - ref).abs().reshape(S, -1).amax(1)
    m = ref.abs().reshape(S, -1).amax(1).clamp_min(1e-300)
    return d / m


def assert_parity(got, ref, tol, what=""):
    e = rel_err(got, ref)
    assert bool((e <= tol).all()), f"{what}: per-state relative errors {e.tolist()} exceed {tol}"
    return e


def cuda(t):
    return t.to("cuda").contiguous()
