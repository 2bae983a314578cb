"""Shared helpers of the GPU parity tests: build a GPU solver and the oracle
with the same configuration, and compare arrays element by element."""
import math

import torch

import oracle
from paper_2312_07725_amd import inputs

TWO_PI = 2 * math.pi
G = 1.4


def make_pair(p, ne, beta=0.2, c=0.0, flux=0, diss=0, source=0, lo=0.0, hi=TWO_PI, tile=0):
    from paper_2312_07725_amd.nsfr import NSFR
    if isinstance(ne, int):
        ne = (ne, ne, ne)
    g = NSFR(p, ne, lo=lo, hi=hi, beta=beta, gamma=G, c=c, flux=flux, diss=diss, source=source, tile=tile)
    o = oracle.Scheme(p, ne, lo=lo, hi=hi, beta=beta, gamma=G, c=c, variant=flux, dissipation=bool(diss),
                      source=bool(source))
    return g, o


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


def assert_parity_scaled(got, ref, scale, tol, what=""):
    """Element-by-element parity in the normwise sense: per state,
    max_i |got_i - ref_i| / max_i scale_i <= tol, where scale_i is the sum of
    the magnitudes of the terms that produce entry i (oracle residual_scale /
    rhs_scale). Returns the per-state errors; the message also reports the
    plain max-normalised errors."""
    got = got.detach().double().cpu()
    ref = ref.detach().double().cpu()
    scale = scale.detach().double().cpu()
    S = ref.shape[0]
    d = (got - ref).abs().reshape(S, -1).amax(1)
    e = d / scale.reshape(S, -1).amax(1).clamp_min(1e-300)
    assert bool((e <= tol).all()), (f"{what}: per-state scaled errors {e.tolist()} exceed {tol} "
                                    f"(max-normalised {rel_err(got, ref).tolist()})")
    return e


def cuda(t):
    return t.to("cuda").contiguous()
