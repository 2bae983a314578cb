"""Seeded synthetic inputs: initial conditions and random directions.

Shared by the tests, the benchmark and the smoke check; it holds no part of the
numerical scheme itself, only the problem definitions of the paper's test
cases evaluated at given node coordinates, and seeded random numbers.

  * Taylor-Green vortex of Sec. 7.3: rho = 1, u = sin x cos y cos z,
    v = -cos x sin y cos z, w = 0, p = p0 + (cos2x cos2z + 2 cos2x + 2 cos2y
    + cos2y cos2z) / 16 with p0 = 1 / (gamma Mach^2) (Mach 0.1 gives the
    printed 100 / gamma), on [0, 2 pi]^3;
  * manufactured solution of Sec. 7.1 at t = 0;
  * ensemble draws: elements per direction, degree and Mach per flow.

Coordinates come in as a (3, ...) float64 tensor; states go out as (5, ...)
conservative variables [rho, rho u, rho v, rho w, rho e] with
rho e = p / (gamma - 1) + rho |u|^2 / 2.
"""
import math

import numpy as np
import torch


def _to_conservative(rho, u, v, w, p, gamma):
    return torch.stack([rho, rho * u, rho * v, rho * w,
                        p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def tgv_state(X, gamma=1.4, mach=0.1):
    x, y, z = X[0], X[1], X[2]
    rho = torch.ones_like(x)
    u = torch.sin(x) * torch.cos(y) * torch.cos(z)
    v = -torch.cos(x) * torch.sin(y) * torch.cos(z)
    w = torch.zeros_like(x)
    p0 = 1.0 / (gamma * mach * mach)
    p = p0 + (torch.cos(2 * x) * torch.cos(2 * z) + 2 * torch.cos(2 * x) + 2 * torch.cos(2 * y)
              + torch.cos(2 * y) * torch.cos(2 * z)) / 16.0
    return _to_conservative(rho, u, v, w, p, gamma)


def mms_initial_state(X, gamma=1.4, t=0.0):
    s = X[0] + X[1] + X[2] - 2.0 * t
    rho = 2.0 + 0.1 * torch.sin(math.pi * s)
    return torch.stack([rho, rho, rho, rho, rho * rho])


def perturbed_state(X, seed, gamma=1.4, amp=0.05):
    """A rough state with independent random smooth-ish variations per node:
    rho in 1 +- amp, |u| ~ 0.3, p in 1 +- amp (nodal noise; exercises the
    logarithmic-mean closed-form branch)."""
    g = torch.Generator().manual_seed(seed)
    shp = X.shape[1:]
    r = lambda: torch.rand(shp, generator=g, dtype=torch.float64) * 2 - 1  # noqa: E731
    rho = 1.0 + amp * r()
    u, v, w = 0.3 * r(), 0.3 * r(), 0.3 * r()
    p = 1.0 + amp * r()
    return _to_conservative(rho, u, v, w, p, gamma)


def constant_state(shape, gamma=1.4, rho=1.3, vel=(0.3, -0.2, 0.5), p=2.0):
    ones = torch.ones(shape, dtype=torch.float64)
    return _to_conservative(rho * ones, vel[0] * ones, vel[1] * ones, vel[2] * ones, p * ones, gamma)


def normal_like(shape, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(shape, generator=g, dtype=torch.float64)


def ensemble_draws(n_flows=64, seed=0, ne_range=(6, 12), p_choices=(2, 3, 4, 5), mach_range=(0.05, 0.3)):
    """Per-flow (ne, p, mach) for the batched-ensemble workload."""
    rng = np.random.default_rng(seed)
    ne = rng.integers(ne_range[0], ne_range[1] + 1, size=n_flows)
    p = rng.choice(np.array(p_choices), size=n_flows)
    mach = rng.uniform(mach_range[0], mach_range[1], size=n_flows)
    return [(int(a), int(b), float(c)) for a, b, c in zip(ne, p, mach)]
