"""The semi-discrete NSFR operator as one object (oracle; test infrastructure).

Paper: Eq. NSFR with the weight-adjusted inverse of Eq. weight-adj ESFR mass:
    du/dt = -A (R_vol + R_surf - W J q),  A ~= (M_m + K_m)^-1,
where q is the manufactured source of Sec. 7.1 when enabled (reading: the
source enters like the DG source term chi^T W J q and is then multiplied by the
inverse modified mass, as every right-hand-side term is).
"""
import math

import torch

from . import flux as fx
from .mesh import Mesh
from .mass import wa_apply, exact_apply
from .problems import mms_source
from .residual import residual, residual_definition
from .timestep import rk4_step, cfl_dt


class Scheme:
    def __init__(self, p, ne, lo=0.0, hi=2 * math.pi, beta=0.0, l=None, gamma=1.4,
                 c=0.0, variant=0, dissipation=False, source=False, mass="wa"):
        self.mesh = Mesh(p, ne, lo, hi, beta, l)
        self.p, self.gamma, self.c = p, float(gamma), float(c)
        self.variant, self.dissipation, self.source = variant, dissipation, bool(source)
        self.mass = mass

    @property
    def X(self):
        return self.mesh.X

    def residual(self, U, t=0.0, definition=False):
        """Pre-mass residual R (source folded in as -W J q)."""
        f = residual_definition if definition else residual
        R = f(self.mesh, U, self.gamma, self.variant, self.dissipation)
        if self.source:
            R = R - self.mesh.WJ * mms_source(self.mesh.X, t, self.gamma)
        return R

    def apply_inverse_mass(self, R):
        if self.mass == "wa":
            return wa_apply(self.mesh, self.c, R)
        return exact_apply(self.mesh, self.c, R)

    def rhs(self, U, t=0.0, definition=False):
        """du/dt = -A R."""
        return -self.apply_inverse_mass(self.residual(U, t, definition))

    def rk4_step(self, U, dt, t=0.0):
        return rk4_step(self.rhs, U, dt, t)

    def dt(self, U, cfl=0.1):
        return cfl_dt(self.mesh, U, self.gamma, cfl)

    def max_wavespeed(self, U):
        return fx.max_wavespeed(U, self.gamma)

    def zeros(self):
        n = self.mesh.n
        return torch.zeros(5, self.mesh.E, n, n, n, dtype=torch.float64)
