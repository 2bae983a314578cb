"""Python binding of libnsfr (ctypes). Argument marshalling only: every step of
the scheme runs in the HIP kernels of the library. PyTorch supplies device
memory and the current HIP stream.

If the library has not been built, or no GPU is visible, the calls raise;
there is no CPU fallback.
"""
import ctypes
import math
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_void_p, c_char_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# NSFR_LIB selects another build of the library (e.g. a variant compiled with
# different kernel options); by default the in-tree build is used.
LIB_PATH = os.environ.get("NSFR_LIB") or os.path.join(_HERE, "libnsfr.so")

NSFR_OK, NSFR_EINVAL, NSFR_ENOMEM, NSFR_EHIP, NSFR_EUNPHYSICAL, NSFR_ENOTSUP = 0, -1, -2, -3, -4, -5


class Config(ctypes.Structure):
    _fields_ = [
        ("p", c_int32), ("ne", c_int32 * 3),
        ("lo", c_double), ("hi", c_double), ("warp_beta", c_double), ("warp_l", c_double),
        ("gamma", c_double), ("c_fr", c_double),
        ("flux", c_int32), ("surface_diss", c_int32), ("source", c_int32), ("tile", c_int32),
        ("quad", c_int32), ("overint", c_int32), ("scheme", c_int32), ("mass", c_int32),
    ]


class NSFRError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib().nsfr_last_error().decode()
        super().__init__(f"{where}: {_lib().nsfr_status_string(status).decode()} ({status}): {msg}")


_L = None

# symbol -> (argtypes); every function returns int (nsfr_status)
_SIGS = {
    "nsfr_create": [POINTER(Config), c_void_p, POINTER(c_void_p)],
    "nsfr_destroy": [c_void_p],
    "nsfr_set_stream": [c_void_p, c_void_p],
    "nsfr_sizes": [c_void_p, POINTER(c_int64), POINTER(c_int64)],
    "nsfr_node_coords": [c_void_p, c_void_p],
    "nsfr_geometry": [c_void_p, c_void_p, c_void_p],
    "nsfr_residual": [c_void_p, c_void_p, c_void_p, c_double],
    "nsfr_rhs": [c_void_p, c_void_p, c_void_p, c_double],
    "nsfr_rk4_step": [c_void_p, c_void_p, c_void_p, c_double, c_void_p],
    "nsfr_rk4_step_static": [c_void_p, c_void_p, c_void_p, c_double],
    "nsfr_rk4_run": [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p],
    "nsfr_max_wavespeed": [c_void_p, c_void_p, c_void_p],
    "nsfr_cfl_dt": [c_void_p, c_void_p, c_double, c_void_p],
    "nsfr_rhs_vjp": [c_void_p, c_void_p, c_void_p, c_void_p, c_double],
    "nsfr_rk4_step_vjp": [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p],
    "nsfr_diagnostics": [c_void_p, c_void_p, c_double, c_void_p],
    "nsfr_check_state": [c_void_p, c_void_p, POINTER(c_int32)],
    "nsfr_kinetic_energy": [c_void_p, c_void_p, c_void_p, c_void_p],
    "nsfr_ens_create": [POINTER(Config), c_int32, c_void_p, POINTER(c_void_p)],
    "nsfr_ens_destroy": [c_void_p],
    "nsfr_ens_set_stream": [c_void_p, c_void_p],
    "nsfr_ens_offsets": [c_void_p, POINTER(c_int64)],
    "nsfr_ens_rhs": [c_void_p, c_void_p, c_void_p, c_double],
    "nsfr_ens_rk4_step": [c_void_p, c_void_p, c_void_p, c_double, c_void_p],
    "nsfr_ens_rk4_run": [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p],
    "nsfr_ens_set_tile": [c_void_p, c_int32, c_int32],
    "nsfr_c_hu": [c_int32, POINTER(c_double)],
}


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2312_07725_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int32
        L.nsfr_status_string.argtypes = [c_int32]
        L.nsfr_status_string.restype = c_char_p
        L.nsfr_last_error.argtypes = []
        L.nsfr_last_error.restype = c_char_p
        _L = L
    return _L


def _check(st, where):
    if st != NSFR_OK:
        raise NSFRError(st, where)


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def c_hu(p):
    """FR parameter c_HU for degree p, computed by the library (Sec. 7.2)."""
    out = c_double()
    _check(_lib().nsfr_c_hu(int(p), byref(out)), "nsfr_c_hu")
    return out.value


def make_config(p, ne, lo=0.0, hi=2 * math.pi, beta=0.0, l=0.0, gamma=1.4, c=0.0, flux=0, diss=0, source=0, tile=0,
                quad=0, overint=0, scheme=0, mass=0):
    if isinstance(ne, int):
        ne = (ne, ne, ne)
    cfg = Config()
    cfg.p = int(p)
    cfg.ne[0], cfg.ne[1], cfg.ne[2] = (int(v) for v in ne)
    cfg.lo, cfg.hi = float(lo), float(hi)
    cfg.warp_beta, cfg.warp_l = float(beta), float(l or 0.0)
    cfg.gamma, cfg.c_fr = float(gamma), float(c)
    cfg.flux, cfg.surface_diss, cfg.source, cfg.tile = int(flux), int(diss), int(source), int(tile)
    cfg.quad, cfg.overint, cfg.scheme, cfg.mass = int(quad), int(overint), int(scheme), int(mass)
    return cfg


class NSFR:
    """One NSFR discretisation on the current GPU (a libnsfr context).

    quad = "lgl" (collocated, the default) or "gl" (Gauss-Legendre volume and
    surface rule with p + 1 + overint points per direction); scheme = "nsfr"
    (the default) or "dg" (conservative strong DG with Roe's flux, on the GL
    rule); mass = "wa" (the weight-adjusted inverse, the default) or "exact"
    (the exact inverse of the FR-modified mass, for checking; rhs only)."""

    def __init__(self, p, ne, lo=0.0, hi=2 * math.pi, beta=0.0, l=0.0, gamma=1.4, c=0.0, flux=0, diss=0,
                 source=0, tile=0, quad="lgl", overint=0, scheme="nsfr", mass="wa"):
        if not torch.cuda.is_available():
            raise RuntimeError("libnsfr needs a HIP GPU; none is visible")
        if quad not in ("lgl", "gl"):
            raise ValueError(f"quad must be 'lgl' or 'gl', got {quad!r}")
        q = 1 if quad == "gl" else 0
        if scheme not in ("nsfr", "dg"):
            raise ValueError(f"scheme must be 'nsfr' or 'dg', got {scheme!r}")
        if mass not in ("wa", "exact"):
            raise ValueError(f"mass must be 'wa' or 'exact', got {mass!r}")
        if not tile and not q:
            from .tune import load_tiles
            tile = load_tiles().get(int(p), 0)
        self.quad, self.overint, self.scheme = quad, int(overint), scheme
        self.cfg = make_config(p, ne, lo, hi, beta, l, gamma, c, flux, diss, source, tile, q, overint,
                               1 if scheme == "dg" else 0, 1 if mass == "exact" else 0)
        self.p, self.n = int(p), int(p) + 1
        self.gamma = float(gamma)
        self._ctx = c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device())
        _check(_lib().nsfr_create(byref(self.cfg), _stream(), byref(self._ctx)), "nsfr_create")
        E, nn = c_int64(), c_int64()
        _check(_lib().nsfr_sizes(self._ctx, byref(E), byref(nn)), "nsfr_sizes")
        self.E, self.nodes_per_elem = E.value, nn.value
        self.shape = (5, self.E, self.n, self.n, self.n)

    def close(self):
        if self._ctx:
            _lib().nsfr_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers
    @property
    def n_nodes(self):
        return self.E * self.nodes_per_elem

    def empty(self, *lead):
        return torch.empty(*lead, *self.shape, dtype=torch.float64, device=self.device)

    def zeros(self, *lead):
        return torch.zeros(*lead, *self.shape, dtype=torch.float64, device=self.device)

    def _arr(self, t, nelem, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device.type != "cuda":
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous() or t.numel() != nelem:
            raise ValueError(f"{name} must be contiguous with {nelem} elements, got {tuple(t.shape)}")
        return c_void_p(t.data_ptr())

    def _st(self, t, name):
        return self._arr(t, 5 * self.n_nodes, name)

    def _sync_stream(self):
        _check(_lib().nsfr_set_stream(self._ctx, _stream()), "nsfr_set_stream")

    # ---- C-ABI entry points
    def node_coords(self):
        X = torch.empty(3, self.E, self.n, self.n, self.n, dtype=torch.float64, device=self.device)
        self._sync_stream()
        _check(_lib().nsfr_node_coords(self._ctx, self._arr(X, 3 * self.n_nodes, "xyz")), "nsfr_node_coords")
        return X

    def geometry(self):
        C = torch.empty(3, 3, self.E, self.n, self.n, self.n, dtype=torch.float64, device=self.device)
        J = torch.empty(self.E, self.n, self.n, self.n, dtype=torch.float64, device=self.device)
        self._sync_stream()
        _check(_lib().nsfr_geometry(self._ctx, self._arr(C, 9 * self.n_nodes, "C"), self._arr(J, self.n_nodes, "J")),
               "nsfr_geometry")
        return C, J

    def residual(self, U, out=None, t=0.0):
        out = self.empty() if out is None else out
        self._sync_stream()
        _check(_lib().nsfr_residual(self._ctx, self._st(U, "U"), self._st(out, "R"), float(t)), "nsfr_residual")
        return out

    def rhs(self, U, out=None, t=0.0):
        out = self.empty() if out is None else out
        self._sync_stream()
        _check(_lib().nsfr_rhs(self._ctx, self._st(U, "U"), self._st(out, "dUdt"), float(t)), "nsfr_rhs")
        return out

    def work(self, k=3):
        return torch.empty(k, *self.shape, dtype=torch.float64, device=self.device)

    def rk4_step(self, U, dt, t=0.0, work=None):
        work = self.work(3) if work is None else work
        self._sync_stream()
        _check(_lib().nsfr_rk4_step(self._ctx, self._st(U, "U"), self._arr(dt, 1, "dt"), float(t),
                                    self._arr(work, 15 * self.n_nodes, "work")), "nsfr_rk4_step")
        return U

    def rk4_step_static(self, U, dt, t=0.0):
        """nsfr_rk4_step without a work argument: the stage arrays live in the
        library's per-GPU static workspace (no allocation by the library)."""
        self._sync_stream()
        _check(_lib().nsfr_rk4_step_static(self._ctx, self._st(U, "U"), self._arr(dt, 1, "dt"), float(t)),
               "nsfr_rk4_step_static")
        return U

    def rk4_run(self, U, dt, t_dev, nsteps, work=None):
        work = self.work(3) if work is None else work
        self._sync_stream()
        tp = self._arr(t_dev, 1, "t") if t_dev is not None else c_void_p(0)
        _check(_lib().nsfr_rk4_run(self._ctx, self._st(U, "U"), self._arr(dt, 1, "dt"), tp,
                                   int(nsteps), self._arr(work, 15 * self.n_nodes, "work")), "nsfr_rk4_run")
        return U

    def max_wavespeed(self, U, out=None):
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        self._sync_stream()
        _check(_lib().nsfr_max_wavespeed(self._ctx, self._st(U, "U"), self._arr(out, 1, "lam")), "nsfr_max_wavespeed")
        return out

    def cfl_dt(self, U, cfl=0.1, out=None):
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        self._sync_stream()
        _check(_lib().nsfr_cfl_dt(self._ctx, self._st(U, "U"), float(cfl), self._arr(out, 1, "dt")), "nsfr_cfl_dt")
        return out

    def rhs_vjp(self, U, lam, out=None, t=0.0):
        out = self.empty() if out is None else out
        self._sync_stream()
        _check(_lib().nsfr_rhs_vjp(self._ctx, self._st(U, "U"), self._st(lam, "lam"), self._st(out, "g"), float(t)),
               "nsfr_rhs_vjp")
        return out

    def rk4_step_vjp(self, U, dt, lam_next, t=0.0, out=None, work=None):
        out = self.empty() if out is None else out
        work = self.work(6) if work is None else work
        self._sync_stream()
        _check(_lib().nsfr_rk4_step_vjp(self._ctx, self._st(U, "U"), self._arr(dt, 1, "dt"), float(t),
                                        self._st(lam_next, "lam_next"), self._st(out, "lam"),
                                        self._arr(work, 30 * self.n_nodes, "work")), "nsfr_rk4_step_vjp")
        return out

    def diagnostics(self, U, t=0.0):
        out = torch.empty(8, dtype=torch.float64, device=self.device)
        self._sync_stream()
        _check(_lib().nsfr_diagnostics(self._ctx, self._st(U, "U"), float(t), self._arr(out, 8, "out")),
               "nsfr_diagnostics")
        return out

    def kinetic_energy(self, U, grad=None):
        """Returns (J_KE as a 1-element device tensor, gradient or None)."""
        ke = torch.empty(1, dtype=torch.float64, device=self.device)
        self._sync_stream()
        gp = self._st(grad, "grad") if grad is not None else c_void_p(0)
        _check(_lib().nsfr_kinetic_energy(self._ctx, self._st(U, "U"), self._arr(ke, 1, "ke"), gp),
               "nsfr_kinetic_energy")
        return ke, grad

    def check_state(self, U):
        bad = c_int32(0)
        self._sync_stream()
        st = _lib().nsfr_check_state(self._ctx, self._st(U, "U"), byref(bad))
        if st not in (NSFR_OK, NSFR_EUNPHYSICAL):
            _check(st, "nsfr_check_state")
        return bad.value


class Ensemble:
    """A batch of independent flows stepped together (libnsfr ensemble)."""

    def __init__(self, configs):
        if not torch.cuda.is_available():
            raise RuntimeError("libnsfr needs a HIP GPU; none is visible")
        self.configs = list(configs)
        arr = (Config * len(self.configs))(*self.configs)
        self._h = c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device())
        _check(_lib().nsfr_ens_create(arr, len(self.configs), _stream(), byref(self._h)), "nsfr_ens_create")
        offs = (c_int64 * (len(self.configs) + 1))()
        _check(_lib().nsfr_ens_offsets(self._h, offs), "nsfr_ens_offsets")
        from .tune import load_ensemble_tiles
        for p, epb in load_ensemble_tiles().items():
            if _lib().nsfr_ens_set_tile(self._h, int(p), int(epb)) != NSFR_OK:
                _lib().nsfr_ens_set_tile(self._h, int(p), 0)
        self.offsets = [int(v) for v in offs]
        self.total = self.offsets[-1]

    def close(self):
        if self._h:
            _lib().nsfr_ens_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, *lead):
        return torch.empty(*lead, self.total, dtype=torch.float64, device=self.device)

    def _a(self, t, n, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device.type != "cuda":
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be contiguous with {n} elements")
        return c_void_p(t.data_ptr())

    def _sync_stream(self):
        _check(_lib().nsfr_ens_set_stream(self._h, _stream()), "nsfr_ens_set_stream")

    def flow_view(self, packed, i):
        c = self.configs[i]
        n = c.p + 1
        E = c.ne[0] * c.ne[1] * c.ne[2]
        return packed[self.offsets[i]:self.offsets[i + 1]].view(5, E, n, n, n)

    def rhs(self, U, out=None, t=0.0):
        out = self.empty() if out is None else out
        self._sync_stream()
        _check(_lib().nsfr_ens_rhs(self._h, self._a(U, self.total, "U"), self._a(out, self.total, "dUdt"), float(t)),
               "nsfr_ens_rhs")
        return out

    def rk4_step(self, U, dt, t=0.0, work=None):
        work = self.empty(3) if work is None else work
        self._sync_stream()
        _check(_lib().nsfr_ens_rk4_step(self._h, self._a(U, self.total, "U"), self._a(dt, len(self.configs), "dt"),
                                        float(t), self._a(work, 3 * self.total, "work")), "nsfr_ens_rk4_step")
        return U

    def rk4_run(self, U, dt, nsteps, t=0.0, work=None):
        work = self.empty(3) if work is None else work
        self._sync_stream()
        _check(_lib().nsfr_ens_rk4_run(self._h, self._a(U, self.total, "U"), self._a(dt, len(self.configs), "dt"),
                                       float(t), int(nsteps), self._a(work, 3 * self.total, "work")),
               "nsfr_ens_rk4_run")
        return U

    def set_tile(self, p, epb):
        _check(_lib().nsfr_ens_set_tile(self._h, int(p), int(epb)), "nsfr_ens_set_tile")
