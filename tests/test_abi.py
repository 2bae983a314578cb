"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/nsfr.h, and rejects invalid
configurations before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2312_07725_amd import nsfr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "nsfr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nsfr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(nsfr.LIB_PATH):
        pytest.fail("libnsfr.so is not built (run python -m paper_2312_07725_amd.build)")
    return nsfr._lib()


def test_exports_every_declared_symbol(L):
    names = declared_symbols()
    assert len(names) >= 25
    for name in names:
        assert hasattr(L, name), name
    # and the Python binding declares a signature for each entry point
    for name in names:
        if name not in ("nsfr_status_string", "nsfr_last_error"):
            assert name in nsfr._SIGS, name


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.nsfr_status_string(code)
    assert L.nsfr_status_string(7) == b"unknown status"


@pytest.mark.parametrize("field,value", [("p", 1), ("p", 6), ("ne", (0, 2, 2)), ("hi", -1.0), ("gamma", 1.0),
                                         ("flux", 2), ("surface_diss", 3), ("source", -1), ("tile", 99),
                                         ("c_fr", -1e-3), ("quad", 2), ("overint", 4), ("overint", 1)])
def test_create_rejects_bad_config(L, field, value):
    cfg = nsfr.make_config(3, 2)
    if field == "ne":
        for i in range(3):
            cfg.ne[i] = value[i]
    else:
        setattr(cfg, field, value)
    ctx = ctypes.c_void_p()
    st = L.nsfr_create(ctypes.byref(cfg), None, ctypes.byref(ctx))
    assert st == nsfr.NSFR_EINVAL
    assert not ctx.value
    assert L.nsfr_last_error()


def test_null_arguments(L):
    ctx = ctypes.c_void_p()
    assert L.nsfr_create(None, None, ctypes.byref(ctx)) == nsfr.NSFR_EINVAL
    assert L.nsfr_rhs(None, None, None, 0.0) == nsfr.NSFR_EINVAL
    assert L.nsfr_destroy(None) == nsfr.NSFR_EINVAL


def test_config_layout_matches_header():
    # int32 p, int32 ne[3], 6 doubles, 8 int32 = 96 bytes
    assert ctypes.sizeof(nsfr.Config) == 96
    assert nsfr.Config.lo.offset == 16
    assert nsfr.Config.flux.offset == 64
    assert nsfr.Config.quad.offset == 80 and nsfr.Config.overint.offset == 84
    assert nsfr.Config.scheme.offset == 88 and nsfr.Config.mass.offset == 92


@pytest.mark.parametrize("kw", [dict(quad=1, tile=2), dict(scheme=2, quad=1), dict(scheme=1, quad=0),
                                dict(scheme=1, quad=1, diss=1), dict(scheme=1, quad=1, overint=5),
                                dict(scheme=0, quad=1, overint=4), dict(mass=2), dict(mass=-1),
                                dict(mass=1, quad=1), dict(mass=1, quad=1, scheme=1)])
def test_create_rejects_invalid_quadrature_or_scheme(L, kw):
    cfg = nsfr.make_config(3, 2, **kw)
    ctx = ctypes.c_void_p()
    assert L.nsfr_create(ctypes.byref(cfg), None, ctypes.byref(ctx)) == nsfr.NSFR_EINVAL
    assert not ctx.value
    assert L.nsfr_last_error()
