"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/sofft.h declares, and rejects bad problems before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1505_06707_amd import sofft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(sofft_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = sofft.lib()
    names = declared_symbols()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(L, name), name
    assert set(sofft.exported_symbols()) <= set(names)


def _create(**kw):
    p = sofft.Problem()
    p.ndim, p.dtype = 2, sofft.C128
    p.n[0] = p.n[1] = 64
    p.L[0] = p.L[1] = 12.8
    p.R0[0] = p.R0[1] = 5.0
    p.theta, p.contour, p.charge, p.a2 = 0.5, sofft.SECS, 1.0, 0.64
    for k, v in kw.items():
        if k in ("n", "L", "R0"):
            getattr(p, k)[0] = v
        else:
            setattr(p, k, v)
    h = ctypes.c_void_p()
    return sofft.lib().sofft_plan_create(ctypes.byref(p), ctypes.byref(h))


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=4), -1),
    (dict(ndim=0), -1),
    (dict(dtype=7), -1),
    (dict(contour=9), -1),
    (dict(theta=0.0), -1),
    (dict(theta=2.0), -1),
    (dict(charge=-1.0), -1),
    (dict(a2=0.0), -1),
    (dict(n=1000), -2),
    (dict(n=2048), -2),          # 2D lines stop at 1024
    (dict(L=-1.0), -1),
    (dict(R0=6.5), -1),          # R0 beyond L/2
])
def test_plan_validation(kw, code):
    assert _create(**kw) == code
    assert sofft.lib().sofft_last_error()


def test_null_arguments_are_rejected():
    L = sofft.lib()
    assert L.sofft_plan_create(None, None) == -1
    assert L.sofft_propagate(None, None, 0.05, 1, None, None) == -1
    assert L.sofft_norm2(None, None, None, None) == -1
    assert L.sofft_set_potential(None, None, None) == -1
    assert L.sofft_make_softcore(None, 1.0, 1.0, None, None) == -1
    assert L.sofft_add_absorber(None, sofft.ABSORBER_TFAP, 0.25, None, None) == -1


def test_workspace_calls_reject_null_arguments():
    L = sofft.lib()
    n = ctypes.c_int64()
    assert L.sofft_workspace_size(None, 0, ctypes.byref(n)) == -1
    assert L.sofft_plan_bind(None, None, 0) == -1
    assert L.sofft_batch_workspace_size(None, ctypes.byref(n)) == -1
    assert L.sofft_batch_bind(None, None, 0) == -1


def _create3(n):
    p = sofft.Problem()
    p.ndim, p.dtype = 3, sofft.C128
    for d in range(3):
        p.n[d] = n[d]
        p.L[d] = 0.2 * n[d]
        p.R0[d] = 0.08 * n[d]
    p.theta, p.contour, p.charge, p.a2 = 0.5, sofft.SECS, 1.0, 0.64
    h = ctypes.c_void_p()
    return sofft.lib().sofft_plan_create(ctypes.byref(p), ctypes.byref(h))


@pytest.mark.parametrize("n", [(1024, 16, 16), (96, 64, 64), (64, 48, 64), (64, 64, 0)])
def test_3d_plan_validation(n):
    """3D lines are powers of two from 16 to 512: other lengths are rejected
    before any device work."""
    assert _create3(n) == -2
