"""C ABI: the library loads, exports every entry point include/ug.h declares,
and rejects invalid arguments on the host before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ug.h")


@pytest.fixture(scope="module")
def L():
    from paper_2505_05643_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ug_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ug_render_planes", "ug_render_planes_backward", "ug_plan_create", "ug_plan_destroy",
                 "ug_plan_status", "ug_mse_grad", "ug_adam_step"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L.lib, name), name
        assert name in L.SIGNATURES, f"binding lacks {name}"


def test_status_strings_and_defaults(L):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = L.lib.ug_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.lib.ug_status_string(-99).decode() == "unknown status"
    p = L.UgParams()
    L.lib.ug_params_default(ctypes.byref(p))
    assert p.chi2 == pytest.approx(7.815) and p.beta == pytest.approx(1e-4)
    assert p.bg_alpha == pytest.approx(1e-2) and p.box_mode == L.UG_BOX_PAPER


def _create(L, n=10, wh=((16, 16),), **kw):
    p = L.UgParams()
    L.lib.ug_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    arr = np.ascontiguousarray(np.asarray(wh, dtype=np.int32))
    out = ctypes.c_void_p()
    code = L.lib.ug_plan_create(n, len(wh), arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(p),
                                100, 100, ctypes.byref(out))
    return code, out


@pytest.mark.parametrize("kw", [dict(n=-1), dict(wh=((0, 5),)), dict(wh=((40000, 5),)), dict(beta=0.0),
                                dict(beta=float("nan")), dict(chi2=-1.0), dict(chi2=float("nan")),
                                dict(bg_alpha=0.0), dict(box_mode=7), dict(flags=4), dict(flags=32), dict(tile_w=12),
                                dict(flags=8, tile_w=32, tile_h=32, lds_batch=256),
                                dict(lds_batch=48), dict(tile_w=8, tile_h=8, px_per_lane=2),
                                dict(bg_color=float("inf")),
                                # 32x32 tiles leave 16 bits of the key word for the tile id: 257 x 256 tiles
                                dict(tile_w=32, tile_h=32, wh=((8200, 8192),))])
def test_plan_create_rejects_invalid(L, kw):
    code, out = _create(L, **kw)
    assert code == L.UG_ERR_INVALID_ARG and not out.value


def test_plan_create_without_device_or_ok(L):
    code, out = _create(L, chi2=math.inf)
    assert code in (L.UG_OK, L.UG_ERR_NO_DEVICE)
    if code == L.UG_OK:
        L.lib.ug_plan_destroy(out)
    # exactly 2^16 tiles of 32x32 still fit the key word
    code, out = _create(L, tile_w=32, tile_h=32, wh=((8192, 8192),))
    assert code in (L.UG_OK, L.UG_ERR_NO_DEVICE)
    if code == L.UG_OK:
        L.lib.ug_plan_destroy(out)


def test_entry_points_reject_null_arguments(L):
    g = L.UgGaussians(None, None, None, None, 0)
    pl = L.UgPlanes(None, None, None, 1)
    cnt = (ctypes.c_int64 * 2)()
    assert L.lib.ug_render_planes(None, ctypes.byref(g), ctypes.byref(pl), None, None, None) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_render_planes_backward(None, ctypes.byref(g), ctypes.byref(pl), None, None, None, None, None,
                                           None, None, 0, None) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_plan_measure(None, ctypes.byref(g), ctypes.byref(pl), None, cnt, None) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_plan_status(None, None, cnt, None) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_plan_reserve(None, 1, 1) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_profile_begin(None, 0xff, 10) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_profile_read(None, None, None) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_plan_workspace_bytes(None) == 0
    assert L.lib.ug_mse_grad(None, None, 10, None, None, None) == L.UG_ERR_INVALID_ARG
    assert L.lib.ug_adam_step(None, None, None, None, 10, 0.1, 0.9, 0.999, 1e-8, 1, None) == L.UG_ERR_INVALID_ARG
    L.lib.ug_plan_destroy(None)


def test_newer_entry_points_reject_invalid_arguments(L):
    """Host-side validation of the fused adjoint, the captured step, the
    record hook, the scoring call and the parameterisation study (no device
    work happens)."""
    g = L.UgGaussians(None, None, None, None, 0)
    pl = L.UgPlanes(None, None, None, 1)
    gm = L.UgGaussiansMut(None, None, None, None, 0)
    hp = L.UgAdamParams(1e-4, 1e-6, 10, 0.05, 0.9, 0.999, 1e-8)
    bad = L.UG_ERR_INVALID_ARG
    assert L.lib.ug_render_planes_backward_mse(None, ctypes.byref(g), ctypes.byref(pl), None, None, None, None,
                                               None, None, None, 0, None, None) == bad
    assert L.lib.ug_step_capture(None, ctypes.byref(gm), ctypes.byref(pl), None, None, None, ctypes.byref(gm),
                                 ctypes.byref(gm), ctypes.byref(gm), ctypes.byref(hp), None, None, None, None) == bad
    assert L.lib.ug_step_replay(None, None) == bad
    assert L.lib.ug_debug_records(None, None, None, 0, None) == bad
    assert L.lib.ug_debug_keys(None, None, None, None, None, None, 0, None) == bad
    ms = ctypes.c_float()
    for kind, blocks, iters, n in ((9, 1, 1, 256), (0, 0, 1, 256), (0, 1, 0, 256), (0, 2, 1, 256), (3, 1, 1, 6)):
        assert L.lib.ug_probe(kind, blocks, iters, None, None, n, ctypes.byref(ms), None) == bad
    assert L.lib.ug_image_quality(None, None, None, 1.0, None, None, None, None) == bad
    assert L.lib.ug_quality_workspace_bytes(None) == 0
    for kind, fp64, n in ((7, 0, 1), (0, 2, 1), (0, 0, -1)):
        assert L.lib.ug_param_eval(kind, fp64, None, None, None, n, 1e-4, None, None, None, None) == bad
    assert L.lib.ug_param_eval(L.UG_PARAM_TRI, 0, None, None, None, 5, 1e-4, None, None, None, None) == bad
    assert L.lib.ug_param_eval(L.UG_PARAM_QUAT, 1, None, None, None, 0, 1e-4, None, None, None, None) == L.UG_OK
