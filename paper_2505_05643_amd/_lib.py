"""ctypes loader of libug.so (include/ug.h).  Argument marshalling only.

The library is built in-tree by ``paper_2505_05643_amd.build``.  There is no
fallback: if it is missing or cannot be loaded, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libug.so")

UG_OK = 0
UG_ERR_INVALID_ARG = -1
UG_ERR_CAPACITY = -2
UG_ERR_NONFINITE = -3
UG_ERR_HIP = -4
UG_ERR_NO_DEVICE = -5
UG_ERR_INTERNAL = -6
UG_ERR_SCRATCH_SIZE = -7
UG_NOALLOC_WORKSPACE_BYTES = 64 << 20

UG_BOX_PAPER = 0
UG_BOX_CONIC = 1
UG_BOX_ROWS = 2

UG_MSE_SCRATCH_FLOATS = 1026
UG_FLAG_COUNT_EVALS = 1
UG_FLAG_SCATTER = 2
UG_FLAG_BOX_SUPPORT = 4
UG_FLAG_SPLIT_FORWARD = 8
UG_FLAG_CULL_EACH_PLANE = 16
UG_PARAM_TRI, UG_PARAM_SYM, UG_PARAM_QUAT = 0, 1, 2
UG_PROBE_FMA, UG_PROBE_EXP, UG_PROBE_PAIRS, UG_PROBE_COPY = 0, 1, 2, 3

STAGES = ("setup", "cull_count", "cull_write", "record", "emit", "sort_hist", "sort_scan", "sort_scatter", "ranges",
          "accum", "bwd_prep", "accum_bwd", "record_adj", "gauss_grad", "scatter")
UG_NUM_STAGES = len(STAGES)

c_i32, c_i64, c_f32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p


class UgGaussians(ctypes.Structure):
    _fields_ = [("means", c_vp), ("lraw", c_vp), ("intensity", c_vp), ("opacity", c_vp), ("n", c_i32)]


class UgPlanes(ctypes.Structure):
    _fields_ = [("rot", c_vp), ("origin", c_vp), ("spacing", c_vp), ("p", c_i32)]


class UgParams(ctypes.Structure):
    _fields_ = [("beta", c_f32), ("chi2", c_f32), ("bg_alpha", c_f32), ("bg_color", c_f32),
                ("tile_w", c_i32), ("tile_h", c_i32), ("px_per_lane", c_i32),
                ("lds_batch", c_i32), ("box_mode", c_i32), ("flags", c_i32)]


class UgGaussiansMut(ctypes.Structure):
    _fields_ = [("means", c_vp), ("lraw", c_vp), ("intensity", c_vp), ("opacity", c_vp), ("n", c_i32)]


class UgAdamParams(ctypes.Structure):
    _fields_ = [("lr_means", c_f32), ("lr_means_final", c_f32), ("decay_steps", c_i32), ("lr", c_f32),
                ("beta1", c_f32), ("beta2", c_f32), ("eps", c_f32)]


class UgRecord(ctypes.Structure):
    _fields_ = [("gaussian", c_i32), ("plane", c_i32), ("t11", c_f32), ("t12", c_f32), ("t22", c_f32),
                ("fu", c_f32), ("fv", c_f32), ("e0", c_f32), ("emin", c_f32), ("c", c_f32),
                ("ub", c_i32), ("vb", c_i32), ("tx0", ctypes.c_uint16), ("tx1", ctypes.c_uint16),
                ("ty0", ctypes.c_uint16), ("ty1", ctypes.c_uint16)]


class UgDensifyParams(ctypes.Structure):
    _fields_ = [("beta", c_f32), ("min_opacity", c_f32), ("grad_thresh", c_f32), ("split_size", c_f32),
                ("max_size", c_f32), ("split_factor", c_f32)]


# name -> (restype, argtypes); mirrors include/ug.h
SIGNATURES = {
    "ug_params_default": (None, [ctypes.POINTER(UgParams)]),
    "ug_plan_create": (c_i32, [c_i32, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(UgParams),
                               c_i64, c_i64, ctypes.POINTER(c_vp)]),
    "ug_plan_reserve": (c_i32, [c_vp, c_i64, c_i64]),
    "ug_plan_workspace_bytes": (ctypes.c_size_t, [c_vp]),
    "ug_plan_num_pixels": (c_i64, [c_vp]),
    "ug_plan_num_tiles": (c_i64, [c_vp]),
    "ug_plan_measure": (c_i32, [c_vp, ctypes.POINTER(UgGaussians), ctypes.POINTER(UgPlanes), c_vp,
                                ctypes.POINTER(c_i64), c_vp]),
    "ug_render_planes": (c_i32, [c_vp, ctypes.POINTER(UgGaussians), ctypes.POINTER(UgPlanes), c_vp, c_vp, c_vp]),
    "ug_render_planes_noalloc": (c_i32, [c_vp, ctypes.POINTER(UgGaussians), ctypes.POINTER(UgPlanes), c_vp, c_vp]),
    "ug_render_planes_backward": (c_i32, [c_vp, ctypes.POINTER(UgGaussians), ctypes.POINTER(UgPlanes), c_vp,
                                          c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp]),
    "ug_render_planes_backward_mse": (c_i32, [c_vp, ctypes.POINTER(UgGaussians), ctypes.POINTER(UgPlanes), c_vp,
                                              c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp]),
    "ug_plan_status": (c_i32, [c_vp, c_vp, ctypes.POINTER(c_i64), c_vp]),
    "ug_mse_grad": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "ug_adam_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, c_f32, c_f32, c_f32, c_f32, c_i32, c_vp]),
    "ug_profile_begin": (c_i32, [c_vp, ctypes.c_uint32, c_i32]),
    "ug_profile_read": (c_i32, [c_vp, ctypes.POINTER(c_f32), ctypes.POINTER(c_i32)]),
    "ug_adam_gaussians": (c_i32, [c_vp, c_vp, ctypes.POINTER(UgGaussiansMut), ctypes.POINTER(UgGaussiansMut),
                                  ctypes.POINTER(UgGaussiansMut), ctypes.POINTER(UgGaussiansMut),
                                  ctypes.POINTER(UgAdamParams), c_vp, c_vp]),
    "ug_sample_gaussians": (c_i32, [ctypes.POINTER(UgGaussians), c_f32, c_vp, c_vp, c_i64, c_vp, c_vp]),
    "ug_accumulate_grad_norm": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "ug_densify_params_default": (None, [ctypes.POINTER(UgDensifyParams)]),
    "ug_densify_workspace_bytes": (ctypes.c_size_t, [c_i32]),
    "ug_densify": (c_i32, [ctypes.POINTER(UgGaussians), c_vp, c_vp, c_vp, ctypes.POINTER(UgDensifyParams),
                           ctypes.POINTER(UgGaussiansMut), c_i64, c_vp, c_vp, c_vp]),
    "ug_quality_workspace_bytes": (ctypes.c_size_t, [c_vp]),
    "ug_image_quality": (c_i32, [c_vp, c_vp, c_vp, c_f32, c_vp, c_vp, c_vp, c_vp]),
    "ug_param_eval": (c_i32, [c_i32, c_i32, c_vp, c_vp, c_vp, c_i64, c_f32, c_vp, c_vp, c_vp, c_vp]),
    "ug_step_capture": (c_i32, [c_vp, ctypes.POINTER(UgGaussiansMut), ctypes.POINTER(UgPlanes), c_vp, c_vp, c_vp,
                                ctypes.POINTER(UgGaussiansMut), ctypes.POINTER(UgGaussiansMut),
                                ctypes.POINTER(UgGaussiansMut), ctypes.POINTER(UgAdamParams), c_vp, c_vp, c_vp,
                                c_vp]),
    "ug_step_replay": (c_i32, [c_vp, c_vp]),
    "ug_debug_records": (c_i64, [c_vp, c_vp, ctypes.POINTER(UgRecord), c_i64, c_vp]),
    "ug_debug_keys": (c_i64, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp]),
    "ug_probe": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_vp, c_i64, ctypes.POINTER(c_f32), c_vp]),
    "ug_status_string": (ctypes.c_char_p, [c_i32]),
    "ug_plan_destroy": (None, [c_vp]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_05643_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class UgError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {lib.ug_status_string(code).decode()} ({code})")


def check(code: int, what: str) -> int:
    if code != UG_OK:
        raise UgError(code, what)
    return code
