"""Python binding of the probe-plane rasterizer: plans, render, backward.

Thin layer over ``libug.so``: it marshals torch device pointers and the
current HIP stream into the C ABI and owns nothing but the workspace tensor.
Every step of the render and its adjoint runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import NamedTuple, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import lib, check


@dataclasses.dataclass
class Params:
    beta: float = 1e-4
    chi2: float = 7.815
    bg_alpha: float = 1e-2
    bg_color: float = 0.0
    tile_w: int = 16
    tile_h: int = 16
    px_per_lane: int = 0
    lds_batch: int = 64
    box_mode: int = _lib.UG_BOX_PAPER
    flags: int = 0

    def to_c(self) -> _lib.UgParams:
        p = _lib.UgParams()
        lib.ug_params_default(ctypes.byref(p))
        for f in dataclasses.fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


class GaussianTensors(NamedTuple):
    means: torch.Tensor      # [N,3]
    lraw: torch.Tensor       # [N,6]
    intensity: torch.Tensor  # [N]
    opacity: torch.Tensor    # [N] logits


class PlaneTensors(NamedTuple):
    rot: torch.Tensor        # [P,9]
    origin: torch.Tensor     # [P,3]
    spacing: torch.Tensor    # [P,2]


def _dev_f32(t: torch.Tensor, shape_tail, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}")
    return t


def _c_gauss(g: GaussianTensors) -> _lib.UgGaussians:
    n = g.means.shape[0]
    _dev_f32(g.means, (3,), "means")
    _dev_f32(g.lraw, (6,), "lraw")
    _dev_f32(g.intensity, (), "intensity")
    _dev_f32(g.opacity, (), "opacity")
    if not (g.lraw.shape[0] == g.intensity.shape[0] == g.opacity.shape[0] == n):
        raise ValueError("Gaussian tensors disagree on N")
    return _lib.UgGaussians(g.means.data_ptr(), g.lraw.data_ptr(), g.intensity.data_ptr(),
                            g.opacity.data_ptr(), n)


def _c_planes(pl: PlaneTensors) -> _lib.UgPlanes:
    p = pl.rot.shape[0]
    _dev_f32(pl.rot, (9,), "rot")
    _dev_f32(pl.origin, (3,), "origin")
    _dev_f32(pl.spacing, (2,), "spacing")
    if not (pl.origin.shape[0] == pl.spacing.shape[0] == p):
        raise ValueError("plane tensors disagree on P")
    return _lib.UgPlanes(pl.rot.data_ptr(), pl.origin.data_ptr(), pl.spacing.data_ptr(), p)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """A render plan: N Gaussians onto P planes of fixed pixel sizes.

    Capacities (records, keys) bound one render's work buffers; ``fit``
    measures them for given inputs.  The workspace tensor carries the
    forward's state to the backward, so a backward must follow its own
    forward before the next forward on the same plan.
    """

    def __init__(self, n: int, wh: Sequence[Sequence[int]], params: Params | None = None,
                 record_capacity: int = 0, key_capacity: int = 0, device=None):
        self.params = params or Params()
        self.wh = np.ascontiguousarray(np.asarray(wh, dtype=np.int32).reshape(-1, 2))
        self.n = int(n)
        self.p = int(self.wh.shape[0])
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._c_params = self.params.to_c()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib.ug_plan_create(self.n, self.p, self.wh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     ctypes.byref(self._c_params), int(record_capacity), int(key_capacity),
                                     ctypes.byref(h)), "ug_plan_create")
        self._h = h
        self.num_pixels = int(lib.ug_plan_num_pixels(h))
        self.num_tiles = int(lib.ug_plan_num_tiles(h))
        self.record_capacity = int(record_capacity)
        self.key_capacity = int(key_capacity)
        self._ws = None
        self._ws_ptr = 0
        self.forward_count = 0
        self._alloc_ws()

    # ---------------------------------------------------------------- workspace
    def _alloc_ws(self):
        nbytes = int(lib.ug_plan_workspace_bytes(self._h))
        if self._ws is not None and self._ws.numel() >= nbytes + 256:
            return
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256

    @property
    def workspace_bytes(self) -> int:
        return int(lib.ug_plan_workspace_bytes(self._h))

    def reserve(self, record_capacity: int, key_capacity: int):
        check(lib.ug_plan_reserve(self._h, int(record_capacity), int(key_capacity)), "ug_plan_reserve")
        self.record_capacity, self.key_capacity = int(record_capacity), int(key_capacity)
        self._alloc_ws()

    def measure(self, g: GaussianTensors, planes: PlaneTensors):
        """(records, keys) a render of these inputs needs (synchronises); keys
        is -1 when the records exceed the current record capacity."""
        cg, cp = _c_gauss(g), _c_planes(planes)
        out = (ctypes.c_int64 * 2)()
        code = lib.ug_plan_measure(self._h, ctypes.byref(cg), ctypes.byref(cp), self._ws_ptr, out, _stream())
        if code not in (_lib.UG_OK, _lib.UG_ERR_NONFINITE):
            check(code, "ug_plan_measure")
        return int(out[0]), int(out[1])

    def fit(self, g: GaussianTensors, planes: PlaneTensors, headroom: float = 1.25):
        """Sizes the capacities for these inputs (plus headroom) if needed."""
        r, k = self.measure(g, planes)
        if k < 0 or r > self.record_capacity:
            self.reserve(max(int(r * headroom) + 16, r), self.key_capacity)
            r, k = self.measure(g, planes)
        if k > self.key_capacity:
            self.reserve(self.record_capacity, max(int(k * headroom) + 64, k))
        return r, k

    # ---------------------------------------------------------------- passes
    def render(self, g: GaussianTensors, planes: PlaneTensors, image: torch.Tensor | None = None,
               check_status: bool = True) -> torch.Tensor:
        cg, cp = _c_gauss(g), _c_planes(planes)
        if image is None:
            image = torch.empty(self.num_pixels, dtype=torch.float32, device=self.device)
        elif image.numel() != self.num_pixels or not image.is_contiguous() or image.dtype != torch.float32:
            raise ValueError("image must be a contiguous float32 tensor of num_pixels elements")
        check(lib.ug_render_planes(self._h, ctypes.byref(cg), ctypes.byref(cp), image.data_ptr(), self._ws_ptr,
                                   _stream()), "ug_render_planes")
        self.forward_count += 1
        if check_status:
            code = self.status()
            if code == _lib.UG_ERR_CAPACITY:
                self.fit(g, planes)
                return self.render(g, planes, image, check_status)
            if code not in (_lib.UG_OK, _lib.UG_ERR_NONFINITE):
                check(code, "render status")
        return image

    def render_noalloc(self, g: GaussianTensors, planes: PlaneTensors, image: torch.Tensor) -> torch.Tensor:
        """The forward through ug_render_planes_noalloc: the library's static
        per-device workspace instead of this plan's (no backward follows it,
        and its device status cannot be read)."""
        cg, cp = _c_gauss(g), _c_planes(planes)
        if image.numel() != self.num_pixels or not image.is_contiguous() or image.dtype != torch.float32:
            raise ValueError("image must be a contiguous float32 tensor of num_pixels elements")
        check(lib.ug_render_planes_noalloc(self._h, ctypes.byref(cg), ctypes.byref(cp), image.data_ptr(), _stream()),
              "ug_render_planes_noalloc")
        return image

    def backward(self, g: GaussianTensors, planes: PlaneTensors, image: torch.Tensor, d_image: torch.Tensor,
                 grads: GaussianTensors | None = None, accumulate: bool = False) -> GaussianTensors:
        cg, cp = _c_gauss(g), _c_planes(planes)
        n = g.means.shape[0]
        if grads is None:
            dev = self.device
            grads = GaussianTensors(torch.empty(n, 3, device=dev), torch.empty(n, 6, device=dev),
                                    torch.empty(n, device=dev), torch.empty(n, device=dev))
        d_image = d_image.contiguous()
        if d_image.numel() != self.num_pixels or d_image.dtype != torch.float32:
            raise ValueError("d_image must be float32 with num_pixels elements")
        check(lib.ug_render_planes_backward(self._h, ctypes.byref(cg), ctypes.byref(cp), image.data_ptr(),
                                            d_image.data_ptr(), self._ws_ptr, grads.means.data_ptr(),
                                            grads.lraw.data_ptr(), grads.intensity.data_ptr(),
                                            grads.opacity.data_ptr(), 1 if accumulate else 0, _stream()),
              "ug_render_planes_backward")
        return grads

    def backward_mse(self, g: GaussianTensors, planes: PlaneTensors, image: torch.Tensor, target: torch.Tensor,
                     grads: GaussianTensors | None = None, accumulate: bool = False,
                     loss_buf: torch.Tensor | None = None) -> GaussianTensors:
        """Adjoint of the mean squared error against ``target`` (the gradient
        of the MSE formed inside the first adjoint kernel); the loss goes to
        loss_buf[0] if given (float32 device tensor)."""
        cg, cp = _c_gauss(g), _c_planes(planes)
        n = g.means.shape[0]
        if grads is None:
            dev = self.device
            grads = GaussianTensors(torch.empty(n, 3, device=dev), torch.empty(n, 6, device=dev),
                                    torch.empty(n, device=dev), torch.empty(n, device=dev))
        target = target.contiguous()
        if target.numel() != self.num_pixels or target.dtype != torch.float32:
            raise ValueError("target must be float32 with num_pixels elements")
        if loss_buf is not None and (loss_buf.dtype != torch.float32 or not loss_buf.is_cuda):
            raise ValueError("loss_buf must be a float32 device tensor")
        check(lib.ug_render_planes_backward_mse(self._h, ctypes.byref(cg), ctypes.byref(cp), image.data_ptr(),
                                                target.data_ptr(), self._ws_ptr, grads.means.data_ptr(),
                                                grads.lraw.data_ptr(), grads.intensity.data_ptr(),
                                                grads.opacity.data_ptr(), 1 if accumulate else 0,
                                                loss_buf.data_ptr() if loss_buf is not None else None, _stream()),
              "ug_render_planes_backward_mse")
        return grads

    def debug_records(self) -> np.ndarray:
        """The records of the last render as a numpy structured array (fields
        of ug_record; synchronises).  A test hook."""
        n = int(lib.ug_debug_records(self._h, self._ws_ptr, None, 0, _stream()))
        if n < 0:
            check(n, "ug_debug_records")
        arr = (_lib.UgRecord * max(n, 1))()
        got = int(lib.ug_debug_records(self._h, self._ws_ptr, arr, n, _stream()))
        if got < 0:
            check(got, "ug_debug_records")
        return np.ctypeslib.as_array(arr)[:n].copy()

    def debug_keys(self):
        """The sorted keys of the last render (key words, emission positions,
        record ids) and the tile ranges, as uint32 numpy arrays (synchronises).
        A test hook."""
        n = int(lib.ug_debug_keys(self._h, self._ws_ptr, None, None, None, None, 0, _stream()))
        if n < 0:
            check(n, "ug_debug_keys")
        key, eidx, rec = (np.empty(max(n, 1), dtype=np.uint32) for _ in range(3))
        ranges = np.empty(self.num_tiles + 1, dtype=np.uint32)
        got = int(lib.ug_debug_keys(self._h, self._ws_ptr, key.ctypes.data, eidx.ctypes.data, rec.ctypes.data,
                                    ranges.ctypes.data, n, _stream()))
        if got < 0:
            check(got, "ug_debug_keys")
        return key[:n], eidx[:n], rec[:n], ranges

    def quality(self, image: torch.Tensor, ref: torch.Tensor, data_range: float = 1.0):
        """Per-plane (ssim, mse) float64 device tensors of ``image`` against
        ``ref`` (both packed like this plan's renders): mean SSIM over the
        11 x 11 Gaussian windows inside each plane and MSE over its pixels."""
        for t in (image, ref):
            if t.numel() != self.num_pixels or not t.is_contiguous() or t.dtype != torch.float32:
                raise ValueError("images must be contiguous float32 tensors of num_pixels elements")
        nbytes = int(lib.ug_quality_workspace_bytes(self._h))
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (ws.data_ptr() + 255) // 256 * 256
        ssim = torch.empty(self.p, dtype=torch.float64, device=self.device)
        mse = torch.empty(self.p, dtype=torch.float64, device=self.device)
        check(lib.ug_image_quality(self._h, image.data_ptr(), ref.data_ptr(), float(data_range), ssim.data_ptr(),
                                   mse.data_ptr(), ptr, _stream()), "ug_image_quality")
        return ssim, mse

    def status(self, counts: bool = False):
        """Device status of the last render (synchronises); with counts=True
        (code, records, keys, in-support pairs, evaluated pairs), the last two
        0 unless the plan counts them (flags=1)."""
        out = (ctypes.c_int64 * 4)()
        code = lib.ug_plan_status(self._h, self._ws_ptr, out, _stream())
        if code == _lib.UG_ERR_HIP:
            check(code, "ug_plan_status")
        return (code, int(out[0]), int(out[1]), int(out[2]), int(out[3])) if counts else code

    # ---------------------------------------------------------------- measurement
    def profile_begin(self, stages=None, max_launches: int = 4096):
        """Start per-stage HIP-event timing on the launch stream."""
        names = _lib.STAGES if stages is None else stages
        mask = 0
        for nm in names:
            mask |= 1 << _lib.STAGES.index(nm)
        check(lib.ug_profile_begin(self._h, mask, int(max_launches)), "ug_profile_begin")

    def profile_read(self):
        """{stage: (total ms, launches)} since profile_begin; stops timing."""
        ms = (ctypes.c_float * _lib.UG_NUM_STAGES)()
        cnt = (ctypes.c_int32 * _lib.UG_NUM_STAGES)()
        check(lib.ug_profile_read(self._h, ms, cnt), "ug_profile_read")
        return {nm: (float(ms[i]), int(cnt[i])) for i, nm in enumerate(_lib.STAGES) if cnt[i]}

    def split_image(self, image: torch.Tensor):
        """Views of a packed image, one [H, W] per plane."""
        out, o = [], 0
        for W, H in self.wh:
            out.append(image[o:o + W * H].view(int(H), int(W)))
            o += int(W) * int(H)
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        # at interpreter exit the module's globals may already be gone: the
        # process is ending and the driver frees the device memory
        if h is not None and h.value and lib is not None:
            lib.ug_plan_destroy(h)
            self._h = None


def mse_grad(image: torch.Tensor, target: torch.Tensor, d_image: torch.Tensor | None = None,
             loss_buf: torch.Tensor | None = None):
    """(loss tensor [1], d_image) of the mean squared error, on the device."""
    m = image.numel()
    if d_image is None:
        d_image = torch.empty_like(image)
    if loss_buf is None:
        loss_buf = torch.zeros(_lib.UG_MSE_SCRATCH_FLOATS, dtype=torch.float32, device=image.device)
    check(lib.ug_mse_grad(image.data_ptr(), target.data_ptr(), m, d_image.data_ptr(), loss_buf.data_ptr(),
                          _stream()), "ug_mse_grad")
    return loss_buf[:1], d_image


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float, step: int,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    check(lib.ug_adam_step(param.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), param.numel(),
                           float(lr), float(beta1), float(beta2), float(eps), int(step), _stream()),
          "ug_adam_step")


def to_device(obj, device="cuda"):
    """synth.Gaussians / synth.Planes (numpy) -> tensor tuples on the device."""
    if hasattr(obj, "lraw"):
        return GaussianTensors(*(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
                                 for a in (obj.means, obj.lraw, obj.intensity, obj.opacity)))
    return PlaneTensors(*(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
                          for a in (obj.rot, obj.origin, obj.spacing)))
