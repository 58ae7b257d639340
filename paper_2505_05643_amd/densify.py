"""Densification and pruning between training steps (the step after the
update on the training path): the Section 4.2 draw y = mu + L^-T z, the
per-Gaussian gradient statistic, and the clone / split / prune pass.  The
rule is stated in include/ug.h (ug_densify); this module only marshals
arguments to the library.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from ._lib import lib, check
from . import raster as R


@dataclasses.dataclass
class DensifyParams:
    beta: float = 1e-4
    min_opacity: float = 0.005
    grad_thresh: float = 2e-4
    split_size: float = 1.0
    max_size: float = 0.0
    split_factor: float = 1.6

    def to_c(self) -> _lib.UgDensifyParams:
        return _lib.UgDensifyParams(self.beta, self.min_opacity, self.grad_thresh, self.split_size,
                                    self.max_size, self.split_factor)


def sample_gaussians(g: R.GaussianTensors, idx: torch.Tensor, z: torch.Tensor, beta: float = 1e-4) -> torch.Tensor:
    """[k, 3] draws means[idx] + L^-T z from standard normals z [k, 3]."""
    idx = idx.to(torch.int32).contiguous()
    z = z.contiguous()
    if z.dtype != torch.float32 or z.shape != (idx.shape[0], 3):
        raise ValueError("z must be float32 [k, 3]")
    out = torch.empty(idx.shape[0], 3, dtype=torch.float32, device=g.means.device)
    cg = R._c_gauss(g)
    check(lib.ug_sample_gaussians(ctypes.byref(cg), float(beta), idx.data_ptr(), z.data_ptr(), idx.shape[0],
                                  out.data_ptr(), R._stream()), "ug_sample_gaussians")
    return out


def accumulate_grad_norm(d_means: torch.Tensor, acc: torch.Tensor, cnt: torch.Tensor,
                         plan: R.Plan | None = None) -> None:
    """acc += |d_means| per Gaussian, cnt += 1 (float32 / int32 device
    tensors); skipped on the device if ``plan``'s last render overflowed."""
    n = d_means.shape[0]
    if acc.shape != (n,) or cnt.shape != (n,) or acc.dtype != torch.float32 or cnt.dtype != torch.int32:
        raise ValueError("acc float32 [n], cnt int32 [n]")
    check(lib.ug_accumulate_grad_norm(plan._h if plan is not None else None,
                                      plan._ws_ptr if plan is not None else None,
                                      d_means.contiguous().data_ptr(), n, acc.data_ptr(), cnt.data_ptr(),
                                      R._stream()), "ug_accumulate_grad_norm")


def densify(g: R.GaussianTensors, acc: torch.Tensor, cnt: torch.Tensor, z: torch.Tensor,
            params: DensifyParams | None = None) -> R.GaussianTensors:
    """The clone / split / prune pass; returns the new Gaussian tensors
    (reads the output count from the device, so it synchronises)."""
    params = params or DensifyParams()
    n = g.means.shape[0]
    dev = g.means.device
    if z.dtype != torch.float32 or z.shape != (n, 2, 3):
        raise ValueError("z must be float32 [n, 2, 3]")
    cap = 2 * n
    out = R.GaussianTensors(torch.empty(cap, 3, device=dev), torch.empty(cap, 6, device=dev),
                            torch.empty(cap, device=dev), torch.empty(cap, device=dev))
    ws = torch.empty(max(1, (lib.ug_densify_workspace_bytes(n) + 3) // 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    cg = R._c_gauss(g)
    co = _lib.UgGaussiansMut(out.means.data_ptr(), out.lraw.data_ptr(), out.intensity.data_ptr(),
                             out.opacity.data_ptr(), cap)
    dp = params.to_c()
    check(lib.ug_densify(ctypes.byref(cg), acc.contiguous().data_ptr(), cnt.contiguous().data_ptr(),
                         z.contiguous().data_ptr(), ctypes.byref(dp), ctypes.byref(co), cap, count.data_ptr(),
                         ws.data_ptr(), R._stream()), "ug_densify")
    m = int(count.item())
    return R.GaussianTensors(*(t[:m].clone() for t in out))
