"""One training step of the Gaussians (render, MSE, adjoint, Adam) as a hipGraph.

The whole step is enqueued on one stream with no host synchronisation and
no allocation, so it is captured once with ``torch.cuda.CUDAGraph`` and
replayed.  The Adam step counter lives in device memory and the Adam kernel
skips itself when the render overflowed its capacity; ``run`` checks the
status every ``check_every`` steps and, on an overflow, re-sizes the plan,
captures again and redoes the step.

Each step also adds |dL/dmu| to a per-Gaussian statistic; ``densify``
(between steps) clones, splits and prunes by it (include/ug.h, ug_densify),
then re-plans for the new number of Gaussians and captures again.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from ._lib import lib, check
from . import densify as D
from . import raster as R


@dataclasses.dataclass
class AdamConfig:
    """Section 4.5: Adam, lr 0.05 for all parameters but the means, which
    start at 1.6e-4 and decay exponentially (final value: 1% of the start,
    an assumption; the paper does not give it)."""
    lr_means: float = 1.6e-4
    lr_means_final: float = 1.6e-6
    decay_steps: int = 2000
    lr: float = 0.05
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def to_c(self) -> _lib.UgAdamParams:
        return _lib.UgAdamParams(self.lr_means, self.lr_means_final, self.decay_steps, self.lr, self.beta1,
                                 self.beta2, self.eps)


def _mut(g: R.GaussianTensors) -> _lib.UgGaussiansMut:
    return _lib.UgGaussiansMut(g.means.data_ptr(), g.lraw.data_ptr(), g.intensity.data_ptr(),
                               g.opacity.data_ptr(), g.means.shape[0])


def adam_gaussians(params: R.GaussianTensors, grads: R.GaussianTensors, m1: R.GaussianTensors,
                   m2: R.GaussianTensors, cfg: AdamConfig, step_dev: torch.Tensor, plan: R.Plan | None = None):
    """One Adam step over the four tensors (step number read on the device)."""
    hp = cfg.to_c()
    a, b, c, d = _mut(params), _mut(grads), _mut(m1), _mut(m2)
    check(lib.ug_adam_gaussians(plan._h if plan is not None else None,
                                plan._ws_ptr if plan is not None else None,
                                ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                                ctypes.byref(hp), step_dev.data_ptr(), R._stream()), "ug_adam_gaussians")


class TrainStep:
    """Fits the Gaussians ``params`` (updated in place) to ``target`` images on
    the planes ``planes`` (both device tensors whose storage stays fixed; new
    poses or targets can be copied into them between steps)."""

    def __init__(self, params: R.GaussianTensors, planes: R.PlaneTensors, wh, target: torch.Tensor,
                 render_params: R.Params | None = None, adam: AdamConfig | None = None, headroom: float = 1.5,
                 native_graph: bool = False):
        self.native = native_graph  # capture with ug_step_capture instead of torch's graph capture
        self.params = params
        self.planes = planes
        self.target = target
        self.adam = adam or AdamConfig()
        self.headroom = headroom
        dev = params.means.device
        self.plan = R.Plan(params.means.shape[0], wh, render_params, device=dev)
        self.plan.fit(params, planes, headroom)
        z = lambda t: torch.zeros_like(t)  # noqa: E731
        self.grads = R.GaussianTensors(*(z(t) for t in params))
        self.m1 = R.GaussianTensors(*(z(t) for t in params))
        self.m2 = R.GaussianTensors(*(z(t) for t in params))
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.image = torch.empty(self.plan.num_pixels, device=dev)
        self.loss_buf = torch.zeros(_lib.UG_MSE_SCRATCH_FLOATS, device=dev)
        self._reset_stats()
        self.graph = None

    def _reset_stats(self):
        n = self.params.means.shape[0]
        dev = self.params.means.device
        self.grad_acc = torch.zeros(n, dtype=torch.float32, device=dev)
        self.grad_cnt = torch.zeros(n, dtype=torch.int32, device=dev)

    # ---------------------------------------------------------------- eager
    def enqueue(self):
        """Enqueue one step on the current stream (no synchronisation)."""
        self.plan.render(self.params, self.planes, self.image, check_status=False)
        self.plan.backward_mse(self.params, self.planes, self.image, self.target, self.grads, loss_buf=self.loss_buf)
        D.accumulate_grad_norm(self.grads.means, self.grad_acc, self.grad_cnt, self.plan)
        adam_gaussians(self.params, self.grads, self.m1, self.m2, self.adam, self.step_dev, self.plan)

    # ---------------------------------------------------------------- graph
    def capture(self):
        """Capture one step as a hipGraph (the capture itself runs no step)."""
        self.graph = None
        torch.cuda.synchronize()
        if self.native:
            cp = R._c_planes(self.planes)
            hp = self.adam.to_c()
            p, gr, a, b = _mut(self.params), _mut(self.grads), _mut(self.m1), _mut(self.m2)
            check(lib.ug_step_capture(self.plan._h, ctypes.byref(p), ctypes.byref(cp), self.target.data_ptr(),
                                      self.image.data_ptr(), self.plan._ws_ptr, ctypes.byref(gr), ctypes.byref(a),
                                      ctypes.byref(b), ctypes.byref(hp), self.step_dev.data_ptr(),
                                      self.loss_buf.data_ptr(), self.grad_acc.data_ptr(), self.grad_cnt.data_ptr()),
                  "ug_step_capture")
            self.graph = "native"
            return self.graph
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.enqueue()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        if self.native:
            check(lib.ug_step_replay(self.plan._h, R._stream()), "ug_step_replay")
        else:
            self.graph.replay()

    # ---------------------------------------------------------------- driver
    def run(self, steps: int, use_graph: bool = True, check_every: int = 1):
        """Runs ``steps`` steps; returns the list of losses read at each check."""
        losses = []
        start = self.step_count
        done = 0
        while done < steps:
            (self.replay if use_graph else self.enqueue)()
            done += 1
            if done % check_every == 0 or done == steps:
                code = self.plan.status()
                if code == _lib.UG_ERR_CAPACITY:
                    # every Adam launch since the overflow skipped itself and
                    # left the device step counter alone: re-size, re-capture
                    # and redo the steps that did not happen
                    self.plan.fit(self.params, self.planes, self.headroom)
                    self.graph = None
                    done = self.step_count - start
                    continue
                if code not in (_lib.UG_OK, _lib.UG_ERR_NONFINITE):
                    check(code, "train step")
                losses.append(float(self.loss_buf[0]))
        return losses

    @property
    def step_count(self) -> int:
        return int(self.step_dev.item())

    # ---------------------------------------------------------------- densify
    def densify(self, params: "D.DensifyParams | None" = None, seed: int = 0) -> int:
        """Clone / split / prune by the accumulated statistic; returns the new
        number of Gaussians.  ``self.params`` then holds new tensors (the old
        ones are not updated any more); the Adam moments of the new set start
        at zero and the statistic restarts.  Synchronises."""
        torch.cuda.synchronize()
        n = self.params.means.shape[0]
        dev = self.params.means.device
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        z = torch.randn(n, 2, 3, generator=gen, device=dev)
        new = D.densify(self.params, self.grad_acc, self.grad_cnt, z, params)
        self.params = R.GaussianTensors(*(t.contiguous() for t in new))
        z0 = lambda t: torch.zeros_like(t)  # noqa: E731
        self.grads = R.GaussianTensors(*(z0(t) for t in self.params))
        self.m1 = R.GaussianTensors(*(z0(t) for t in self.params))
        self.m2 = R.GaussianTensors(*(z0(t) for t in self.params))
        self.plan = R.Plan(self.params.means.shape[0], self.plan.wh, self.plan.params, device=dev)
        self.plan.fit(self.params, self.planes, self.headroom)
        self._reset_stats()
        self.graph = None
        return self.params.means.shape[0]
