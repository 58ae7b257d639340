"""Synthetic reconstruction-quality workload: the evaluation protocol of
Section 5.2 on a seeded stand-in for its volumes.

The ground truth is a seeded phantom of Gaussians in the unit cube (a bright
thin shell, a textured interior, an empty exterior); its images on probe
planes (rendered by this library) stand in for the slices of a scanned
volume.  Training follows Section 4.5 (uniform means, intensity
0.5, alpha 0.731, raw factor entries U[4, 5); Adam with lr 0.05 and a
decaying mean lr), every step over all training slices at once (one
hipGraph).  The training slices are ``size`` linearly spaced axial slices
(full coverage), half as many (50%), or half as many tilted about x and y by
U(-5, 5) degrees (jitter).  Scoring: ``size`` linearly spaced axial,
coronal and sagittal slices of the model against the ground truth's, SSIM
and PSNR per slice (``ug_image_quality``), averaged per view; coronal and
sagittal slices are never seen in training.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import raster as R
from . import synth
from .step import AdamConfig, TrainStep

VIEWS = ("axial", "coronal", "sagittal")
CASES = {"full": (1.0, 0.0), "half": (0.5, 0.0), "half_jitter": (0.5, 5.0)}


@dataclasses.dataclass
class ReconSetup:
    size: int = 160                  # slices are size^2 pixels of the unit cube
    n_truth: int = 30_000            # Gaussians of the ground-truth phantom
    n_model: int = 100_000           # Gaussians fitted
    steps: int = 300
    seed: int = 0
    check_every: int = 50


def truth_gaussians(setup: ReconSetup) -> synth.Gaussians:
    return synth.phantom_gaussians(setup.n_truth, 4000 + setup.seed)


def eval_planes(setup: ReconSetup) -> synth.Planes:
    """All three views, ``size`` slices each, in VIEWS order."""
    parts = [synth.volume_sweep(v, setup.size, setup.size) for v in VIEWS]
    return synth.Planes(np.concatenate([p.rot for p in parts]), np.concatenate([p.origin for p in parts]),
                        np.concatenate([p.spacing for p in parts]), np.concatenate([p.wh for p in parts]))


def train_planes(setup: ReconSetup, case: str) -> synth.Planes:
    frac, jitter = CASES[case]
    return synth.volume_sweep("axial", max(1, round(setup.size * frac)), setup.size, jitter, 5000 + setup.seed)


class Scorer:
    """Renders a Gaussian set on the evaluation slices and scores it against
    the ground truth's images there."""

    def __init__(self, setup: ReconSetup, truth: R.GaussianTensors, params: R.Params, device):
        pl = eval_planes(setup)
        self.planes = R.to_device(pl, device)
        self.size = setup.size
        self.params = params
        self.device = device
        plan = R.Plan(truth.means.shape[0], pl.wh, params, device=device)
        plan.fit(truth, self.planes)
        self.truth_images = plan.render(truth, self.planes)
        self.wh = pl.wh
        self._plan = None

    def images(self, g: R.GaussianTensors) -> torch.Tensor:
        n = g.means.shape[0]
        if self._plan is None or self._plan.n != n:
            self._plan = R.Plan(n, self.wh, self.params, device=self.device)
        self._plan.fit(g, self.planes)
        return self._plan.render(g, self.planes)

    def quality_ms(self, image: torch.Tensor, reps: int = 10) -> float:
        """Average time of one ug_image_quality call over every evaluation
        slice (HIP events on the launch stream)."""
        self._plan.quality(image, self.truth_images, 1.0)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            self._plan.quality(image, self.truth_images, 1.0)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / reps

    def score(self, g: R.GaussianTensors) -> dict:
        img = self.images(g)
        ssim, mse = self._plan.quality(img, self.truth_images, 1.0)
        ssim, mse = ssim.cpu().numpy(), mse.cpu().numpy()
        psnr = 10.0 * np.log10(1.0 / np.maximum(mse, 1e-30))
        out = {"ssim": {}, "psnr": {}}
        for k, v in enumerate(VIEWS):
            sl = slice(k * self.size, (k + 1) * self.size)
            out["ssim"][v] = float(np.mean(ssim[sl]))
            out["psnr"][v] = float(np.mean(psnr[sl]))
        return out


def run_case(setup: ReconSetup, case: str, device=None, params: R.Params | None = None,
             scorer: Scorer | None = None) -> dict:
    """Fits one case and scores it; returns the scores before and after
    training, the losses and the training time."""
    device = torch.device(device) if device is not None else torch.device("cuda", 0)
    params = params or R.Params()
    truth = R.to_device(truth_gaussians(setup), device)
    scorer = scorer or Scorer(setup, truth, params, device)
    tpl = train_planes(setup, case)
    tpd = R.to_device(tpl, device)
    tplan = R.Plan(truth.means.shape[0], tpl.wh, params, device=device)
    tplan.fit(truth, tpd)
    target = tplan.render(truth, tpd)
    del tplan
    model = R.to_device(synth.paper_init(setup.n_model, 6000 + setup.seed), device)
    before = scorer.score(model)
    ts = TrainStep(model, tpd, tpl.wh, target, params, adam=AdamConfig(decay_steps=setup.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = ts.run(setup.steps, check_every=setup.check_every)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    after = scorer.score(ts.params)
    return {"case": case, "train_slices": tpl.p, "steps": setup.steps, "gaussians": setup.n_model,
            "train_s": train_s, "ms_per_step": 1e3 * train_s / max(setup.steps, 1),
            "loss_first_check": losses[0] if losses else math.nan, "loss_last": losses[-1] if losses else math.nan,
            "init": before, "trained": after}
