"""Launch-configuration autotuner for the probe-plane rasterizer.

Searches tile shape, pixels per lane, LDS batch, binning box and the
forward's split (UG_FLAG_SPLIT_FORWARD) for a given workload by timing the
library's own forward + backward on the device, and checks that every
candidate renders the same image and back-propagates the same gradients:
bit for bit within a tile shape (the split: shape, batch and box); across them the
tile-relative FP32 coordinates round differently, so images to 2e-5 of the
peak (a fifth of the parity tolerance) except for rare pixels whose pair
sits on the cut-off, and gradients as GRAD_REL below says.  Results can be cached per
workload signature in a JSON file.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os

import numpy as np
import torch

from . import raster as R

SHAPES = ((8, 8, 1), (16, 8, 2), (8, 16, 1), (16, 16, 2), (32, 8, 4), (32, 16, 4), (16, 32, 2), (32, 32, 4))
BATCHES = (32, 64, 128, 256)
BOXES = (R._lib.UG_BOX_PAPER, R._lib.UG_BOX_CONIC, R._lib.UG_BOX_ROWS)
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
# Tile shapes round the tile-relative pixel coordinates differently, so a
# pair whose d^2 sits on the cut-off can flip between shapes and move its own
# Gaussian's gradient by a sizeable fraction of the largest entry (1.4e-3 of
# it seen at the 1M-Gaussian workload).  Each candidate's gradients are
# therefore checked twice: on a cut-off-free probe (the workload's first 512
# Gaussians on its first two planes with chi^2 = inf, where nothing can flip)
# to GRAD_REL of each tensor's largest entry, and on the workload itself
# normwise to GRAD_REL_WORKLOAD, a bound for gross errors at the parity
# tolerance.
GRAD_REL = 1e-5
GRAD_REL_WORKLOAD = 1e-3


def signature(n: int, wh) -> str:
    wh = np.asarray(wh, dtype=np.int32)
    h = hashlib.sha1(wh.tobytes()).hexdigest()[:12]
    dev = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    return f"n={n};p={len(wh)};wh={h};dev={dev}"


def _time_candidate(params: R.Params, g, planes, wh, d_image, steps: int):
    plan = R.Plan(g.means.shape[0], wh, params)
    plan.fit(g, planes)
    img = torch.empty(plan.num_pixels, device=plan.device)
    grads = R.GaussianTensors(torch.empty_like(g.means), torch.empty_like(g.lraw),
                              torch.empty_like(g.intensity), torch.empty_like(g.opacity))
    for _ in range(2):
        plan.render(g, planes, img, check_status=False)
        plan.backward(g, planes, img, d_image, grads)
    torch.cuda.synchronize()
    code = plan.status()
    if code != 0:
        raise RuntimeError(f"status {code}")
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        plan.render(g, planes, img, check_status=False)
        plan.backward(g, planes, img, d_image, grads)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps, img.clone(), plan.status(counts=True), [t.clone() for t in grads]


def _probe_grads(params: R.Params, g, planes, wh, d_probe):
    """Gradients of the cut-off-free probe (chi^2 = inf) in a candidate's
    launch configuration."""
    prm = dataclasses.replace(params, chi2=float("inf"))
    plan = R.Plan(g.means.shape[0], wh, prm)
    plan.fit(g, planes)
    img = plan.render(g, planes)
    grads = plan.backward(g, planes, img, d_probe)
    torch.cuda.synchronize()
    return [t.clone() for t in grads]


def tune(g: R.GaussianTensors, planes: R.PlaneTensors, wh, base: R.Params | None = None, steps: int = 5,
         shapes=SHAPES, batches=BATCHES, boxes=BOXES, verbose: bool = False):
    """Returns (best Params, list of result dicts).  Two stages: tile shape x
    box at LDS batch 64, then the LDS batch for the three best."""
    base = base or R.Params()
    rng = np.random.default_rng(0)
    npx = int(np.sum(np.asarray(wh, dtype=np.int64)[:, 0] * np.asarray(wh, dtype=np.int64)[:, 1]))
    d_image = torch.from_numpy(rng.standard_normal(npx).astype(np.float32)).to(g.means.device)
    results = []
    ref_img = {}
    ref_grad = {}
    ref_probe = {}
    peak = None
    n_pr, p_pr = min(512, g.means.shape[0]), min(2, planes.rot.shape[0])
    g_pr = R.GaussianTensors(*(t[:n_pr].contiguous() for t in g))
    pl_pr = R.PlaneTensors(*(t[:p_pr].contiguous() for t in planes))
    wh_pr = np.asarray(wh, dtype=np.int32)[:p_pr]
    d_probe = torch.from_numpy(rng.standard_normal(int(np.sum(wh_pr[:, 0].astype(np.int64) * wh_pr[:, 1])))
                               .astype(np.float32)).to(g.means.device)

    def run(tw, th, ppl, bg, box, split=False):
        nonlocal peak
        flags = (base.flags | R._lib.UG_FLAG_SPLIT_FORWARD) if split else (base.flags & ~R._lib.UG_FLAG_SPLIT_FORWARD)
        prm = dataclasses.replace(base, tile_w=tw, tile_h=th, px_per_lane=ppl, lds_batch=bg, box_mode=box,
                                  flags=flags)
        ms, img, st, grads = _time_candidate(prm, g, planes, wh, d_image, steps)
        probe = _probe_grads(prm, g_pr, pl_pr, wh_pr, d_probe) if n_pr > 0 else []
        if peak is None:
            peak = float(img.abs().max())
        # the split forward groups each pixel's sum by alternate rounds of
        # lds_batch keys, so its image also depends on the batch and on the
        # binning (which keys a tile holds)
        key = (tw, th, bg, box) if split else (tw, th)
        off = 0
        gerr = {}
        if key in ref_img:
            if not torch.equal(img, ref_img[key]):
                raise RuntimeError(f"candidate {prm} renders a different image than its tile shape's first")
            if not all(torch.equal(a, b) for a, b in zip(grads, ref_grad[key])):
                raise RuntimeError(f"candidate {prm}: gradients differ from its tile shape's first")
            if not all(torch.equal(a, b) for a, b in zip(probe, ref_probe[key])):
                raise RuntimeError(f"candidate {prm}: probe gradients differ from its tile shape's first")
        else:
            ref_img[key] = img
            ref_grad[key] = grads
            ref_probe[key] = probe
            first_g = next(iter(ref_grad.values()))
            first_p = next(iter(ref_probe.values()))
            for name, a, b, ap, bp in zip(("means", "lraw", "intensity", "opacity"), grads, first_g, probe, first_p):
                err = float(torch.linalg.vector_norm((a - b).double())) / max(
                    float(torch.linalg.vector_norm(b.double())), 1e-300)
                perr = float((ap - bp).abs().max()) / max(float(bp.abs().max()), 1e-30)
                gerr[name] = (err, perr)
                if perr > GRAD_REL:
                    raise RuntimeError(f"candidate {prm}: probe gradient {name} differs from the first tile "
                                       f"shape's by {perr:.3e} of its largest entry")
                if err > GRAD_REL_WORKLOAD:
                    raise RuntimeError(f"candidate {prm}: gradient {name} differs from the first tile shape's by "
                                       f"{err:.3e} (normwise)")
            first = next(iter(ref_img.values()))
            # Pixels with a pair on the cut-off (d^2 = chi^2 to rounding) may
            # legitimately flip between shapes; they must stay rare.
            off = int(((img - first).abs() > 2e-5 * max(peak, 1e-30)).sum())
            if off > max(1, 1e-4 * img.numel()):
                raise RuntimeError(f"candidate {prm}: {off} pixels differ from the first tile shape")
        rec = {"tile_w": tw, "tile_h": th, "px_per_lane": ppl, "lds_batch": bg, "box_mode": box,
               "split_forward": split, "ms": ms,
               "records": st[1], "keys": st[2], "cutoff_flips": off,
               "grad_vs_first_shape": {k: {"workload_normwise": v[0], "probe_max_by_largest": v[1]}
                                       for k, v in gerr.items()}}
        results.append(rec)
        if verbose:
            print(rec, flush=True)
        return rec

    for tw, th, ppl in shapes:
        for box in boxes:
            run(tw, th, ppl, 64, box)
    best = sorted(results, key=lambda r: r["ms"])[:3]
    for b in best:
        for bg in batches:
            if bg != 64:
                run(b["tile_w"], b["tile_h"], b["px_per_lane"], bg, b["box_mode"])
    # the forward split (two waves per band) for the three best so far
    for b in sorted(results, key=lambda r: r["ms"])[:3]:
        if split_ok(b["tile_h"], b["lds_batch"]):
            run(b["tile_w"], b["tile_h"], b["px_per_lane"], b["lds_batch"], b["box_mode"], split=True)
    top = min(results, key=lambda r: r["ms"])
    flags = base.flags | R._lib.UG_FLAG_SPLIT_FORWARD if top["split_forward"] else base.flags
    params = dataclasses.replace(base, tile_w=top["tile_w"], tile_h=top["tile_h"], px_per_lane=top["px_per_lane"],
                                 lds_batch=top["lds_batch"], box_mode=top["box_mode"], flags=flags)
    return params, results


def split_ok(tile_h: int, lds_batch: int) -> bool:
    """The split forward's staging fits (tile_h / 8 bands x 2 waves x
    max(batch, 64) records x 80 B <= 128 KB)."""
    return (tile_h // 8) * 2 * max(lds_batch, 64) * 80 <= 128 * 1024


def load_cache(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def cached_params(sig: str, path: str = CACHE) -> R.Params | None:
    entry = load_cache(path).get(sig)
    if entry is None:
        return None
    prm = R.Params(**{k: entry[k] for k in ("tile_w", "tile_h", "px_per_lane", "lds_batch", "box_mode")})
    prm.flags = int(entry.get("flags", 0))
    return prm


def store(sig: str, params: R.Params, ms: float, path: str = CACHE):
    cache = load_cache(path)
    cache[sig] = {"tile_w": params.tile_w, "tile_h": params.tile_h, "px_per_lane": params.px_per_lane,
                  "lds_batch": params.lds_batch, "box_mode": params.box_mode,
                  "flags": params.flags & R._lib.UG_FLAG_SPLIT_FORWARD, "ms": ms}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
