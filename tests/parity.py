"""Helpers shared by the GPU parity tests (HIP path vs the FP64 oracle)."""
from __future__ import annotations

import numpy as np

import oracle

IMAGE_TOL = 1e-4   # max abs error / peak |oracle| intensity
GRAD_TOL = 1e-3    # max abs error / max |oracle gradient|, per tensor
AMBIG_FRAC = 1e-3  # pixels allowed to rely on the cut-off ambiguity interval


def oracle_params(params) -> oracle.Params:
    """The FP32 values the GPU received, upcast (same inputs on both sides)."""
    f = np.float32
    return oracle.Params(beta=float(f(params.beta)), chi2=float(f(params.chi2)),
                         bg_alpha=float(f(params.bg_alpha)), bg_color=float(f(params.bg_color)))


def check_image(gpu: np.ndarray, g, planes, params, pix=None, tol_rel=IMAGE_TOL, peak=None):
    """Element-wise parity; pixels off by more than tol must lie within tol of
    the oracle's cut-off ambiguity interval.  Returns a stats dict."""
    op = oracle_params(params)
    X = oracle.plane_points(planes, pix)
    ref, _ = oracle.render_points(g, X, op)
    gpu = np.asarray(gpu, dtype=np.float64).reshape(-1)
    assert gpu.shape == ref.shape
    assert np.all(np.isfinite(gpu)), "non-finite GPU output"
    pk = float(np.abs(ref).max()) if peak is None else float(peak)
    tol = tol_rel * max(pk, 1e-30)
    diff = np.abs(gpu - ref)
    bad = np.nonzero(diff > tol)[0]
    n_amb = 0
    if bad.size:
        lo, hi, k = oracle.ambiguity_points(g, X[bad], op)
        dist = np.maximum(lo - gpu[bad], gpu[bad] - hi)
        worst = int(np.argmax(dist))
        assert np.all(dist <= tol), (
            f"{int(np.sum(dist > tol))} pixels outside tolerance; worst idx {int(bad[worst])}: gpu "
            f"{gpu[bad[worst]]:.8g} oracle {ref[bad[worst]]:.8g} interval [{lo[worst]:.8g}, {hi[worst]:.8g}] "
            f"tol {tol:.3g}")
        n_amb = int(np.sum(k > 0))
        assert n_amb <= max(1, AMBIG_FRAC * gpu.size), f"{n_amb} ambiguous pixels"
    return {"max_abs": float(diff.max()), "tol": tol, "peak": pk, "ambiguous": n_amb,
            "max_rel_peak": float(diff.max() / max(pk, 1e-30))}


def check_image_box_support(gpu: np.ndarray, g, planes, params, pix=None, tol_rel=IMAGE_TOL):
    """Element-wise parity against the paper-literal box-support reference;
    pixels off by more than tol must lie within tol of the interval spanned
    by its borderline decisions.  Returns a stats dict."""
    from oracle.box_support import render_box_support
    ref, _, lo, hi, k = render_box_support(g, planes, oracle_params(params), pix=pix)
    gpu = np.asarray(gpu, dtype=np.float64).reshape(-1)
    assert gpu.shape == ref.shape
    assert np.all(np.isfinite(gpu)), "non-finite GPU output"
    pk = float(np.abs(ref).max())
    tol = tol_rel * max(pk, 1e-30)
    diff = np.abs(gpu - ref)
    bad = diff > tol
    dist = np.maximum(lo - gpu, gpu - hi)
    assert np.all(dist[bad] <= tol), f"{int(np.sum(dist[bad] > tol))} pixels outside tolerance"
    n_amb = int(np.sum(k > 0))
    assert n_amb <= max(1, AMBIG_FRAC * gpu.size), f"{n_amb} ambiguous pixels"
    return {"max_abs": float(diff.max()), "tol": tol, "peak": pk, "ambiguous": n_amb,
            "max_rel_peak": float(diff.max() / max(pk, 1e-30))}


def check_grads(gpu: dict, ref: dict, tol_rel=GRAD_TOL):
    errs = {}
    for name in ("means", "lraw", "intensity", "opacity"):
        a = np.asarray(gpu[name], dtype=np.float64).reshape(ref[name].shape)
        assert np.all(np.isfinite(a)), f"non-finite gradient {name}"
        scale = float(np.abs(ref[name]).max())
        err = float(np.abs(a - ref[name]).max()) / max(scale, 1e-300)
        errs[name] = err
        assert err <= tol_rel, f"gradient {name}: relative max error {err:.3e} > {tol_rel}"
    return errs
