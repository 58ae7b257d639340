"""Helpers shared by the GPU parity tests (HIP path vs the FP64 oracle)."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import pool

IMAGE_TOL = 1e-4   # max abs error / peak |oracle| intensity
GRAD_TOL = 1e-3    # max abs error / max |oracle gradient|, per tensor
AMBIG_FRAC = 1e-3  # pixels allowed to rely on the cut-off ambiguity interval
# Per element: |gpu - ref| <= GRAD_ELEM_REL |ref| + GRAD_ELEM_FLOOR max|ref|.
# The floor covers entries that are sums of terms cancelling far below the
# tensor's scale (FP32 keeps about 1e-7 of each term, not of their sum).
GRAD_ELEM_REL = 1e-3
GRAD_ELEM_FLOOR = 1e-5
# Above this many Gaussian-point pairs the oracle runs in worker processes.
POOL_PAIRS = 2e7


def _big(g, m: int) -> bool:
    return float(np.asarray(g.means).shape[0]) * m > POOL_PAIRS


def reference_points(g, X, params):
    """(c_hat, alpha_hat) of the oracle at the world points X."""
    op = oracle_params(params)
    return pool.render_points(g, X, op) if _big(g, X.shape[0]) else oracle.render_points(g, X, op)


def reference_grad(g, X, dout, params):
    """The oracle's gradient of sum dout(x) c_hat(x) at the world points X."""
    op = oracle_params(params)
    nz = int(np.count_nonzero(dout))
    return pool.grad_points(g, X, dout, op) if _big(g, nz) else oracle.grad_points(g, X, dout, op)


def oracle_params(params) -> oracle.Params:
    """The FP32 values the GPU received, upcast (same inputs on both sides)."""
    f = np.float32
    return oracle.Params(beta=float(f(params.beta)), chi2=float(f(params.chi2)),
                         bg_alpha=float(f(params.bg_alpha)), bg_color=float(f(params.bg_color)))


def check_image(gpu: np.ndarray, g, planes, params, pix=None, tol_rel=IMAGE_TOL, peak=None, ref=None):
    """Element-wise parity; pixels off by more than tol must lie within tol of
    the oracle's cut-off ambiguity interval.  ``ref`` = the oracle's c_hat at
    these pixels if already computed.  Returns a stats dict."""
    op = oracle_params(params)
    X = oracle.plane_points(planes, pix)
    if ref is None:
        ref, _ = reference_points(g, X, params)
    gpu = np.asarray(gpu, dtype=np.float64).reshape(-1)
    assert gpu.shape == ref.shape
    assert np.all(np.isfinite(gpu)), "non-finite GPU output"
    pk = float(np.abs(ref).max()) if peak is None else float(peak)
    tol = tol_rel * max(pk, 1e-30)
    diff = np.abs(gpu - ref)
    bad = np.nonzero(diff > tol)[0]
    n_amb = 0
    if bad.size:
        amb = pool.ambiguity_points if _big(g, bad.size) else oracle.ambiguity_points
        lo, hi, k = amb(g, X[bad], op)
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


def check_grads(gpu: dict, ref: dict, tol_rel=GRAD_TOL, elem_rel=GRAD_ELEM_REL, elem_floor=GRAD_ELEM_FLOOR):
    """Per tensor: max abs error / max |ref| <= tol_rel, and per element
    |gpu - ref| <= elem_rel |ref| + elem_floor max|ref|.  Returns, per tensor,
    the max-normalised error and the worst per-element ratio (error over its
    bound)."""
    errs = {}
    for name in ("means", "lraw", "intensity", "opacity"):
        a = np.asarray(gpu[name], dtype=np.float64).reshape(ref[name].shape)
        b = ref[name]
        assert np.all(np.isfinite(a)), f"non-finite gradient {name}"
        scale = float(np.abs(b).max())
        diff = np.abs(a - b)
        err = float(diff.max()) / max(scale, 1e-300)
        bound = elem_rel * np.abs(b) + elem_floor * max(scale, 1e-300)
        ratio = diff / bound
        worst = int(np.argmax(ratio))
        # the same ratio with a floor ten times lower, reported only
        tight = float(np.max(diff / (elem_rel * np.abs(b) + 0.1 * elem_floor * max(scale, 1e-300))))
        errs[name] = {"max_rel": err, "elem_worst": float(ratio.reshape(-1)[worst]), "elem_worst_floor_1e-6": tight}
        assert err <= tol_rel, f"gradient {name}: relative max error {err:.3e} > {tol_rel}"
        assert ratio.reshape(-1)[worst] <= 1.0, (
            f"gradient {name}[{np.unravel_index(worst, b.shape)}]: gpu {a.reshape(-1)[worst]:.8g} oracle "
            f"{b.reshape(-1)[worst]:.8g} exceeds {elem_rel} relative + {elem_floor} of max|ref| ({scale:.4g})")
    return errs
