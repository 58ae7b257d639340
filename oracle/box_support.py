"""Reference for the paper-literal support of Phase 2 (Section 4.4).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Section 4.4 rasterises an accepted Gaussian over every pixel of its in-plane
box instead of testing each pair against the Eq. 12 ellipsoid.  Taken in the
paper's order:

1. Eq. 13: the box b_min/max = m -/+ h of the chi^2 ellipsoid in each probe
   frame (``render.box_eq13``, precision reading; m = probe coordinates of
   the mean).
2. Phase 1: the Gaussian is rejected for the plane if b3_min > 0 or
   b3_max < 0.
3. Phase 2: pixel x (Section 4.1 centres, x1 = (u + 1/2 - W/2) sx,
   x2 = (v + 1/2 - H/2) sy) takes the Gaussian iff b1_min <= x1 <= b1_max
   and b2_min <= x2 <= b2_max, with the Eq. 8 weight sigmoid(a) exp(-d^2/2)
   and no Eq. 12 test.
4. Eq. 5-7 as in ``render``.

Every decision is a comparison of FP64 quantities; another FP64 evaluation
(different operation order) can take the other side only when the two sides
agree to about 1e-15 relative.  Decisions within ``tol`` (relative to the
magnitudes compared) are borderline, and (lo, hi) spans c_hat over every
inclusion choice of the borderline pairs of a pixel.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .render import Params, _chunk, _unpack, box_eq13


def _near(x, lo, hi, band):
    """x within ``band`` of a finite bound lo or hi."""
    with np.errstate(invalid="ignore"):
        a = np.isfinite(lo) & (np.abs(x - lo) <= band)
        b = np.isfinite(hi) & (np.abs(x - hi) <= band)
    return a | b


def render_box_support(g, planes, params: Params | None = None, pix=None, tol: float = 1e-9, max_k: int = 12):
    """Every pixel of every plane (or the ``pix`` [M,3] (plane, u, v)
    samples) -> (c_hat, D, lo, hi, k): the image with the box as the support,
    the denominators, the interval over borderline decisions and their
    number per pixel (k > max_k gives an unbounded interval)."""
    params = params or Params()
    mu, L, c, alpha = _unpack(g, params)
    if pix is None:
        sel = []
        for p in range(planes.p):
            W, H = int(planes.wh[p, 0]), int(planes.wh[p, 1])
            vv, uu = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
            sel.append(np.stack([np.full(W * H, p), uu.ravel(), vv.ravel()], axis=1))
        pix = np.concatenate(sel, axis=0)
    pix = np.asarray(pix, dtype=np.int64)
    M = pix.shape[0]
    out, den = np.empty(M), np.empty(M)
    lo, hi = np.empty(M), np.empty(M)
    kk = np.zeros(M, dtype=np.int64)
    # boxes only for the planes sampled (the same arithmetic per plane)
    used = [int(p) for p in np.unique(pix[:, 0])]
    bmin_u, bmax_u = box_eq13(g, planes.subset(used), params)
    for ui, p in enumerate(used):
        rows = np.nonzero(pix[:, 0] == p)[0]
        R = np.asarray(planes.rot[p], dtype=np.float64).reshape(3, 3)
        o = np.asarray(planes.origin[p], dtype=np.float64)
        W, H = float(planes.wh[p, 0]), float(planes.wh[p, 1])
        sx, sy = (float(s) for s in planes.spacing[p])
        b0, b1 = bmin_u[:, ui], bmax_u[:, ui]
        # Phase 1 (step 2), with its borderline band (chi^2 = inf: unbounded
        # boxes, never borderline)
        acc = (b0[:, 2] <= 0.0) & (b1[:, 2] >= 0.0)
        acc_b = _near(0.0, b0[:, 2], b1[:, 2], tol * (np.abs(b0[:, 2]) + np.abs(b1[:, 2])))
        cand = np.nonzero(acc | acc_b)[0]
        x1 = (pix[rows, 1].astype(np.float64) + 0.5 - W / 2) * sx
        x2 = (pix[rows, 2].astype(np.float64) + 0.5 - H / 2) * sy
        X = o[None, :] + x1[:, None] * R[:, 0][None, :] + x2[:, None] * R[:, 1][None, :]
        lo1, hi1, lo2, hi2 = b0[cand, 0], b1[cand, 0], b0[cand, 1], b1[cand, 1]
        lc, ac, cc = L[cand], alpha[cand], c[cand]
        sure_acc = (acc & ~acc_b)[cand]
        s1 = tol * (np.abs(lo1) + np.abs(hi1) + W * sx)
        s2 = tol * (np.abs(lo2) + np.abs(hi2) + H * sy)
        step = _chunk(max(cand.size, 1))
        for s in range(0, rows.size, step):
            r = rows[s:s + step]
            a1, a2 = x1[s:s + step, None], x2[s:s + step, None]
            in1 = (a1 >= lo1[None, :]) & (a1 <= hi1[None, :])
            in2 = (a2 >= lo2[None, :]) & (a2 <= hi2[None, :])
            e1 = _near(a1, lo1[None, :], hi1[None, :], s1[None, :])
            e2 = _near(a2, lo2[None, :], hi2[None, :], s2[None, :])
            take = acc[cand][None, :] & in1 & in2
            sure = sure_acc[None, :] & in1 & ~e1 & in2 & ~e2
            maybe = (in1 | e1) & (in2 | e2)  # every candidate passes Phase 1 or is borderline there
            delta = X[s:s + step, None, :] - mu[cand][None, :, :]
            y = np.einsum("cnj,njk->cnk", delta, lc)
            d2 = np.sum(y * y, axis=-1)
            wfull = ac[None, :] * np.exp(-0.5 * d2)
            w = np.where(take, wfull, 0.0)
            D = w.sum(axis=1) + params.bg_alpha
            out[r] = (w @ cc + params.bg_alpha * params.bg_color) / D
            den[r] = D
            ws = np.where(sure, wfull, 0.0)
            D0 = ws.sum(axis=1) + params.bg_alpha
            N0 = ws @ cc + params.bg_alpha * params.bg_color
            border = maybe & ~sure
            for i in range(r.size):
                j = np.nonzero(border[i])[0]
                kk[r[i]] = j.size
                if j.size == 0:
                    lo[r[i]] = hi[r[i]] = N0[i] / D0[i]
                elif j.size > max_k:
                    lo[r[i]], hi[r[i]] = -math.inf, math.inf
                else:
                    vals = []
                    for mask in itertools.product((0.0, 1.0), repeat=j.size):
                        wj = wfull[i, j] * np.asarray(mask)
                        vals.append((N0[i] + wj @ cc[j]) / (D0[i] + wj.sum()))
                    lo[r[i]], hi[r[i]] = min(vals), max(vals)
    return out, den, lo, hi, kk
