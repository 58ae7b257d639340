"""Reference for the densify / prune pass between training steps.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Section 4.2 draws a new point from a Gaussian through its triangular factor,
y = mu + L^-T z (``sample_gaussian``).  The clone / split / prune rule is only
referred to by the paper (3D Gaussian splatting); the library's stated
choice, followed here step by step:

* size^2 = trace(Sigma) = the sum of squares of the entries of L^-1 (L lower
  triangular, so L^-1 is written out entry by entry);
* prune if sigmoid(a) < min_opacity (compared as a < logit(min_opacity)) or,
  with max_size > 0, size^2 > max_size^2;
* else if cnt > 0 and acc >= grad_thresh * cnt: split if size^2 >
  split_size^2, otherwise clone;
* else keep.

These are integer outcomes of floating-point comparisons, so they are taken
in float32 with every operation in the library's order (numpy rounds each
float32 operation once, as the device does with contraction off).  The
outputs are float64: kept and cloned Gaussians are copies; a split gives two
children with means mu + L^-T z[i][c] and factor phi L (every standard
deviation divided by phi), intensity and opacity copied.  Outputs are in
Gaussian order, a Gaussian's children together.
"""
from __future__ import annotations

import math

import numpy as np

from .render import sample_gaussian

PRUNE, KEEP, CLONE, SPLIT = 0, 1, 2, 3


def size2_f32(lraw, beta: float) -> np.ndarray:
    """float32 trace of the covariance from the raw factor (Eq. 11)."""
    f = np.float32
    r = np.asarray(lraw, dtype=f).reshape(-1, 6)
    b = f(beta)
    l11 = r[:, 0] * r[:, 0] + b
    l21, l31 = r[:, 1], r[:, 2]
    l22 = r[:, 3] * r[:, 3] + b
    l32 = r[:, 4]
    l33 = r[:, 5] * r[:, 5] + b
    one = f(1.0)
    i11, i22, i33 = one / l11, one / l22, one / l33
    i21 = -l21 * i11 * i22
    i32 = -l32 * i22 * i33
    i31 = (l21 * l32 - l22 * l31) * i11 * i22 * i33
    return i11 * i11 + i21 * i21 + i22 * i22 + i31 * i31 + i32 * i32 + i33 * i33


def decisions(lraw, opacity, acc, cnt, beta=1e-4, min_opacity=0.005, grad_thresh=2e-4, split_size=1.0,
              max_size=0.0) -> np.ndarray:
    """PRUNE / KEEP / CLONE / SPLIT per Gaussian."""
    f = np.float32
    s2 = size2_f32(lraw, beta)
    a = np.asarray(opacity, dtype=f)
    acc = np.asarray(acc, dtype=f)
    cnt = np.asarray(cnt, dtype=np.int32)
    t = float(min_opacity)
    amin = f(-math.inf) if t <= 0.0 else (f(math.inf) if t >= 1.0 else f(math.log(t / (1.0 - t))))
    split2 = f(split_size) * f(split_size)
    max2 = f(max_size) * f(max_size)
    d = np.full(a.shape[0], KEEP, dtype=np.int64)
    grow = (cnt > 0) & (acc >= f(grad_thresh) * cnt.astype(f))
    d[grow] = np.where(s2[grow] > split2, SPLIT, CLONE)
    prune = ~(a >= amin)
    if max2 > 0:
        prune |= ~(s2 <= max2)
    d[prune] = PRUNE
    return d


def scaled_lraw(lraw, beta: float, phi: float) -> np.ndarray:
    """Raw factor of phi L: diagonal l'^2 + beta = phi (l^2 + beta), off-diagonal phi l."""
    r = np.asarray(lraw, dtype=np.float64).reshape(-1, 6)
    out = phi * r
    for k in (0, 3, 5):
        out[:, k] = np.sqrt(phi * (r[:, k] ** 2 + beta) - beta)
    return out


def densify(g, acc, cnt, z, beta=1e-4, min_opacity=0.005, grad_thresh=2e-4, split_size=1.0, max_size=0.0,
            split_factor=1.6):
    """(means, lraw, intensity, opacity, source index, decisions): the outputs
    in Gaussian order (float64) and the input Gaussian each came from."""
    d = decisions(g.lraw, g.opacity, acc, cnt, beta, min_opacity, grad_thresh, split_size, max_size)
    z = np.asarray(z, dtype=np.float64).reshape(-1, 2, 3)
    means, lraw, inten, opac, src = [], [], [], [], []
    mu = np.asarray(g.means, dtype=np.float64)
    raw = np.asarray(g.lraw, dtype=np.float64)
    for i in range(mu.shape[0]):
        if d[i] == PRUNE:
            continue
        n_out = 1 if d[i] == KEEP else 2
        for c in range(n_out):
            if d[i] == SPLIT:
                means.append(sample_gaussian(mu[i:i + 1], raw[i:i + 1], z[i, c:c + 1], beta)[0])
                lraw.append(scaled_lraw(raw[i:i + 1], beta, split_factor)[0])
            else:
                means.append(mu[i].copy())
                lraw.append(raw[i].copy())
            inten.append(float(g.intensity[i]))
            opac.append(float(g.opacity[i]))
            src.append(i)
    m = len(src)
    return (np.asarray(means).reshape(m, 3), np.asarray(lraw).reshape(m, 6), np.asarray(inten),
            np.asarray(opac), np.asarray(src, dtype=np.int64), d)
