"""Reference for the densify / prune pass between training steps.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Section 4.2 draws a new point from a Gaussian through its triangular factor,
y = mu + L^-T z (``sample_gaussian``).  The clone / split / prune rule is only
referred to by the paper (3D Gaussian splatting); the library's stated
choice, evaluated here in float64:

* size^2 = trace(Sigma), Sigma from the Section 4.2 forward substitution
  (``covariance``);
* prune if sigmoid(a) < min_opacity or, with max_size > 0,
  size^2 > max_size^2;
* else if cnt > 0 and the mean accumulated gradient acc / cnt reaches
  grad_thresh (acc >= grad_thresh * cnt): split if size^2 > split_size^2,
  otherwise clone;
* else keep.

Each decision is an integer outcome of a comparison of real numbers, which a
float32 evaluation may take the other way when the two sides are within its
rounding.  A comparison whose sides differ by at most BAND (relative) is
borderline, and ``decisions`` also returns every outcome the rule gives
under any choice of the borderline comparisons.  Outputs are float64: kept
and cloned Gaussians are copies; a split gives two children with means
mu + L^-T z[i][c] and factor phi L (every standard deviation divided by
phi), intensity and opacity copied.  Outputs are in Gaussian order, a
Gaussian's children together.
"""
from __future__ import annotations

import itertools

import numpy as np

from .render import covariance, sample_gaussian, sigmoid

PRUNE, KEEP, CLONE, SPLIT = 0, 1, 2, 3
# Relative half-width of the borderline band of a comparison (a float32
# evaluation of either side is within a few 1e-7 of it).
BAND = 1e-5


def size2(lraw, beta: float) -> np.ndarray:
    """trace(Sigma) of each Gaussian (float64)."""
    return np.trace(covariance(lraw, beta), axis1=1, axis2=2)


def _rule(prune_op, prune_max, grow, split):
    return np.where(prune_op | prune_max, PRUNE, np.where(grow, np.where(split, SPLIT, CLONE), KEEP))


def decisions(lraw, opacity, acc, cnt, beta=1e-4, min_opacity=0.005, grad_thresh=2e-4, split_size=1.0,
              max_size=0.0):
    """(d, possible): d = PRUNE / KEEP / CLONE / SPLIT per Gaussian with every
    comparison taken exactly in float64; possible [N, 4] marks every outcome
    that some choice of the borderline comparisons gives (d included)."""
    s2 = size2(lraw, beta)
    alpha = sigmoid(np.asarray(opacity, dtype=np.float64))
    acc = np.asarray(acc, dtype=np.float64)
    cnt = np.asarray(cnt, dtype=np.int64)
    t_op = float(min_opacity)
    split2 = float(split_size) ** 2
    max2 = float(max_size) ** 2
    gc = float(grad_thresh) * cnt.astype(np.float64)
    # (outcome, borderline) of the four comparisons
    comps = [
        (alpha < t_op, np.abs(alpha - t_op) <= BAND * abs(t_op)),
        ((s2 > max2) if max2 > 0 else np.zeros(s2.shape, bool),
         (np.abs(s2 - max2) <= BAND * max2) if max2 > 0 else np.zeros(s2.shape, bool)),
        ((cnt > 0) & (acc >= gc), (cnt > 0) & (np.abs(acc - gc) <= BAND * np.abs(gc))),
        (s2 > split2, np.abs(s2 - split2) <= BAND * split2),
    ]
    d = _rule(*(c[0] for c in comps))
    possible = np.zeros((d.shape[0], 4), dtype=bool)
    idx = np.arange(d.shape[0])
    for flips in itertools.product((False, True), repeat=4):
        alt = [np.where(b & f, ~o, o) for (o, b), f in zip(comps, flips)]
        possible[idx, _rule(*alt)] = True
    return d, possible


def children(mu, lraw, z2, beta: float, phi: float):
    """The two split children of one Gaussian: (means [2,3], lraw [2,6])."""
    mu = np.asarray(mu, dtype=np.float64).reshape(1, 3)
    raw = np.asarray(lraw, dtype=np.float64).reshape(1, 6)
    z2 = np.asarray(z2, dtype=np.float64).reshape(2, 3)
    means = np.stack([sample_gaussian(mu, raw, z2[c:c + 1], beta)[0] for c in range(2)])
    return means, np.repeat(scaled_lraw(raw, beta, phi), 2, axis=0)


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
    in Gaussian order (float64) and the input Gaussian each came from, for
    the float64 decisions."""
    d, _ = decisions(g.lraw, g.opacity, acc, cnt, beta, min_opacity, grad_thresh, split_size, max_size)
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
                cm, cl = children(mu[i], raw[i], z[i], beta, split_factor)
                means.append(cm[c])
                lraw.append(cl[c])
            else:
                means.append(mu[i].copy())
                lraw.append(raw[i].copy())
            inten.append(float(g.intensity[i]))
            opac.append(float(g.opacity[i]))
            src.append(i)
    m = len(src)
    return (np.asarray(means).reshape(m, 3), np.asarray(lraw).reshape(m, 6), np.asarray(inten),
            np.asarray(opac), np.asarray(src, dtype=np.int64), d)
