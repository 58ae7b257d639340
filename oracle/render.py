"""FP64 brute-force reference of UltraGauss's probe-plane image formation.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

What is computed, in the paper's order (UltraGauss, Section 4.1-4.3):

1. Eq. 11 (Section 4.2): the precision factor L from the raw parameters,
   diagonal entries squared plus beta; the entry printed at (3,2) is read as
   an independent L32 (the printed repeat of L12 would leave five degrees of
   freedom).  Sigma^-1 = L L^T.
2. Section 4.1: a pixel x is lifted to x|0 = [x1, x2, 0] in the probe frame.
   Eq. 9 moves the Gaussian into that frame with the rigid world->probe map
   W; the squared Mahalanobis distance of Eq. 8 is invariant under a rigid
   map, so it is evaluated here at the pixel's world point X as
   d^2 = || L^T (X - mu) ||^2.
3. Eq. 12 (Section 4.3): a pair contributes only if d^2 <= chi^2 (ties
   included).
4. Eq. 8: alpha_i(x) = sigmoid(a_i) exp(-d^2 / 2).
5. Eq. 5-7: c(x) = (sum_i alpha_i(x) c_i + a_BG c_BG) / (sum_i alpha_i(x) + a_BG).

Nothing is culled, boxed or tiled: every Gaussian meets every point.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

# Section 4.3, Eq. 12: chi^2 with 3 degrees of freedom at p = 95%, as printed.
CHI2_PAPER = 7.815


@dataclasses.dataclass
class Params:
    beta: float = 1e-4       # Eq. 11 diagonal shift (value not given in the paper)
    chi2: float = CHI2_PAPER  # Eq. 12 bound on the squared distance
    bg_alpha: float = 1e-2   # Eq. 5 background coefficient (value not given)
    bg_color: float = 0.0    # Eq. 6 background colour (value not given)


# ------------------------------------------------------------------ params
def sigmoid(a):
    """Opacity activation, Section 4.5: alpha = 1 / (1 + exp(-a))."""
    a = np.asarray(a, dtype=np.float64)
    return 1.0 / (1.0 + np.exp(-a))


def activate_l(lraw, beta: float) -> np.ndarray:
    """Eq. 11: raw (l11, l21, l31, l22, l32, l33) -> lower-triangular L [N,3,3]."""
    r = np.asarray(lraw, dtype=np.float64).reshape(-1, 6)
    L = np.zeros((r.shape[0], 3, 3))
    L[:, 0, 0] = r[:, 0] ** 2 + beta
    L[:, 1, 0] = r[:, 1]
    L[:, 2, 0] = r[:, 2]
    L[:, 1, 1] = r[:, 3] ** 2 + beta
    L[:, 2, 1] = r[:, 4]
    L[:, 2, 2] = r[:, 5] ** 2 + beta
    return L


def _forward_subst(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve L X = B for lower-triangular L [N,3,3], B [N,3,k] (forward substitution)."""
    X = np.zeros_like(B, dtype=np.float64)
    for i in range(3):
        acc = B[:, i, :].copy()
        for j in range(i):
            acc -= L[:, i, j, None] * X[:, j, :]
        X[:, i, :] = acc / L[:, i, i, None]
    return X


def covariance(lraw, beta: float) -> np.ndarray:
    """Section 4.2: Sigma = (L^-1)^T L^-1, with L^-1 from forward substitution."""
    L = activate_l(lraw, beta)
    Linv = _forward_subst(L, np.broadcast_to(np.eye(3), L.shape).copy())
    return np.transpose(Linv, (0, 2, 1)) @ Linv


def sample_gaussian(means, lraw, z, beta: float) -> np.ndarray:
    """Section 4.2 sampling: y = mu + L^-T z for standard-normal z [N,3]."""
    L = activate_l(lraw, beta)
    LT = np.transpose(L, (0, 2, 1))
    # back substitution with the upper-triangular L^T
    z = np.asarray(z, dtype=np.float64)
    y = np.zeros_like(z)
    for i in (2, 1, 0):
        acc = z[:, i].copy()
        for j in range(i + 1, 3):
            acc -= LT[:, i, j] * y[:, j]
        y[:, i] = acc / LT[:, i, i]
    return np.asarray(means, dtype=np.float64) + y


# ------------------------------------------------------------------ planes
def _frame(planes, p):
    R = np.asarray(planes.rot[p], dtype=np.float64).reshape(3, 3)
    return R[:, 0], R[:, 1], R[:, 2], np.asarray(planes.origin[p], dtype=np.float64)


def plane_points(planes, pix=None) -> np.ndarray:
    """World points of pixel centres (Section 4.1 lifting, inverse of W).

    Pixel (u, v) of a W x H plane sits at in-plane coordinates
    x1 = (u + 1/2 - W/2) sx, x2 = (v + 1/2 - H/2) sy, i.e. world point
    X = o + x1 e1 + x2 e2.  ``pix`` = optional [M,3] (plane, u, v) samples;
    otherwise every pixel of every plane, packed plane-major, row-major.
    """
    if pix is None:
        out = []
        for p in range(planes.p):
            W, H = int(planes.wh[p, 0]), int(planes.wh[p, 1])
            vv, uu = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
            out.append(_points_on(planes, p, uu.ravel(), vv.ravel()))
        return np.concatenate(out, axis=0)
    pix = np.asarray(pix, dtype=np.int64)
    out = np.empty((pix.shape[0], 3))
    for p in np.unique(pix[:, 0]):
        sel = pix[:, 0] == p
        out[sel] = _points_on(planes, int(p), pix[sel, 1], pix[sel, 2])
    return out


def _points_on(planes, p, u, v):
    e1, e2, _, o = _frame(planes, p)
    W, H = float(planes.wh[p, 0]), float(planes.wh[p, 1])
    sx, sy = (float(s) for s in planes.spacing[p])
    x1 = (np.asarray(u, dtype=np.float64) + 0.5 - W / 2) * sx
    x2 = (np.asarray(v, dtype=np.float64) + 0.5 - H / 2) * sy
    return o[None, :] + x1[:, None] * e1[None, :] + x2[:, None] * e2[None, :]


# ------------------------------------------------------------------ core
def _unpack(g, params):
    mu = np.asarray(g.means, dtype=np.float64)
    L = activate_l(g.lraw, params.beta)
    c = np.asarray(g.intensity, dtype=np.float64)
    alpha = sigmoid(g.opacity)
    return mu, L, c, alpha


def _chunk(n: int, budget: float = 1.2e7) -> int:
    return max(1, int(budget // max(3 * n, 1)))


def d2_points(g, X, params: Params | None = None) -> np.ndarray:
    """Eq. 8 squared Mahalanobis distances [M, N] at world points X [M,3]."""
    params = params or Params()
    mu, L, _, _ = _unpack(g, params)
    X = np.asarray(X, dtype=np.float64)
    delta = X[:, None, :] - mu[None, :, :]
    y = np.einsum("cnj,njk->cnk", delta, L)
    return np.sum(y * y, axis=-1)


def render_points(g, X, params: Params | None = None):
    """Eq. 5-8 at world points X [M,3] -> (c_hat [M], alpha_hat [M])."""
    params = params or Params()
    mu, L, c, alpha = _unpack(g, params)
    X = np.asarray(X, dtype=np.float64)
    out = np.empty(X.shape[0])
    den = np.empty(X.shape[0])
    step = _chunk(mu.shape[0])
    for s in range(0, X.shape[0], step):
        Xc = X[s:s + step]
        delta = Xc[:, None, :] - mu[None, :, :]
        y = np.einsum("cnj,njk->cnk", delta, L)
        d2 = np.sum(y * y, axis=-1)
        w = np.where(d2 <= params.chi2, alpha[None, :] * np.exp(-0.5 * d2), 0.0)
        D = w.sum(axis=1) + params.bg_alpha
        num = w @ c + params.bg_alpha * params.bg_color
        out[s:s + step] = num / D
        den[s:s + step] = D
    return out, den


def render(g, planes, params: Params | None = None, pix=None):
    """Every pixel of every plane (or the ``pix`` samples) -> (image, alpha_hat)."""
    return render_points(g, plane_points(planes, pix), params)


def grad_points(g, X, dout, params: Params | None = None):
    """Exact derivative of sum_x dout(x) c_hat(x) w.r.t. the raw parameters.

    The inclusion set {d^2 <= chi^2} is held fixed (the map is piecewise
    smooth).  Chain rule of Eq. 5-8 and Eq. 11:
      dc_hat/dc_i = w_i / D,  dc_hat/dw_i = (c_i - c_hat) / D,
      dw/da = w (1 - alpha),  dw/d(d^2) = -w / 2,
      with y = L^T (X - mu): d(d^2)/dmu = -2 L y, d(d^2)/dL = 2 (X - mu) y^T,
      dL_kk/dl_kk = 2 l_kk.
    Returns dict(means [N,3], lraw [N,6], intensity [N], opacity [N]).
    """
    params = params or Params()
    mu, L, c, alpha = _unpack(g, params)
    X = np.asarray(X, dtype=np.float64)
    dout = np.asarray(dout, dtype=np.float64)
    n = mu.shape[0]
    dmu = np.zeros((n, 3))
    dL = np.zeros((n, 3, 3))
    dc = np.zeros(n)
    da = np.zeros(n)
    step = _chunk(n, 6e6)
    nz = np.nonzero(dout)[0]
    for s in range(0, nz.size, step):
        idx = nz[s:s + step]
        Xc = X[idx]
        gbar = dout[idx]
        delta = Xc[:, None, :] - mu[None, :, :]
        y = np.einsum("cnj,njk->cnk", delta, L)
        d2 = np.sum(y * y, axis=-1)
        w = np.where(d2 <= params.chi2, alpha[None, :] * np.exp(-0.5 * d2), 0.0)
        D = w.sum(axis=1) + params.bg_alpha
        chat = (w @ c + params.bg_alpha * params.bg_color) / D
        gam = gbar / D
        dc += gam @ w
        dw = gam[:, None] * (c[None, :] - chat[:, None])
        da += np.sum(dw * w, axis=0) * (1.0 - alpha)
        dd2 = -0.5 * w * dw
        Sy = np.einsum("cn,cnk->nk", dd2, y)
        dmu += -2.0 * np.einsum("njk,nk->nj", L, Sy)
        dL += 2.0 * np.einsum("cn,cnj,cnk->njk", dd2, delta, y)
    r = np.asarray(g.lraw, dtype=np.float64)
    dlraw = np.stack([dL[:, 0, 0] * 2 * r[:, 0], dL[:, 1, 0], dL[:, 2, 0],
                      dL[:, 1, 1] * 2 * r[:, 3], dL[:, 2, 1],
                      dL[:, 2, 2] * 2 * r[:, 5]], axis=1)
    return {"means": dmu, "lraw": dlraw, "intensity": dc, "opacity": da}


def grad(g, planes, dimage, params: Params | None = None, pix=None):
    """``grad_points`` over every pixel of every plane (or the ``pix`` samples)."""
    return grad_points(g, plane_points(planes, pix), dimage, params)


# ------------------------------------------------------------------ cut-off ambiguity
def ambiguity_points(g, X, params: Params | None = None, tau: float = 2e-4,
                     max_k: int = 12):
    """Interval of c_hat over every inclusion choice for borderline pairs.

    Eq. 12 decides each pair by d^2 <= chi^2; an FP32 evaluation can take the
    other side when |d^2 - chi^2| is within its rounding.  Pairs with
    |d^2 - chi^2| <= tau * max(1, chi^2) are borderline; the interval spans
    c_hat over all 2^k subsets of them.  Returns (lo, hi, k) per point;
    k > max_k gives lo = -inf, hi = +inf.
    """
    params = params or Params()
    mu, L, c, alpha = _unpack(g, params)
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    lo = np.empty(M)
    hi = np.empty(M)
    kk = np.zeros(M, dtype=np.int64)
    band = tau * max(1.0, params.chi2) if math.isfinite(params.chi2) else 0.0
    step = _chunk(mu.shape[0])
    for s in range(0, M, step):
        Xc = X[s:s + step]
        delta = Xc[:, None, :] - mu[None, :, :]
        y = np.einsum("cnj,njk->cnk", delta, L)
        d2 = np.sum(y * y, axis=-1)
        wfull = alpha[None, :] * np.exp(-0.5 * d2)
        border = np.abs(d2 - params.chi2) <= band
        sure = (d2 <= params.chi2) & ~border
        w = np.where(sure, wfull, 0.0)
        D0 = w.sum(axis=1) + params.bg_alpha
        N0 = w @ c + params.bg_alpha * params.bg_color
        for i in range(Xc.shape[0]):
            j = np.nonzero(border[i])[0]
            kk[s + i] = j.size
            if j.size == 0:
                lo[s + i] = hi[s + i] = N0[i] / D0[i]
            elif j.size > max_k:
                lo[s + i], hi[s + i] = -np.inf, np.inf
            else:
                vals = []
                for mask in itertools.product((0.0, 1.0), repeat=j.size):
                    m = np.asarray(mask)
                    wj = wfull[i, j] * m
                    vals.append((N0[i] + wj @ c[j]) / (D0[i] + wj.sum()))
                lo[s + i], hi[s + i] = min(vals), max(vals)
    return lo, hi, kk


# ------------------------------------------------------------------ boundaries
def box_eq13(g, planes, params: Params | None = None, matrix: str = "precision"):
    """Eq. 13 axis-aligned box in each probe frame: b = mu3D -/+ sqrt(lambda v).

    lambda = chi^2 / det(Q) and v = the diagonal cofactors of Q.  As printed,
    Q is Sigma3D; the box of the Eq. 12 ellipsoid comes out only when Q is the
    probe-frame precision (Sigma3D)^-1 = R^T L L^T R, whose cofactor over
    determinant is the covariance diagonal.  ``matrix`` picks the reading
    ("precision" is the one used for rasterization; "covariance" is the
    literal text, kept to show it fails the brute-force check).
    Returns (bmin, bmax) [N, P, 3] in probe coordinates.
    """
    params = params or Params()
    mu, L, _, _ = _unpack(g, params)
    prec = L @ np.transpose(L, (0, 2, 1))
    n, P = mu.shape[0], planes.p
    bmin = np.empty((n, P, 3))
    bmax = np.empty((n, P, 3))
    for p in range(P):
        R = np.asarray(planes.rot[p], dtype=np.float64).reshape(3, 3)
        o = np.asarray(planes.origin[p], dtype=np.float64)
        m = np.linalg.solve(R, (mu - o).T).T   # probe coordinates: mu - o = R m
        Pp = np.transpose(R) @ prec @ R         # probe-frame precision
        Q = Pp if matrix == "precision" else np.linalg.inv(Pp)
        v = np.stack([Q[:, 1, 1] * Q[:, 2, 2] - Q[:, 1, 2] ** 2,
                      Q[:, 0, 0] * Q[:, 2, 2] - Q[:, 0, 2] ** 2,
                      Q[:, 0, 0] * Q[:, 1, 1] - Q[:, 0, 1] ** 2], axis=1)
        lam = params.chi2 / np.linalg.det(Q)
        h = np.sqrt(lam[:, None] * v)
        bmin[:, p] = m - h
        bmax[:, p] = m + h
    return bmin, bmax


def inplane_conic(g, planes, params: Params | None = None):
    """Restriction of the Eq. 8 quadratic form to the probe plane x3 = 0.

    Completing the square in the probe frame with P = R^T L L^T R,
    A = P[:2,:2], b = P[:2,2], m = R^-1 (mu - o) (= R^T (mu - o) for an
    exactly orthonormal frame; the inverse keeps float32-rounded frames exact):
      d^2(x) = (x - c)^T A (x - c) + r^2,
      c = m[:2] + m3 A^-1 b,   r^2 = m3^2 (P33 - b^T A^-1 b)  (Schur complement).
    Returns (centre [N,P,2] in-plane coords, A [N,P,2,2], r2 [N,P]).
    """
    params = params or Params()
    mu, L, _, _ = _unpack(g, params)
    prec = L @ np.transpose(L, (0, 2, 1))
    n, P = mu.shape[0], planes.p
    cen = np.empty((n, P, 2))
    A = np.empty((n, P, 2, 2))
    r2 = np.empty((n, P))
    for p in range(P):
        R = np.asarray(planes.rot[p], dtype=np.float64).reshape(3, 3)
        o = np.asarray(planes.origin[p], dtype=np.float64)
        m = np.linalg.solve(R, (mu - o).T).T
        Pp = np.transpose(R) @ prec @ R
        Ap = Pp[:, :2, :2]
        b = Pp[:, :2, 2]
        Ainv_b = np.linalg.solve(Ap, b[..., None])[..., 0]
        cen[:, p] = m[:, :2] + m[:, 2:3] * Ainv_b
        A[:, p] = Ap
        r2[:, p] = m[:, 2] ** 2 * (Pp[:, 2, 2] - np.sum(b * Ainv_b, axis=1))
    return cen, A, r2
