"""Reference image-quality scores for reconstructions (Section 5.2 evaluates
with SSIM and PSNR).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

SSIM follows Wang et al. (2004) with its usual constants: the local
statistics of a window position are Gaussian-weighted moments (an 11 x 11
window, standard deviation 1.5 pixels, weights normalised to sum to one;
population moments, sigma_x^2 = sum w (x - mu_x)^2), and

    SSIM = (2 mu_x mu_y + C1) (2 sigma_xy + C2)
           / ((mu_x^2 + mu_y^2 + C1) (sigma_x^2 + sigma_y^2 + C2)),
    C1 = (0.01 L)^2,  C2 = (0.03 L)^2,  L = the data range,

averaged over the window positions that lie wholly inside the image (the
5-pixel border has none; a plane narrower than 11 pixels has no position
and scores NaN).  PSNR = 10 log10(L^2 / MSE), MSE over every pixel.
Everything is float64; the moments are centred (two passes), not
E[x^2] - mu^2.
"""
from __future__ import annotations

import math

import numpy as np

WIN = 11
SIGMA = 1.5
K1, K2 = 0.01, 0.03


def window(size: int = WIN, sigma: float = SIGMA) -> np.ndarray:
    """[size, size] Gaussian weights summing to one."""
    k = np.arange(size, dtype=np.float64) - (size - 1) / 2
    g = np.exp(-(k * k) / (2 * sigma * sigma))
    w = np.outer(g, g)
    return w / w.sum()


def ssim_map(x, y, data_range: float = 1.0) -> np.ndarray:
    """SSIM of every window position inside the image: [H - 10, W - 10]."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape[0] < WIN or x.shape[1] < WIN:
        return np.empty((0, 0))
    w = window()
    wx = np.lib.stride_tricks.sliding_window_view(x, (WIN, WIN))
    wy = np.lib.stride_tricks.sliding_window_view(y, (WIN, WIN))
    mx = np.einsum("ijab,ab->ij", wx, w)
    my = np.einsum("ijab,ab->ij", wy, w)
    dx = wx - mx[:, :, None, None]
    dy = wy - my[:, :, None, None]
    vx = np.einsum("ijab,ab->ij", dx * dx, w)
    vy = np.einsum("ijab,ab->ij", dy * dy, w)
    cxy = np.einsum("ijab,ab->ij", dx * dy, w)
    c1 = (K1 * data_range) ** 2
    c2 = (K2 * data_range) ** 2
    return ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))


def ssim(x, y, data_range: float = 1.0) -> float:
    m = ssim_map(x, y, data_range)
    return float(m.mean()) if m.size else math.nan


def mse(x, y) -> float:
    d = np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return float(np.mean(d * d))


def psnr(mse_value: float, data_range: float = 1.0) -> float:
    return 10.0 * math.log10(data_range * data_range / mse_value) if mse_value > 0 else math.inf


def quality(img, ref, wh, data_range: float = 1.0):
    """Per plane of packed row-major images (plane offsets = prefix of W H):
    (ssim [P], mse [P])."""
    img = np.asarray(img).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    out_s, out_m = [], []
    off = 0
    for W, H in np.asarray(wh, dtype=np.int64).reshape(-1, 2):
        n = int(W * H)
        a = img[off:off + n].reshape(int(H), int(W))
        b = ref[off:off + n].reshape(int(H), int(W))
        out_s.append(ssim(a, b, data_range))
        out_m.append(mse(a, b))
        off += n
    return np.asarray(out_s), np.asarray(out_m)
