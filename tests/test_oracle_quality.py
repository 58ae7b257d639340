"""Pins of the SSIM / PSNR reference against closed forms.  None of these
tests uses the HIP path.

The checkerboard pin fixes every part of the SSIM definition at once: for
x = m + a s and y = m + b s with s(u, v) = (-1)^(u+v), a window centred on
(u, v) sees mu_s = (-1)^(u+v) G^2 with G = sum_k g_k (-1)^(k-5) over the
normalised 1D Gaussian taps g (scipy's normal density here), and population
moments sigma_s^2 = 1 - G^4, so each position has a closed-form SSIM.  A
wrong window width or normalisation, sample instead of population moments,
a wrong constant or a wrong crop all change the mean."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import quality as Q


def _taps():
    k = np.arange(11) - 5
    g = scipy.stats.norm.pdf(k, scale=1.5)
    return g / g.sum()


def test_window_is_the_normalised_gaussian():
    g = _taps()
    np.testing.assert_allclose(Q.window(), np.outer(g, g), rtol=1e-14, atol=1e-17)
    assert Q.window().sum() == pytest.approx(1.0, abs=1e-15)


def test_identical_images_score_one():
    rng = np.random.default_rng(1)
    x = rng.random((23, 31))
    assert Q.ssim(x, x) == pytest.approx(1.0, abs=1e-14)
    assert Q.mse(x, x) == 0.0 and Q.psnr(0.0) == math.inf


@pytest.mark.parametrize("a,b,L", [(0.3, 0.7, 1.0), (0.0, 0.5, 1.0), (0.9, 0.2, 2.0)])
def test_constant_images(a, b, L):
    """No variance: the contrast-structure term is C2 / C2 = 1."""
    x = np.full((15, 12), a)
    y = np.full((15, 12), b)
    c1 = (0.01 * L) ** 2
    assert Q.ssim(x, y, L) == pytest.approx((2 * a * b + c1) / (a * a + b * b + c1), rel=1e-12)
    assert Q.ssim_map(x, y, L).shape == (5, 2)


@pytest.mark.parametrize("m,a,b,L,W,H", [(0.5, 0.2, 0.1, 1.0, 20, 17), (0.4, 0.3, -0.25, 1.0, 13, 11),
                                         (1.0, 0.5, 0.45, 2.0, 30, 12)])
def test_checkerboard_closed_form(m, a, b, L, W, H):
    g = _taps()
    G = float(np.sum(g * (-1.0) ** np.arange(11)))   # tap 5 (the centre) has sign +1
    v, u = np.mgrid[0:H, 0:W]
    s = (-1.0) ** (u + v)
    x, y = m + a * s, m + b * s
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    var_s = 1.0 - G ** 4
    expect = []
    for vv in range(5, H - 5):
        for uu in range(5, W - 5):
            ms = (-1.0) ** (uu + vv) * G * G
            mx, my = m + a * ms, m + b * ms
            expect.append((2 * mx * my + c1) * (2 * a * b * var_s + c2)
                          / ((mx * mx + my * my + c1) * ((a * a + b * b) * var_s + c2)))
    assert Q.ssim(x, y, L) == pytest.approx(float(np.mean(expect)), rel=1e-12)
    # the scores are symmetric and bounded by one
    assert Q.ssim(y, x, L) == pytest.approx(Q.ssim(x, y, L), rel=1e-14)
    assert Q.ssim(x, y, L) <= 1.0


def test_psnr_of_a_shift():
    rng = np.random.default_rng(2)
    x = rng.random((16, 16))
    d = 0.05
    e = Q.mse(x, x + d)
    assert e == pytest.approx(d * d, rel=1e-12)
    assert Q.psnr(e) == pytest.approx(-20 * math.log10(d), rel=1e-12)
    assert Q.psnr(e, 2.0) == pytest.approx(20 * math.log10(2.0 / d), rel=1e-12)


def test_packed_planes_and_small_planes():
    rng = np.random.default_rng(3)
    wh = np.array([[20, 13], [8, 30], [11, 11]])
    img = rng.random(int(np.sum(wh[:, 0] * wh[:, 1])))
    ref = img + 0.1 * rng.standard_normal(img.size)
    s, m = Q.quality(img, ref, wh)
    off = 0
    for p, (W, H) in enumerate(wh):
        a = img[off:off + W * H].reshape(H, W)
        b = ref[off:off + W * H].reshape(H, W)
        assert m[p] == pytest.approx(np.mean((a - b) ** 2), rel=1e-14)
        off += W * H
    assert math.isnan(s[1])  # 8 pixels wide: no window fits
    assert Q.ssim_map(img[-121:].reshape(11, 11), ref[-121:].reshape(11, 11)).shape == (1, 1)
    assert np.isfinite(s[0]) and np.isfinite(s[2])
