"""Pins of the box-support reference (Section 4.4 Phase 2 with the Eq. 13 box
as the support) against closed forms, a plain loop and the pinned
ellipsoid-support reference.  None of these tests uses the HIP path."""
import math

import numpy as np

import oracle
from oracle import Params
from oracle.box_support import render_box_support
from paper_2505_05643_amd import synth


def _one_gaussian(mu, scales, rot=None, c=1.0, a=1.0, beta=1e-4):
    rot = np.eye(3) if rot is None else np.asarray(rot, dtype=np.float64)
    lraw = synth.scales_rots_to_lraw(np.asarray([scales], dtype=np.float64), rot[None], beta)
    return synth.Gaussians(np.asarray([mu], dtype=np.float64), lraw, np.asarray([c], dtype=np.float64),
                           np.asarray([a], dtype=np.float64))


def _plane(frame, origin, wh, spacing):
    return synth.pack_planes([frame], [origin], [spacing], [wh])


def test_axis_aligned_box_closed_form():
    """Axis-aligned Gaussian, axial plane at offset t: the box half-widths are
    sqrt(chi^2) s_k, every pixel centre inside takes the full textbook weight
    (corners outside the ellipse included), and Phase 1 keeps the Gaussian
    iff |t| <= sqrt(chi^2) s_3."""
    s = np.array([1.1, 0.7, 0.9])
    prm = Params(bg_alpha=0.02)
    pl = _plane(np.eye(3), (0, 0, 0), (24, 20), (0.4, 0.3))
    X = oracle.plane_points(pl)
    for t, kept in ((0.4, True), (-2.3, True), (2.6, False), (-2.6, False)):
        mu = np.array([0.3, -0.2, t])
        g = _one_gaussian(mu, s, c=0.8, a=0.0)
        img, D, lo, hi, k = render_box_support(g, pl, prm)
        assert np.all(k == 0)
        np.testing.assert_array_equal(lo, img)
        np.testing.assert_array_equal(hi, img)
        r = math.sqrt(prm.chi2)
        inbox = (np.abs(X[:, 0] - mu[0]) <= r * s[0]) & (np.abs(X[:, 1] - mu[1]) <= r * s[1]) & kept
        q = ((X[:, 0] - mu[0]) / s[0]) ** 2 + ((X[:, 1] - mu[1]) / s[1]) ** 2 + (t / s[2]) ** 2
        w = np.where(inbox, 0.5 * np.exp(-0.5 * q), 0.0)
        np.testing.assert_allclose(img, 0.8 * w / (w + 0.02), rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(D, w + 0.02, rtol=1e-12)
        if kept:  # the box support reaches pixels the Eq. 12 ellipsoid excludes
            assert np.any(inbox & (q > prm.chi2))
            ell, _ = oracle.render(g, pl, prm)
            assert np.any((img > 0) & (ell == 0))


def test_plain_loop_tiny_scene():
    """A plain loop over planes, Gaussians and pixels, with the probe-frame
    covariance from an explicit inverse and the box tested in world units."""
    g = synth.make_gaussians(12, 61, (0, 0, 0), (1, 1, 1), (0.08, 0.3), aniso_max=6.0, opacity="random")
    pl = synth.random_planes(2, 62, (9, 7), 1 / 8, 0.35, 0.65)
    prm = Params(bg_alpha=0.05, bg_color=0.1)
    img, D, lo, hi, k = render_box_support(g, pl, prm)
    ref = []
    for p in range(pl.p):
        R = pl.rot[p].astype(np.float64).reshape(3, 3)
        Ri = np.linalg.inv(R)
        o = pl.origin[p].astype(np.float64)
        W, H = int(pl.wh[p, 0]), int(pl.wh[p, 1])
        sx, sy = float(pl.spacing[p, 0]), float(pl.spacing[p, 1])
        for v in range(H):
            for u in range(W):
                x1, x2 = (u + 0.5 - W / 2) * sx, (v + 0.5 - H / 2) * sy
                X = o + x1 * R[:, 0] + x2 * R[:, 1]
                num, den = prm.bg_alpha * prm.bg_color, prm.bg_alpha
                for i in range(g.n):
                    r = g.lraw[i].astype(np.float64)
                    L = np.array([[r[0] ** 2 + prm.beta, 0, 0], [r[1], r[3] ** 2 + prm.beta, 0],
                                  [r[2], r[4], r[5] ** 2 + prm.beta]])
                    S = np.linalg.inv(L @ L.T)
                    Sp = Ri @ S @ Ri.T
                    m = Ri @ (g.means[i].astype(np.float64) - o)
                    h = [math.sqrt(prm.chi2 * Sp[j, j]) for j in range(3)]
                    if abs(m[2]) > h[2] or abs(x1 - m[0]) > h[0] or abs(x2 - m[1]) > h[1]:
                        continue
                    dx = X - g.means[i].astype(np.float64)
                    d2 = float(dx @ L @ L.T @ dx)
                    w = math.exp(-0.5 * d2) / (1 + math.exp(-float(g.opacity[i])))
                    num += w * float(g.intensity[i])
                    den += w
                ref.append(num / den)
    assert np.all(k == 0)
    np.testing.assert_allclose(img, ref, rtol=1e-10, atol=1e-13)
    assert np.sum(D > prm.bg_alpha) > 20


def test_chi2_inf_is_the_plain_sum():
    """chi^2 = inf: every box is unbounded and every Gaussian kept, so the
    image is the unculled Gaussian sum of the ellipsoid reference."""
    g = synth.make_gaussians(30, 63, (0, 0, 0), (1, 1, 1), (0.05, 0.2), opacity="random")
    pl = synth.random_planes(2, 64, (12, 10), 1 / 12)
    prm = Params(chi2=math.inf)
    img, D, lo, hi, k = render_box_support(g, pl, prm)
    ref, Dr = oracle.render(g, pl, prm)
    np.testing.assert_allclose(img, ref, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(D, Dr, rtol=1e-12)
    assert np.all(k == 0)


def test_box_support_contains_the_ellipsoid_support():
    """The Eq. 13 box contains the Eq. 12 ellipse cut, and Phase 1 keeps
    every Gaussian whose ellipsoid meets the plane: for one Gaussian at a time
    the box-support weight equals the ellipsoid one wherever that is
    non-zero, and the sum over a scene dominates the ellipsoid sum."""
    prm = Params(bg_alpha=0.01)
    pl = synth.random_planes(2, 66, (20, 18), 1 / 16, 0.4, 0.6)
    g = synth.make_gaussians(25, 65, (0.25, 0.25, 0.25), (0.75, 0.75, 0.75), (0.05, 0.25), aniso_max=10.0)
    _, Db, _, _, _ = render_box_support(g, pl, prm)
    _, De = oracle.render(g, pl, prm)
    assert np.all(Db >= De - 1e-15)
    assert np.any(Db > De * (1 + 1e-3))
    for i in range(g.n):
        gi = synth.Gaussians(g.means[i:i + 1], g.lraw[i:i + 1], g.intensity[i:i + 1], g.opacity[i:i + 1])
        _, db, _, _, _ = render_box_support(gi, pl, prm)
        _, de = oracle.render(gi, pl, prm)
        on = de > prm.bg_alpha
        np.testing.assert_allclose(db[on], de[on], rtol=1e-12)


def test_borderline_box_edge_and_phase1():
    """A box edge through a pixel centre and a plane tangent to the
    ellipsoid are borderline: the interval spans both choices."""
    prm = Params(chi2=4.0, bg_alpha=0.1)
    pl = _plane(np.eye(3), (0, 0, 0), (21, 21), (0.5, 0.5))
    g = _one_gaussian((0.0, 0.0, 0.0), (1.5, 1.0, 2.0), c=1.0, a=0.0)
    img, D, lo, hi, k = render_box_support(g, pl, prm)
    row = 10 * 21
    # x1 = (u + 1/2 - 10.5) / 2: u = 16 sits on the edge h1 = 2 * 1.5 = 3
    assert k[row + 16] == 1 and k[row + 15] == 0 and k[row + 17] == 0
    w16 = 0.5 * math.exp(-0.5 * (3.0 / 1.5) ** 2)
    assert lo[row + 16] <= 0.0 + 1e-12 and hi[row + 16] >= w16 / (w16 + 0.1) - 1e-9
    assert img[row + 17] == 0.0 and img[row + 15] > 0.0
    # plane at t = h3 = 2 * 2: every in-box pixel is borderline
    g = _one_gaussian((0.0, 0.0, 4.0), (1.5, 1.0, 2.0), c=1.0, a=0.0)
    img, D, lo, hi, k = render_box_support(g, pl, prm)
    assert k[row + 10] == 1 and lo[row + 10] <= 1e-12 and hi[row + 10] > 0.05
    assert np.all(k[row:row + 21][np.abs(np.arange(21) - 10) > 6] == 0)


def test_sampled_pixels_match_the_full_image():
    g = synth.make_gaussians(40, 67, (0, 0, 0), (1, 1, 1), (0.05, 0.2), opacity="random")
    pl = synth.random_planes(3, 68, (10, 12), 1 / 10)
    pl.wh[:] = [[10, 12], [7, 5], [13, 9]]
    full, Df, _, _, _ = render_box_support(g, pl, Params())
    pix = synth.sample_pixels(pl, 50, 69)
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    part, Dp, _, _, _ = render_box_support(g, pl, Params(), pix=pix)
    np.testing.assert_array_equal(part, full[flat])
    np.testing.assert_array_equal(Dp, Df[flat])
