"""Seeded workload generators: shapes, ranges and determinism (no method arithmetic)."""
import math

import numpy as np

from paper_2505_05643_amd import synth


def test_config_shapes_small():
    g, pl, tg = synth.make_config(0)
    assert g.n == 1000 and tg.n == 1000 and pl.p == 4
    assert g.means.dtype == np.float32 and g.lraw.shape == (1000, 6)
    assert np.all((g.means >= 0) & (g.means <= 1))
    assert pl.npix == 4 * 128 * 128
    assert not np.array_equal(g.means, tg.means)
    g2, _, _ = synth.make_config(0)
    assert np.array_equal(g.lraw, g2.lraw)          # seeded


def test_plane_frames_are_right_handed_orthonormal():
    for k in (0, 1, 3, 4):
        pl = synth.config_planes(k)
        R = pl.rot.astype(np.float64).reshape(-1, 3, 3)
        np.testing.assert_allclose(R @ np.transpose(R, (0, 2, 1)), np.broadcast_to(np.eye(3), R.shape), atol=1e-6)
        np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-6)


def test_ragged_config_sizes():
    pl = synth.config_planes(3)
    assert pl.p == 128
    sizes = {tuple(x) for x in pl.wh.tolist()}
    assert sizes <= set(synth.RAGGED_SIZES) and len(sizes) == 4


def test_sample_pixels_in_range():
    pl = synth.config_planes(3)
    pix = synth.sample_pixels(pl, 1000, 7)
    assert pix.shape == (1000, 3)
    assert np.all(pix[:, 1] < pl.wh[pix[:, 0], 0]) and np.all(pix[:, 2] < pl.wh[pix[:, 0], 1])


# ---------------------------------------------------------------- reconstruction and study inputs
def test_volume_sweeps_frames_positions_and_jitter():
    for view, normal in (("axial", (0, 0, 1)), ("coronal", (0, -1, 0)), ("sagittal", (1, 0, 0))):
        pl = synth.volume_sweep(view, 8, 32)
        R = pl.rot.astype(np.float64).reshape(-1, 3, 3)
        assert np.allclose(np.einsum("pji,pjk->pik", R, R), np.eye(3), atol=1e-6)
        assert np.allclose(np.linalg.det(R), 1.0, atol=1e-6)
        assert np.allclose(R[:, :, 2], normal, atol=1e-7)
        along = pl.origin.astype(np.float64) @ np.abs(np.asarray(normal, dtype=np.float64))
        np.testing.assert_allclose(along, (np.arange(8) + 0.5) / 8, atol=1e-7)
        off = pl.origin.astype(np.float64) - np.outer(along, np.abs(normal))
        other = off + 0.5 * np.abs(np.asarray(normal, dtype=np.float64))
        np.testing.assert_allclose(other, 0.5, atol=1e-7)  # centred in the other directions
        assert np.all(pl.spacing == np.float32(1 / 32)) and np.all(pl.wh == 32)
    a = synth.volume_sweep("axial", 50, 16, 5.0, 3)
    b = synth.volume_sweep("axial", 50, 16, 5.0, 3)
    assert np.array_equal(a.rot, b.rot)
    n = a.rot.astype(np.float64).reshape(-1, 3, 3)[:, :, 2]
    tilt = np.degrees(np.arccos(np.clip(n[:, 2], -1, 1)))
    assert tilt.max() <= math.hypot(5.0, 5.0) + 1e-3 and tilt.max() > 2.0


def test_phantom_structure():
    g = synth.phantom_gaussians(2000, 9)
    assert g.n == 2000 and np.all(np.isfinite(g.lraw))
    r = np.array([0.38, 0.32, 0.42])
    rad = np.linalg.norm((g.means.astype(np.float64) - 0.5) / r, axis=1)
    shell, inner = rad[:1000], rad[1000:]
    np.testing.assert_allclose(shell, 1.0, atol=1e-6)
    assert inner.max() <= 0.85 + 1e-6
    assert g.intensity[:1000].min() >= 0.7 and g.intensity[1000:].max() <= 0.6
    assert np.array_equal(synth.phantom_gaussians(2000, 9).means, g.means)


def test_paper_init_section_4_5():
    g = synth.paper_init(5000, 4)
    assert g.means.min() >= 0 and g.means.max() < 1
    assert g.lraw.min() >= 4 and g.lraw.max() < 5
    assert np.all(g.intensity == np.float32(0.5)) and np.all(g.opacity == np.float32(1.0))


def test_param_study_inputs_shapes_and_distances():
    d = synth.param_study_inputs(256, 5, 100.0)
    for k in ("tri", "sym", "quat"):
        assert d[k].shape == (256, 8) and d[k].dtype == np.float32 and np.all(d[k][:, 7] == 0)
    assert np.all(d["tri"][:, 6:] == 0) and np.all(d["sym"][:, 6:] == 0)
    np.testing.assert_allclose(np.linalg.norm(d["quat"][:, :4], axis=1), 1.0, atol=1e-6)
    s = d["scales"]
    np.testing.assert_allclose(s.max(axis=1) / s.min(axis=1), 100.0, rtol=1e-12)
    # delta = R (s * w) with |w| in [0.5, 2.8]: its Mahalanobis length is |w|
    w = np.einsum("nji,nj->ni", d["rots"], d["delta"].astype(np.float64)) / s
    length = np.linalg.norm(w, axis=1)
    assert length.min() >= 0.5 - 1e-3 and length.max() <= 2.8 + 1e-3


def test_rescale_keeps_every_squared_distance():
    # positions, origins and spacings scale by f, the precision by 1/f^2: the
    # factor L (diagonal l^2 + beta) by 1/f, so d^2 = |L^T (X - mu)|^2 of a
    # pixel point and a Gaussian is the same in both frames
    g = synth.make_gaussians(40, 8, (0, 0, 0), (256, 256, 256), (0.5, 8.0))
    pl = synth.random_planes(2, 9, (16, 12), 4.0, 100, 150)
    f = 1.0 / 256.0
    g2, pl2 = synth.rescale(g, pl, f)
    beta = synth.DEFAULT_BETA

    def factor(lr):
        lr = lr.astype(np.float64)
        L = np.zeros((lr.shape[0], 3, 3))
        L[:, 0, 0] = lr[:, 0] ** 2 + beta
        L[:, 1, 0], L[:, 2, 0] = lr[:, 1], lr[:, 2]
        L[:, 1, 1] = lr[:, 3] ** 2 + beta
        L[:, 2, 1] = lr[:, 4]
        L[:, 2, 2] = lr[:, 5] ** 2 + beta
        return L

    np.testing.assert_allclose(factor(g2.lraw), factor(g.lraw) / f, rtol=2e-6)
    np.testing.assert_allclose(g2.means, g.means * f, rtol=1e-6)
    np.testing.assert_allclose(pl2.origin, pl.origin * f, rtol=1e-6)
    np.testing.assert_allclose(pl2.spacing, pl.spacing * f, rtol=1e-6)
    assert np.array_equal(pl2.rot, pl.rot) and np.array_equal(pl2.wh, pl.wh)
    assert np.array_equal(g2.intensity, g.intensity) and np.array_equal(g2.opacity, g.opacity)

    def d2(gg, pp):
        R = pp.rot[0].astype(np.float64).reshape(3, 3)
        x = (np.arange(16) + 0.5 - 8) * pp.spacing[0, 0]
        y = (np.arange(12) + 0.5 - 6) * pp.spacing[0, 1]
        X = pp.origin[0].astype(np.float64) + x[None, :, None] * R[:, 0] + y[:, None, None] * R[:, 1]
        delta = X.reshape(-1, 1, 3) - gg.means.astype(np.float64)[None]
        return np.sum(np.einsum("nji,pnj->pni", factor(gg.lraw), delta) ** 2, axis=2)

    np.testing.assert_allclose(d2(g2, pl2), d2(g, pl), rtol=1e-5, atol=1e-6)
