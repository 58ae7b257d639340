"""Seeded workload generators: shapes, ranges and determinism (no method arithmetic)."""
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
