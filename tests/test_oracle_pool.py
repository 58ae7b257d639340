"""The multi-process driver of the reference returns what the reference
returns, to the rounding of a different chunking (numpy's contractions may
sum in another order for another chunk shape): per-point values and the
gradient (a sum over points) within 1e-12, the borderline counts exactly."""
import numpy as np

import oracle
from oracle import pool
from paper_2505_05643_amd import synth


def test_pool_equals_serial_reference():
    g = synth.make_gaussians(300, 91, (0, 0, 0), (1, 1, 1), (0.03, 0.15), aniso_max=5.0, opacity="random")
    pl = synth.random_planes(2, 92, (20, 17), 1 / 24, 0.4, 0.6)
    X = oracle.plane_points(pl)
    prm = oracle.Params(chi2=7.815, bg_alpha=0.02, bg_color=0.1)
    a = oracle.render_points(g, X, prm)
    b = pool.render_points(g, X, prm, workers=3)
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(x))
    la = oracle.ambiguity_points(g, X, prm)
    lb = pool.ambiguity_points(g, X, prm, workers=3)
    for x, y in zip(la[:2], lb[:2]):
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(x))
    assert np.array_equal(la[2], lb[2])
    dout = np.random.default_rng(3).standard_normal(X.shape[0])
    dout[::3] = 0.0
    ga = oracle.grad_points(g, X, dout, prm)
    gb = pool.grad_points(g, X, dout, prm, workers=3)
    for k in ga:
        assert np.max(np.abs(ga[k] - gb[k])) <= 1e-12 * np.max(np.abs(ga[k])), k
