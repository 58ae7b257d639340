"""Pins of the densify / prune reference (oracle/densify.py): closed forms
for isotropic Gaussians, the covariance scaling of a split, the size measure
against the covariance computed by a library inverse of the precision, and
the borderline outcomes of constructed ties."""
import math

import numpy as np
import pytest

import oracle
from oracle import densify as D
from paper_2505_05643_amd import synth

BETA = 1e-4


def _iso(sigmas, a=1.0):
    """Isotropic Gaussians: L = I / sigma, so Sigma = sigma^2 I and trace = 3 sigma^2."""
    s = np.asarray(sigmas, dtype=np.float64)
    n = s.shape[0]
    raw = np.zeros((n, 6))
    d = np.sqrt(1.0 / s - BETA)
    raw[:, 0], raw[:, 3], raw[:, 5] = d, d, d
    f = np.float32
    return synth.Gaussians(np.zeros((n, 3), f) + np.arange(n, dtype=f)[:, None], raw.astype(f),
                           np.linspace(0.1, 0.9, n).astype(f), np.full(n, a, f))


def test_size_is_trace_of_covariance():
    """size^2 against the trace of the library inverse of the precision L L^T."""
    g = synth.make_gaussians(500, 3, (0, 0, 0), (1, 1, 1), (0.01, 0.3), aniso_max=20.0)
    L = oracle.activate_l(g.lraw, BETA)
    tr = np.trace(np.linalg.inv(L @ np.transpose(L, (0, 2, 1))), axis1=1, axis2=2)
    np.testing.assert_allclose(D.size2(g.lraw, BETA), tr, rtol=1e-9)


def test_split_scaling_divides_every_std():
    g = synth.make_gaussians(200, 4, (0, 0, 0), (1, 1, 1), (0.01, 0.3), aniso_max=20.0)
    phi = 1.6
    S = oracle.covariance(g.lraw, BETA)
    S2 = oracle.covariance(D.scaled_lraw(g.lraw, BETA, phi), BETA)
    np.testing.assert_allclose(S2, S / phi ** 2, rtol=1e-9, atol=1e-12 * np.abs(S).max())


def test_decisions_on_constructed_cases():
    sig = [0.1, 0.1, 0.1, 2.0, 100.0]      # size^2 = 0.03, 0.03, 0.03, 12, 30000
    g = _iso(sig)
    g.opacity[0] = math.log(0.001 / 0.999)  # alpha 0.001 < 0.005: prune
    acc = np.array([1.0, 0.0, 3e-3, 3e-3, 3e-3], np.float32)
    cnt = np.array([10, 0, 10, 10, 10], np.int32)
    d, possible = D.decisions(g.lraw, g.opacity, acc, cnt, BETA, 0.005, 2e-4, 1.0, 50.0)
    assert list(d) == [D.PRUNE, D.KEEP, D.CLONE, D.SPLIT, D.PRUNE]
    assert np.array_equal(possible, np.eye(4, dtype=bool)[d])  # nothing borderline
    # just under / over the gradient threshold (acc / cnt = 1.9e-4, 2.1e-4)
    d, _ = D.decisions(g.lraw[:2], np.ones(2, np.float32), np.array([1.9e-3, 2.1e-3], np.float32),
                       np.array([10, 10], np.int32), BETA, 0.005, 2e-4, 1.0, 0.0)
    assert list(d) == [D.KEEP, D.CLONE]


def test_borderline_ties_give_both_outcomes():
    """Comparisons whose sides are equal to float rounding admit either
    outcome: alpha at the opacity floor (prune or keep), the mean gradient at
    its threshold (keep or grow), size^2 at the split size (clone or split)."""
    s_split = math.sqrt(1.0 / 3.0)            # isotropic: size^2 = 3 sigma^2 = 1
    g = _iso([0.1, 0.1, s_split])
    g.opacity[0] = np.float32(math.log(0.005 / 0.995))
    acc = np.array([0.0, 2e-3, 1.0], np.float32)
    cnt = np.array([0, 10, 1], np.int32)
    d, possible = D.decisions(g.lraw, g.opacity, acc, cnt, BETA, 0.005, 2e-4, 1.0, 0.0)
    assert set(np.nonzero(possible[0])[0]) == {D.PRUNE, D.KEEP}
    assert set(np.nonzero(possible[1])[0]) == {D.KEEP, D.CLONE}
    assert set(np.nonzero(possible[2])[0]) == {D.CLONE, D.SPLIT}
    assert all(possible[i, d[i]] for i in range(3))


def test_outputs_in_order_with_closed_form_children():
    sig = [0.1, 2.0, 0.5]
    g = _iso(sig)
    acc = np.array([0.0, 1.0, 1.0], np.float32)
    cnt = np.array([5, 1, 1], np.int32)   # keep, split (size^2 12 > 1), clone (0.75 <= 1)
    rng = np.random.default_rng(0)
    z = rng.standard_normal((3, 2, 3))
    phi = 1.6
    means, lraw, inten, opac, src, d = D.densify(g, acc, cnt, z, BETA, 0.005, 2e-4, 1.0, 0.0, phi)
    assert list(d) == [D.KEEP, D.SPLIT, D.CLONE] and list(src) == [0, 1, 1, 2, 2]
    np.testing.assert_array_equal(means[0], g.means[0])
    # a split child of an isotropic Gaussian: mu + sigma z, std sigma / phi
    for c in range(2):
        np.testing.assert_allclose(means[1 + c], g.means[1].astype(np.float64) + 2.0 * z[1, c], rtol=0, atol=1e-5)
        np.testing.assert_allclose(lraw[1 + c][[0, 3, 5]], math.sqrt(phi / 2.0 - BETA), rtol=1e-5)
        np.testing.assert_allclose(lraw[1 + c][[1, 2, 4]], 0.0)
    np.testing.assert_array_equal(lraw[3], lraw[4])
    np.testing.assert_array_equal(means[3], means[4])
    np.testing.assert_allclose(inten, g.intensity[[0, 1, 1, 2, 2]])
