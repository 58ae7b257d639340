"""Pins of the parameterisation-study reference: every route's covariance,
factor and distance against the covariance they were built from, scipy's
rotation and normal density, and the render reference's draw.  None of
these tests uses the HIP path."""
import numpy as np
import pytest
import scipy.stats
from scipy.spatial.transform import Rotation

import oracle
from oracle import params as P
from paper_2505_05643_amd import synth

BETA = 1e-4


def _inputs(aniso, n=64, seed=3):
    d = synth.param_study_inputs(n, seed, aniso, BETA)
    target = d["rots"] @ (np.transpose(d["rots"], (0, 2, 1)) * (d["scales"] ** 2)[:, :, None])
    return d, target


def _fp64_raw(d, kind):
    """The raw layouts recomputed in float64 (no float32 rounding)."""
    s, R = d["scales"], d["rots"]
    if kind == P.TRI:
        raw = np.zeros((s.shape[0], 8))
        raw[:, :6] = synth.scales_rots_to_lraw(s, R, BETA)
        return raw
    if kind == P.SYM:
        ev = np.sqrt(s ** -2 - BETA)
        M = R @ (np.transpose(R, (0, 2, 1)) * ev[:, :, None])
        raw = np.zeros((s.shape[0], 8))
        raw[:, :6] = np.stack([M[:, 0, 0], M[:, 0, 1], M[:, 0, 2], M[:, 1, 1], M[:, 1, 2], M[:, 2, 2]], axis=1)
        return raw
    raw = np.asarray(d["quat"], dtype=np.float64)
    raw[:, 4:7] = s
    return raw


@pytest.mark.parametrize("aniso", [1.0, 10.0, 100.0])
@pytest.mark.parametrize("kind", [P.TRI, P.SYM, P.QUAT])
def test_routes_reproduce_the_covariance_and_factor(kind, aniso):
    d, target = _inputs(aniso)
    raw = _fp64_raw(d, kind)
    if kind == P.QUAT:  # the stored quaternion is float32: compare with its own rotation
        R = P.quat_rotation(raw[:, :4])
        target = R @ (np.transpose(R, (0, 2, 1)) * (d["scales"] ** 2)[:, :, None])
    S = P.covariance(kind, raw, BETA)
    np.testing.assert_allclose(S, target, rtol=0, atol=1e-9 * np.abs(target).max())
    np.testing.assert_allclose(P.precision(kind, raw, BETA) @ S, np.broadcast_to(np.eye(3), S.shape), atol=1e-8)
    # the draw's factor F (its columns are the draws of the unit vectors) has F F^T = Sigma
    F = np.stack([P.draw(kind, raw, np.tile(e, (raw.shape[0], 1)), BETA) for e in np.eye(3)], axis=-1)
    np.testing.assert_allclose(F @ np.transpose(F, (0, 2, 1)), target, rtol=0, atol=1e-9 * np.abs(target).max())


def test_mahalanobis_matches_the_library_density():
    d, target = _inputs(20.0, n=16)
    raw = _fp64_raw(d, P.TRI)
    delta = d["delta"].astype(np.float64)
    got = P.mahalanobis(P.TRI, raw, delta, BETA)
    S = P.covariance(P.TRI, raw, BETA)
    for i in range(16):
        mvn = scipy.stats.multivariate_normal(np.zeros(3), S[i])
        ref = -2.0 * (mvn.logpdf(delta[i]) - mvn.logpdf(np.zeros(3)))
        assert got[i] == pytest.approx(ref, rel=1e-9)
    # the offsets were drawn at Mahalanobis distance in [0.5, 2.8]
    assert np.all(got > 0.24) and np.all(got < 7.9)


def test_quaternion_rotation_matches_scipy_and_normalises():
    rng = np.random.default_rng(5)
    q = rng.standard_normal((20, 4))
    R = P.quat_rotation(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()  # scipy orders (x, y, z, w)
    np.testing.assert_allclose(R, ref, atol=1e-14)
    np.testing.assert_allclose(P.quat_rotation(3.7 * q), R, atol=1e-14)


def test_triangular_draw_is_the_render_reference_draw():
    d, _ = _inputs(30.0, n=32)
    mu = np.zeros((32, 3))
    a = P.draw(P.TRI, d["tri"], d["z"], BETA)
    b = oracle.sample_gaussian(mu, d["tri"][:, :6], d["z"], BETA)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
