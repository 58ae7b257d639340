"""Reference for the covariance parameterisation study (Section 4.2).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Section 4.2 compares three ways to keep a Gaussian's covariance positive
definite: scale and unit quaternion, Sigma = R diag(s^2) R^T (3D Gaussian
splatting); a symmetric M with Sigma^-1 = M M^T + beta I (Eq. 10); and the
lower-triangular L of Eq. 11 with Sigma^-1 = L L^T.  Resampling needs the
covariance itself and a factor to draw y = mu + F z with F F^T = Sigma;
rendering needs d^2 = delta^T Sigma^-1 delta.  Everything here is float64
from the stored float32 parameters (so it is the value each float32 route
approximates):

* ``precision``  Sigma^-1 of each parameterisation, formed directly;
* ``covariance`` Sigma: the explicit inverse of the precision (Eq. 10,
  Eq. 11) or R diag(s^2) R^T (quaternion);
* ``draw``       F z with the factor each route uses: L^-T (Eq. 11, back
  substitution), the lower Cholesky factor of Sigma (Eq. 10: invert, then
  factorise), R diag(s) (quaternion);
* ``mahalanobis`` delta^T Sigma^-1 delta.

Raw layouts (8 floats per Gaussian, the last ones unused):
TRI (l11, l21, l31, l22, l32, l33) with diagonal l^2 + beta (Eq. 11, the
entry printed at (3,2) read as l32); SYM (M11, M12, M13, M22, M23, M33);
QUAT (qw, qx, qy, qz, s1, s2, s3), the quaternion normalised before use.
"""
from __future__ import annotations

import numpy as np

TRI, SYM, QUAT = 0, 1, 2
KINDS = {"tri": TRI, "sym": SYM, "quat": QUAT}


def _sym(raw):
    r = np.asarray(raw, dtype=np.float64)
    M = np.empty(r.shape[:-1] + (3, 3))
    M[..., 0, 0], M[..., 0, 1], M[..., 0, 2] = r[..., 0], r[..., 1], r[..., 2]
    M[..., 1, 0], M[..., 1, 1], M[..., 1, 2] = r[..., 1], r[..., 3], r[..., 4]
    M[..., 2, 0], M[..., 2, 1], M[..., 2, 2] = r[..., 2], r[..., 4], r[..., 5]
    return M


def _tri(raw, beta):
    r = np.asarray(raw, dtype=np.float64)
    L = np.zeros(r.shape[:-1] + (3, 3))
    L[..., 0, 0] = r[..., 0] ** 2 + beta
    L[..., 1, 0] = r[..., 1]
    L[..., 2, 0] = r[..., 2]
    L[..., 1, 1] = r[..., 3] ** 2 + beta
    L[..., 2, 1] = r[..., 4]
    L[..., 2, 2] = r[..., 5] ** 2 + beta
    return L


def quat_rotation(q):
    """Rotation matrix of the normalised quaternion (w, x, y, z)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def precision(kind: int, raw, beta: float) -> np.ndarray:
    raw = np.asarray(raw, dtype=np.float64)
    if kind == TRI:
        L = _tri(raw[..., :6], beta)
        return L @ np.swapaxes(L, -1, -2)
    if kind == SYM:
        M = _sym(raw[..., :6])
        return M @ np.swapaxes(M, -1, -2) + beta * np.eye(3)
    R = quat_rotation(raw[..., :4])
    s = raw[..., 4:7]
    return R @ (np.swapaxes(R, -1, -2) / (s * s)[..., :, None])


def covariance(kind: int, raw, beta: float) -> np.ndarray:
    raw = np.asarray(raw, dtype=np.float64)
    if kind == QUAT:
        R = quat_rotation(raw[..., :4])
        s = raw[..., 4:7]
        return R @ (np.swapaxes(R, -1, -2) * (s * s)[..., :, None])
    return np.linalg.inv(precision(kind, raw, beta))


def draw(kind: int, raw, z, beta: float) -> np.ndarray:
    """F z per Gaussian, F the factor the route uses (see the module text)."""
    raw = np.asarray(raw, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if kind == TRI:
        L = _tri(raw[..., :6], beta)
        return np.linalg.solve(np.swapaxes(L, -1, -2), z[..., None])[..., 0]
    if kind == SYM:
        C = np.linalg.cholesky(covariance(SYM, raw, beta))
        return (C @ z[..., None])[..., 0]
    R = quat_rotation(raw[..., :4])
    return (R @ (raw[..., 4:7] * z)[..., None])[..., 0]


def mahalanobis(kind: int, raw, delta, beta: float) -> np.ndarray:
    d = np.asarray(delta, dtype=np.float64)
    P = precision(kind, raw, beta)
    return np.einsum("...j,...jk,...k->...", d, P, d)
