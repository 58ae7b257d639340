"""Covariance parameterisation study (Section 4.2): how much float32
rounding each route loses as the covariance grows anisotropic.

For each anisotropy (largest over smallest standard deviation) a seeded
population is stored in the three raw layouts (Eq. 11's triangular factor,
Eq. 10's symmetric M, quaternion and scales; ``synth.param_study_inputs``),
and ``ug_param_eval`` evaluates every route in float32 and in float64 on the
device.  Reported per route: the relative error of the float32 covariance
and squared distance against the float64 evaluation of the same stored
parameters; for the draw y = F z, which depends on the factor chosen, the
relative error of its squared Mahalanobis length y^T Sigma^-1 y (the
precision formed directly in float64) against |z|^2, which every exact
factor gives (median, 99th percentile, maximum, and the count of non-finite
results); the storage error (the float64 covariance of the float32-stored
parameters against the covariance they were built from), and (``throughput``) the float32 kernel's rate.
"""
from __future__ import annotations

import torch

from . import _lib, synth
from ._lib import check, lib
from . import raster as R

ROUTES = {"tri": _lib.UG_PARAM_TRI, "sym": _lib.UG_PARAM_SYM, "quat": _lib.UG_PARAM_QUAT}


def evaluate(kind: int, raw: torch.Tensor, z: torch.Tensor, delta: torch.Tensor, beta: float, fp64: bool):
    """(sigma [n,6], draw [n,3], d2 [n]) of one route on the device."""
    n = raw.shape[0]
    dt = torch.float64 if fp64 else torch.float32
    sigma = torch.empty(n, 6, dtype=dt, device=raw.device)
    draw = torch.empty(n, 3, dtype=dt, device=raw.device)
    d2 = torch.empty(n, dtype=dt, device=raw.device)
    check(lib.ug_param_eval(int(kind), 1 if fp64 else 0, raw.data_ptr(), z.data_ptr(), delta.data_ptr(), n,
                            float(beta), sigma.data_ptr(), draw.data_ptr(), d2.data_ptr(), R._stream()),
          "ug_param_eval")
    return sigma, draw, d2


def _frob(s: torch.Tensor) -> torch.Tensor:
    """Frobenius norm of symmetric matrices stored as (11, 12, 13, 22, 23, 33)."""
    w = torch.tensor([1.0, 2.0, 2.0, 1.0, 2.0, 1.0], dtype=s.dtype, device=s.device)
    return torch.sqrt(torch.sum(w * s * s, dim=1))


def _stats(err: torch.Tensor) -> dict:
    e = err.double()
    fin = torch.isfinite(e)
    nonfinite = int((~fin).sum())
    e = e[fin]
    if e.numel() == 0:
        return {"median": None, "p99": None, "max": None, "nonfinite": nonfinite}
    return {"median": float(torch.quantile(e, 0.5)), "p99": float(torch.quantile(e, 0.99)),
            "max": float(e.max()), "nonfinite": nonfinite}


def study(anisos=(1.0, 10.0, 100.0, 1e3, 1e4), n: int = 262_144, seed: int = 0, beta: float = 1e-4,
          device=None) -> dict:
    device = torch.device(device) if device is not None else torch.device("cuda", 0)
    out = {"gaussians": n, "beta": beta, "anisotropy": {}}
    for k, a in enumerate(anisos):
        d = synth.param_study_inputs(n, seed + k, float(a), beta)
        z = torch.from_numpy(d["z"]).to(device)
        delta = torch.from_numpy(d["delta"]).to(device)
        s = torch.from_numpy(d["scales"]).to(device)
        rot = torch.from_numpy(d["rots"]).to(device)
        full = rot @ (rot.transpose(1, 2) * (s * s)[:, :, None])
        target = torch.stack([full[:, 0, 0], full[:, 0, 1], full[:, 0, 2], full[:, 1, 1], full[:, 1, 2],
                              full[:, 2, 2]], dim=1)
        res = {}
        for name, kind in ROUTES.items():
            raw = torch.from_numpy(d[name]).to(device)
            s32, y32, q32 = evaluate(kind, raw, z, delta, beta, False)
            s64, _, q64 = evaluate(kind, raw, z, delta, beta, True)
            _, _, len64 = evaluate(kind, raw, z, y32.contiguous(), beta, True)  # y32^T Sigma^-1 y32
            z2 = torch.sum(z.double() ** 2, dim=1)
            res[name] = {
                "sigma": _stats(_frob(s32.double() - s64) / _frob(s64)),
                "draw": _stats((len64 - z2).abs() / z2),
                "d2": _stats((q32.double() - q64).abs() / q64.abs()),
                "storage": _stats(_frob(s64 - target) / _frob(target)),
            }
        out["anisotropy"][f"{a:g}"] = res
    return out


def throughput(n: int = 1 << 22, reps: int = 20, beta: float = 1e-4, device=None) -> dict:
    """Float32 evaluation rate of each route over ``n`` Gaussians (a seeded
    population of anisotropy 100, repeated), HIP events around ``reps`` back-to-back launches on the stream.
    Algorithmic bytes: 56 read (raw 32, z 12, delta 12) and 40 written
    (sigma 24, draw 12, d2 4) per Gaussian."""
    device = torch.device(device) if device is not None else torch.device("cuda", 0)
    base = 1 << 18  # a seeded population, repeated up to n on the device
    d = synth.param_study_inputs(base, 99, 100.0, beta)
    rep = (n + base - 1) // base

    def dev(a):
        return torch.from_numpy(a).to(device).repeat(rep, 1)[:n].contiguous()

    z = dev(d["z"])
    delta = dev(d["delta"])
    sigma = torch.empty(n, 6, device=device)
    draw = torch.empty(n, 3, device=device)
    d2 = torch.empty(n, device=device)
    out = {"gaussians": n}
    for name, kind in ROUTES.items():
        raw = dev(d[name])

        def call():
            check(lib.ug_param_eval(int(kind), 0, raw.data_ptr(), z.data_ptr(), delta.data_ptr(), n, float(beta),
                                    sigma.data_ptr(), draw.data_ptr(), d2.data_ptr(), R._stream()), "ug_param_eval")

        call()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            call()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = {"ms": ms, "ggaussians_per_s": n / (ms * 1e6), "hbm_gbs": 96 * n / (ms * 1e6)}
    return out
