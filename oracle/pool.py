"""Multi-process driver of the FP64 reference for large point samples.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

The reference evaluates every Gaussian at every point, so a sample of a few
hundred pixels against a million Gaussians costs minutes on one core.  This
module only splits the points into chunks and runs the unchanged
``render_points``, ``ambiguity_points`` or ``grad_points`` on each chunk in
a child Python process (started with ``subprocess``, so no child inherits
a GPU context or open device files; children see no GPU).  Inputs and
outputs travel through ``.npz`` files.  Per-point outputs are concatenated
in point order; the gradient, a sum over points, is the sum of the chunks'
sums.  No arithmetic of the method lives here.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

import importlib

import numpy as np

# the submodule (the package re-exports a function of the same name)
_r = importlib.import_module(__package__ + ".render")

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import importlib
r = importlib.import_module("oracle.render")


class G:
    pass


z = np.load(sys.argv[2])
g = G()
for k in ("means", "lraw", "intensity", "opacity"):
    setattr(g, k, z[k])
prm = r.Params(beta=float(z["beta"]), chi2=float(z["chi2"]), bg_alpha=float(z["bg_alpha"]),
               bg_color=float(z["bg_color"]))
c = np.load(sys.argv[3])
kind = sys.argv[4]
if kind == "render":
    out, den = r.render_points(g, c["X"], prm)
    np.savez(sys.argv[5], a=out, b=den)
elif kind == "ambiguity":
    lo, hi, k = r.ambiguity_points(g, c["X"], prm)
    np.savez(sys.argv[5], a=lo, b=hi, c=k)
else:
    d = r.grad_points(g, c["X"], c["dout"], prm)
    np.savez(sys.argv[5], **d)
"""


def default_workers() -> int:
    """Worker count: the cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _split(m: int, workers: int):
    parts = max(1, min(m, workers))
    edges = np.linspace(0, m, parts + 1).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def _run(kind: str, g, params, chunks, timeout: float):
    """Runs one child per chunk (dicts of arrays); returns their npz outputs."""
    params = params or _r.Params()
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    with tempfile.TemporaryDirectory(prefix="ug_oracle_") as tmp:
        gpath = os.path.join(tmp, "g.npz")
        np.savez(gpath, means=np.asarray(g.means), lraw=np.asarray(g.lraw), intensity=np.asarray(g.intensity),
                 opacity=np.asarray(g.opacity), beta=params.beta, chi2=params.chi2, bg_alpha=params.bg_alpha,
                 bg_color=params.bg_color)
        procs = []
        for i, ch in enumerate(chunks):
            cpath = os.path.join(tmp, f"in{i}.npz")
            opath = os.path.join(tmp, f"out{i}.npz")
            np.savez(cpath, **ch)
            procs.append((subprocess.Popen([sys.executable, "-c", _CHILD, _ROOT, gpath, cpath, kind, opath],
                                           env=env, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE), opath))
        outs, err = [], None
        for pr, opath in procs:
            try:
                _, se = pr.communicate(timeout=timeout)
            except subprocess.TimeoutExpired:
                pr.kill()
                pr.communicate()
                err = err or f"oracle child timed out after {timeout} s"
                continue
            if pr.returncode != 0:
                err = err or f"oracle child failed ({pr.returncode}):\n{se.decode(errors='replace')[-2000:]}"
                continue
            with np.load(opath) as z:
                outs.append({k: z[k] for k in z.files})
        if err:
            raise RuntimeError(err)
    return outs


def render_points(g, X, params=None, workers: int | None = None, timeout: float = 900.0):
    """``render.render_points`` over the points X [M,3], chunked over workers."""
    X = np.asarray(X, dtype=np.float64)
    workers = workers or default_workers()
    if workers == 1 or X.shape[0] < 2:
        return _r.render_points(g, X, params)
    outs = _run("render", g, params, [{"X": X[a:b]} for a, b in _split(X.shape[0], workers)], timeout)
    return np.concatenate([o["a"] for o in outs]), np.concatenate([o["b"] for o in outs])


def ambiguity_points(g, X, params=None, workers: int | None = None, timeout: float = 900.0):
    """``render.ambiguity_points`` over the points X [M,3], chunked over workers."""
    X = np.asarray(X, dtype=np.float64)
    workers = workers or default_workers()
    if workers == 1 or X.shape[0] < 2:
        return _r.ambiguity_points(g, X, params)
    outs = _run("ambiguity", g, params, [{"X": X[a:b]} for a, b in _split(X.shape[0], workers)], timeout)
    return tuple(np.concatenate([o[k] for o in outs]) for k in ("a", "b", "c"))


def grad_points(g, X, dout, params=None, workers: int | None = None, timeout: float = 900.0):
    """``render.grad_points`` of sum_x dout(x) c_hat(x): the sum over chunks of
    the points with non-zero dout."""
    X = np.asarray(X, dtype=np.float64)
    dout = np.asarray(dout, dtype=np.float64)
    workers = workers or default_workers()
    nz = np.nonzero(dout)[0]
    if workers == 1 or nz.size < 2:
        return _r.grad_points(g, X, dout, params)
    X, dout = X[nz], dout[nz]
    outs = _run("grad", g, params, [{"X": X[a:b], "dout": dout[a:b]} for a, b in _split(X.shape[0], workers)],
                timeout)
    return {k: np.sum([o[k] for o in outs], axis=0) for k in ("means", "lraw", "intensity", "opacity")}
