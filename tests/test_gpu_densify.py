"""Densify / prune and the Section 4.2 draw on the GPU against the
reference (oracle/densify.py): the float64 decisions of the reference, a
Gaussian whose comparison sits within rounding of its threshold allowed any
outcome the reference lists for it; copies bit for bit, split children and
draws to float rounding."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import densify as D
from paper_2505_05643_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BETA = 1e-4


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05643_amd import densify, raster
    return raster, densify


def _population(n, seed):
    """Mixed population: opacities around the floor, gradient statistics
    around the threshold, sizes on both sides of the split size."""
    rng = np.random.default_rng(seed)
    g = synth.make_gaussians(n, seed, (0, 0, 0), (4, 4, 4), (0.05, 1.5), aniso_max=8.0, opacity="random")
    g.opacity[:] = rng.uniform(-7.0, 3.0, n).astype(np.float32)
    cnt = rng.integers(0, 20, n).astype(np.int32)
    acc = (rng.uniform(0.0, 4e-4, n) * cnt).astype(np.float32)
    z = rng.standard_normal((n, 2, 3)).astype(np.float32)
    return g, acc, cnt, z


def test_sample_matches_reference(M):
    R, Dn = M
    dev = torch.device("cuda", 0)
    g = synth.make_gaussians(300, 11, (0, 0, 0), (1, 1, 1), (0.01, 0.3), aniso_max=30.0)
    rng = np.random.default_rng(1)
    idx = rng.integers(0, 300, 2000).astype(np.int32)
    idx[:3] = [-1, 300, 299]
    z = rng.standard_normal((2000, 3)).astype(np.float32)
    out = Dn.sample_gaussians(R.to_device(g, dev), torch.from_numpy(idx).to(dev), torch.from_numpy(z).to(dev),
                              BETA).cpu().numpy()
    assert np.all(np.isnan(out[:2]))
    ref = oracle.sample_gaussian(g.means[idx[2:]], g.lraw[idx[2:]], z[2:], BETA)
    scale = np.abs(ref - g.means[idx[2:]]).max()
    assert np.abs(out[2:] - ref).max() <= 1e-5 * max(scale, 1.0)


def test_accumulate_grad_norm(M):
    R, Dn = M
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(2)
    dm = rng.standard_normal((1000, 3)).astype(np.float32)
    acc = torch.full((1000,), 0.5, device=dev)
    cnt = torch.full((1000,), 3, dtype=torch.int32, device=dev)
    for _ in range(2):
        Dn.accumulate_grad_norm(torch.from_numpy(dm).to(dev), acc, cnt)
    ref = 0.5 + 2 * np.linalg.norm(dm.astype(np.float64), axis=1)
    np.testing.assert_allclose(acc.cpu().numpy(), ref, rtol=1e-6)
    assert np.all(cnt.cpu().numpy() == 5)


def _gpu_decisions(g, gm, gl, z, d, possible, phi):
    """The decision the GPU took for every Gaussian, read from its outputs:
    outside the reference's borderline Gaussians it must be the reference's
    (the output count of each stretch between borderline Gaussians follows);
    at a borderline Gaussian the outputs at the current position tell it
    (one or two bit-exact copies: keep or clone; two children: split;
    neither: prune).  Returns the decisions and the number of outputs walked."""
    nout = np.array([0, 1, 2, 2])
    border = np.nonzero(possible.sum(axis=1) > 1)[0]
    out = d.copy()
    m = gm.shape[0]
    ptr, prev = 0, 0

    def copy_at(j, i):
        return j < m and np.array_equal(gm[j], g.means[i]) and np.array_equal(gl[j], g.lraw[i])

    def children_at(j, i):
        if j + 1 >= m:
            return False
        cm, cl = D.children(g.means[i], g.lraw[i], z[i], BETA, phi)
        tol_m = 1e-5 * max(1.0, np.abs(cm).max())
        return (np.abs(gm[j:j + 2] - cm).max() <= tol_m
                and np.abs(gl[j:j + 2] - cl).max() <= 2e-6 * np.abs(cl).max() + 1e-6)

    for b in list(border) + [d.shape[0]]:
        ptr += int(nout[d[prev:b]].sum())
        if b == d.shape[0]:
            break
        if copy_at(ptr, b):
            out[b] = D.CLONE if copy_at(ptr + 1, b) else D.KEEP
        else:
            out[b] = D.SPLIT if children_at(ptr, b) else D.PRUNE
        ptr += int(nout[out[b]])
        prev = b + 1
    return out, ptr


@pytest.mark.parametrize("n,seed", [(1, 5), (257, 6), (20_000, 7), (600_000, 8)])
def test_densify_matches_reference(M, n, seed):
    R, Dn = M
    dev = torch.device("cuda", 0)
    g, acc, cnt, z = _population(n, seed)
    prm = Dn.DensifyParams(beta=BETA, min_opacity=0.005, grad_thresh=2e-4, split_size=1.0, max_size=3.0,
                           split_factor=1.6)
    out = Dn.densify(R.to_device(g, dev), torch.from_numpy(acc).to(dev), torch.from_numpy(cnt).to(dev),
                     torch.from_numpy(z).to(dev), prm)
    d, possible = D.decisions(g.lraw, g.opacity, acc, cnt, BETA, 0.005, 2e-4, 1.0, 3.0)
    if n > 100:
        assert all(np.any(d == k) for k in (D.PRUNE, D.KEEP, D.CLONE, D.SPLIT)), np.bincount(d)
    gm, gl = out.means.cpu().numpy(), out.lraw.cpu().numpy()
    gd, walked = _gpu_decisions(g, gm, gl, z, d, possible, 1.6)
    assert walked == gm.shape[0], "the outputs do not follow the reference's decisions"
    off = np.nonzero(gd != d)[0]
    assert np.all(possible[off, gd[off]]), "a decision outside the reference's borderline outcomes"
    n_border = int(np.sum(possible.sum(axis=1) > 1))
    assert n_border <= max(2, 1e-4 * n), n_border
    print(f"n={n}: {n_border} borderline Gaussians, {off.size} decided the other way")
    src = np.repeat(np.arange(n), np.array([0, 1, 2, 2])[gd])
    assert gm.shape[0] == src.shape[0]
    np.testing.assert_array_equal(out.intensity.cpu().numpy(), g.intensity[src])
    np.testing.assert_array_equal(out.opacity.cpu().numpy(), g.opacity[src])
    split = gd[src] == D.SPLIT
    np.testing.assert_array_equal(gm[~split], g.means[src[~split]])  # copies are exact
    np.testing.assert_array_equal(gl[~split], g.lraw[src[~split]])
    if split.any():
        first = np.nonzero(split & np.r_[True, src[1:] != src[:-1]])[0]  # first child of each split
        ref_m = np.empty((first.size * 2, 3))
        ref_l = np.empty((first.size * 2, 6))
        for q, j in enumerate(first):
            ref_m[2 * q:2 * q + 2], ref_l[2 * q:2 * q + 2] = D.children(g.means[src[j]], g.lraw[src[j]],
                                                                        z[src[j]], BETA, 1.6)
        sel = np.sort(np.concatenate([first, first + 1]))
        assert np.abs(gm[sel] - ref_m).max() <= 1e-5 * max(1.0, np.abs(ref_m).max())
        np.testing.assert_allclose(gl[sel], ref_l, rtol=2e-6, atol=1e-6 * np.abs(ref_l).max())


def test_densify_capacity_overflow_reports_the_total(M):
    R, Dn = M
    from paper_2505_05643_amd import _lib
    dev = torch.device("cuda", 0)
    g, acc, cnt, z = _population(3000, 9)
    _, possible = D.decisions(g.lraw, g.opacity, acc, cnt, BETA, 0.005, 2e-4, 1.0, 0.0)
    assert np.all(possible.sum(axis=1) == 1)  # no borderline Gaussian: the total is fixed
    _, _, _, _, src, _ = D.densify(g, acc, cnt, z, BETA, 0.005, 2e-4, 1.0, 0.0, 1.6)
    total = src.shape[0]
    cap = total - 7
    gd = R.to_device(g, dev)
    out = [torch.full((cap + 16,) + s, -1.0, device=dev) for s in ((3,), (6,), (), ())]
    ws = torch.empty((_lib.lib.ug_densify_workspace_bytes(3000) + 3) // 4, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    cg = R._c_gauss(gd)
    co = _lib.UgGaussiansMut(*(t.data_ptr() for t in out), cap)
    dp = _lib.UgDensifyParams()
    _lib.lib.ug_densify_params_default(ctypes.byref(dp))
    da, dc, dz = (torch.from_numpy(x).to(dev) for x in (acc, cnt, z))
    code = _lib.lib.ug_densify(ctypes.byref(cg), da.data_ptr(), dc.data_ptr(), dz.data_ptr(), ctypes.byref(dp),
                               ctypes.byref(co), cap, count.data_ptr(), ws.data_ptr(), R._stream())
    assert code == 0
    assert int(count.item()) == total
    assert torch.all(out[2][cap:] == -1.0)  # nothing past the capacity
    np.testing.assert_array_equal(out[2][:cap].cpu().numpy(), g.intensity[src[:cap]])
