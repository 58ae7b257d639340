"""Adjoint parity: HIP backward vs the oracle's analytic gradient and FP64
finite differences of the oracle's forward."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_05643_amd import synth
from tests.parity import check_grads, oracle_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05643_amd import raster
    return raster


def _fwd_bwd(R, g, pl, dimg, params=None):
    params = params or R.Params()
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    plan = R.Plan(g.n, pl.wh, params, device=dev)
    plan.fit(gd, pd)
    img = plan.render(gd, pd)
    grads = plan.backward(gd, pd, img, torch.from_numpy(np.asarray(dimg, dtype=np.float32)).to(dev))
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy().astype(np.float64) for k, v in zip(("means", "lraw", "intensity", "opacity"), grads)}
    return img.cpu().numpy(), out, plan


def test_config0_gradients_full(R):
    g, pl, _ = synth.make_config(0)
    rng = np.random.default_rng(1)
    dimg = rng.standard_normal(pl.npix)
    _, gg, plan = _fwd_bwd(R, g, pl, dimg)
    ref = oracle.grad(g, pl, dimg.astype(np.float32).astype(np.float64), oracle_params(plan.params))
    print("c0 grads", check_grads(gg, ref))


def test_mse_loss_gradients_random_opacity(R):
    """d_image from an MSE against a second Gaussian set, as in training."""
    g = synth.make_gaussians(250, 51, (0, 0, 0), (1, 1, 1), (0.03, 0.15), aniso_max=10.0, opacity="random")
    t = synth.make_gaussians(250, 52, (0, 0, 0), (1, 1, 1), (0.03, 0.15))
    pl = synth.random_planes(3, 53, (40, 33), 1 / 36, 0.35, 0.65)
    img_ref, _ = oracle.render(t, pl)
    op = oracle.Params()
    cur, _ = oracle.render(g, pl, op)
    dimg = 2.0 * (cur - img_ref) / cur.size
    for bm in (0, 2):
        _, gg, plan = _fwd_bwd(R, g, pl, dimg, R.Params(box_mode=bm, tile_w=16, tile_h=8))
        ref = oracle.grad(g, pl, dimg.astype(np.float32).astype(np.float64), oracle_params(plan.params))
        check_grads(gg, ref)


@pytest.mark.parametrize("chi2", [60.0, 200.0])
def test_large_cutoff_forward_and_gradients(R, chi2):
    """Cut-offs near and beyond chi^2 = 88.7, where the kernels' scaled
    weights switch to dropping weights below 2^-64 of a Gaussian's peak (a
    stated reading of Eq. 12 for such chi^2): image and gradients against the
    oracle's exact cut-off, no overflow or non-finite value anywhere."""
    from tests.parity import check_image
    g = synth.make_gaussians(200, 61, (0, 0, 0), (1, 1, 1), (0.03, 0.12), aniso_max=6.0, opacity="random")
    pl = synth.random_planes(3, 62, (36, 30), 1 / 32, 0.35, 0.65)
    rng = np.random.default_rng(63)
    dimg = rng.standard_normal(pl.npix).astype(np.float32).astype(np.float64)
    for tw, th in ((16, 16), (32, 16)):
        img, gg, plan = _fwd_bwd(R, g, pl, dimg, R.Params(chi2=chi2, tile_w=tw, tile_h=th, box_mode=2))
        assert np.all(np.isfinite(img)) and all(np.all(np.isfinite(v)) for v in gg.values())
        check_image(img, g, pl, plan.params)
        ref = oracle.grad(g, pl, dimg, oracle_params(plan.params))
        print((chi2, tw, th), check_grads(gg, ref))


def _fd_oracle(g, X, dout, prm, h=1e-6):
    base = {k: np.array(getattr(g, k), dtype=np.float64) for k in ("means", "lraw", "intensity", "opacity")}
    out = {}
    for k in base:
        num = np.zeros_like(base[k])
        flat = num.reshape(-1)
        for j in range(flat.size):
            ap = {kk: vv.copy() for kk, vv in base.items()}
            am = {kk: vv.copy() for kk, vv in base.items()}
            x0 = ap[k].reshape(-1)[j]
            step = h * max(1.0, abs(x0))
            ap[k].reshape(-1)[j] += step
            am[k].reshape(-1)[j] -= step
            lp = oracle.render_points(synth.Gaussians(**ap), X, prm)[0] @ dout
            lm = oracle.render_points(synth.Gaussians(**am), X, prm)[0] @ dout
            flat[j] = (lp - lm) / (2 * step)
        out[k] = num
    return out


@pytest.mark.parametrize("chi2", [math.inf, 7.815])
def test_gradients_vs_fp64_finite_differences(R, chi2):
    rng = np.random.default_rng(7)
    for seed in range(60, 120):
        g = synth.make_gaussians(6, seed, (0.35, 0.35, 0.35), (0.65, 0.65, 0.65), (0.05, 0.18), opacity="random")
        pl = synth.random_planes(2, seed + 200, (20, 18), 0.025, 0.47, 0.53)
        X = oracle.plane_points(pl)
        d2 = oracle.d2_points(g, X)
        if math.isinf(chi2) or (np.min(np.abs(d2 - chi2)) > 2e-3 and np.any(d2 <= chi2)):
            break
    dimg = rng.standard_normal(X.shape[0]).astype(np.float32).astype(np.float64)
    _, gg, plan = _fwd_bwd(R, g, pl, dimg, R.Params(chi2=chi2, tile_w=8, tile_h=8))
    fd = _fd_oracle(g, X, dimg, oracle_params(plan.params))
    print("fd", check_grads(gg, fd))


@pytest.mark.parametrize("k,count", [(1, 400), (2, 200), (3, 150), (4, 150)])
def test_configs_sparse_upstream_gradient(R, k, count):
    """Full-size renders and adjoints in the library's default launch
    configuration and in the autotuner's stored pick (the configuration the
    benchmark times); d_image is non-zero on seeded pixels only, so the
    oracle's exact gradient needs just those pixels."""
    from tests.configs import launch_configs
    from tests.parity import reference_grad
    g, pl, _ = synth.make_config(k)
    pix = synth.sample_pixels(pl, count, 600 + k)
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    rng = np.random.default_rng(k)
    vals = rng.standard_normal(count).astype(np.float32)
    dimg = np.zeros(pl.npix, dtype=np.float32)
    dimg[flat] = vals
    ref = None
    for name, params in launch_configs(R, g, pl):
        _, gg, plan = _fwd_bwd(R, g, pl, dimg, params)
        if ref is None:
            ref = reference_grad(g, oracle.plane_points(pl, pix), vals.astype(np.float64), plan.params)
        print(f"c{k} {name} {params.tile_w}x{params.tile_h} batch {params.lds_batch} box {params.box_mode} grads",
              check_grads(gg, ref))


def test_run_to_run_bitwise_adjoint(R):
    """The adjoint is deterministic (no atomics; every sum in a fixed order):
    two backward passes of the 200k anisotropic workload in its tuned
    configuration, and the MSE-fused adjoint run twice, give the same
    gradients bit for bit."""
    from tests.configs import tuned_params
    g, pl, tg = synth.make_config(2)
    params = tuned_params(g, pl)
    dev = torch.device("cuda", 0)
    gd, pd, td = R.to_device(g, dev), R.to_device(pl, dev), R.to_device(tg, dev)
    tplan = R.Plan(tg.n, pl.wh, params, device=dev)
    tplan.fit(td, pd)
    target = tplan.render(td, pd).clone()
    del tplan
    plan = R.Plan(g.n, pl.wh, params, device=dev)
    plan.fit(gd, pd)
    img = plan.render(gd, pd)
    rng = np.random.default_rng(5)
    dimg = torch.from_numpy(rng.standard_normal(plan.num_pixels).astype(np.float32)).to(dev)
    a = [t.clone() for t in plan.backward(gd, pd, img, dimg)]
    b = [t.clone() for t in plan.backward(gd, pd, img, dimg)]
    c = [t.clone() for t in plan.backward_mse(gd, pd, img, target)]
    img2 = plan.render(gd, pd)
    d = [t.clone() for t in plan.backward_mse(gd, pd, img2, target)]
    torch.cuda.synchronize()
    assert torch.equal(img, img2)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    for x, y in zip(c, d):
        assert torch.equal(x, y)


def test_accumulate_flag_and_autograd(R):
    from paper_2505_05643_amd.autograd import render_planes
    g = synth.make_gaussians(120, 71, (0, 0, 0), (1, 1, 1), (0.03, 0.15), opacity="random")
    pl = synth.random_planes(2, 72, (30, 30), 1 / 30, 0.4, 0.6)
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    plan = R.Plan(g.n, pl.wh, device=dev)
    plan.fit(gd, pd)
    leaves = [t.clone().requires_grad_(True) for t in gd]
    img = render_planes(R.GaussianTensors(*leaves), pd, plan)
    w = torch.randn(img.shape, device=dev)
    (img * w).sum().backward()
    img2 = plan.render(gd, pd)
    assert torch.equal(img.detach(), img2)
    g1 = plan.backward(gd, pd, img2, w)
    for a, b in zip(leaves, g1):
        assert torch.equal(a.grad, b)
    plan.backward(gd, pd, img2, w, grads=g1, accumulate=True)
    for a, b in zip(leaves, g1):
        torch.testing.assert_close(b, 2 * a.grad, rtol=1e-6, atol=0)


def test_fused_mse_backward_equals_separate(R):
    """ug_render_planes_backward_mse: the gradients equal ug_mse_grad then
    ug_render_planes_backward bit for bit (tile shapes, aligned and unaligned
    arrays, ragged planes); the loss is the float64 mean squared error; with
    no Gaussians the loss is still written."""
    dev = torch.device("cuda", 0)
    g = synth.make_gaussians(400, 61, (0, 0, 0), (1, 1, 1), (0.03, 0.15), aniso_max=6.0, opacity="random")
    t = synth.make_gaussians(400, 62, (0, 0, 0), (1, 1, 1), (0.03, 0.15))
    pl = synth.random_planes(3, 63, (40, 33), 1 / 36, 0.35, 0.65)
    pl.wh[:] = [[41, 33], [8, 8], [57, 21]]
    gd, td, pd = R.to_device(g, dev), R.to_device(t, dev), R.to_device(pl, dev)
    for tile, off in (((16, 16), 0), ((16, 8), 1), ((32, 32), 0), ((8, 8), 3)):
        params = R.Params(tile_w=tile[0], tile_h=tile[1])
        tplan = R.Plan(t.n, pl.wh, params, device=dev)
        tplan.fit(td, pd)
        tgt_buf = torch.empty(tplan.num_pixels + off, device=dev)
        target = tgt_buf[off:]
        tplan.render(td, pd, target)
        plan = R.Plan(g.n, pl.wh, params, device=dev)
        plan.fit(gd, pd)
        img_buf = torch.empty(plan.num_pixels + off, device=dev)
        img = img_buf[off:]
        plan.render(gd, pd, img)
        d_image = torch.empty_like(img)
        loss_a = torch.zeros(1026, device=dev)
        R.mse_grad(img, target, d_image, loss_a)
        ga = plan.backward(gd, pd, img, d_image)
        loss_b = torch.full((4,), -1.0, device=dev)
        gb = plan.backward_mse(gd, pd, img, target, loss_buf=loss_b)
        torch.cuda.synchronize()
        for a, b in zip(ga, gb):
            assert torch.equal(a, b), (tile, off)
        ref = float(np.mean((img.cpu().numpy().astype(np.float64) - target.cpu().numpy()) ** 2))
        assert abs(float(loss_b[0]) - ref) <= 1e-6 * ref, (tile, off, float(loss_b[0]), ref)
        assert abs(float(loss_a[0]) - ref) <= 1e-6 * ref
        assert float(loss_b[1]) == -1.0  # only the first element is written
        # accumulate = 1 adds the same gradients again
        gc = plan.backward_mse(gd, pd, img, target, grads=R.GaussianTensors(*(x.clone() for x in gb)),
                               accumulate=True)
        for a, c in zip(gb, gc):
            assert torch.allclose(c, 2 * a, rtol=1e-6, atol=0)
    g0 = synth.make_gaussians(0, 1)
    g0d = R.to_device(g0, dev)
    plan = R.Plan(0, pl.wh, R.Params(), device=dev)
    img = plan.render(g0d, pd)
    target = torch.full_like(img, 0.25)
    loss = torch.full((1,), -1.0, device=dev)
    plan.backward_mse(g0d, pd, img, target, loss_buf=loss)
    ref = float(np.mean((img.cpu().numpy().astype(np.float64) - 0.25) ** 2))
    assert abs(float(loss[0]) - ref) <= 1e-6 * ref


def test_config4_training_pool_planes(R):
    """The 1M-Gaussian workload's training planes (8 interleaved oblique
    sweeps) in the launch configuration tuned for it: 16 seeded planes of the
    2,048-plane pool, a sample of pixels against the oracle and the gradient
    of a sparse upstream signal against the oracle's."""
    from tests.configs import tuned_params
    from tests.parity import check_image, reference_grad, reference_points
    g = synth.config_gaussians(4)
    pool = synth.config4_training_pool()
    params = tuned_params(g, synth.config_planes(4))
    sel = np.sort(np.random.default_rng(44).choice(pool.p, size=16, replace=False))
    pl = pool.subset(sel)
    pix = synth.sample_pixels(pl, 300, 644)
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    X = oracle.plane_points(pl, pix)
    vals = np.random.default_rng(45).standard_normal(pix.shape[0]).astype(np.float32)
    vals[150:] = 0.0  # the gradient of the first 150 sampled pixels
    dimg = np.zeros(pl.npix, dtype=np.float32)
    dimg[flat] = vals
    img, gg, plan = _fwd_bwd(R, g, pl, dimg, params)
    ref, _ = reference_points(g, X, plan.params)
    print("pool planes", sel.tolist(), check_image(img[flat], g, pl, plan.params, pix=pix, ref=ref))
    gref = reference_grad(g, X, vals.astype(np.float64), plan.params)
    print("pool planes grads", check_grads(gg, gref))


def test_config1_gradients_vs_fp64_finite_differences(R):
    """The 50k-Gaussian 16-plane sweep with its gradients checked against
    FP64 finite differences of the oracle, at full size and in the tuned
    launch configuration.  Twelve seeded Gaussians (footprints of at most
    2,000 pixels over all planes) each get one seeded raw parameter; the
    upstream gradient is non-zero on the pixels those Gaussians touch, minus
    every pixel with a borderline pair (|d^2 - chi^2| <= 2e-4: the FP32 and
    FP64 inclusion sets agree elsewhere).  A central difference of
    L = sum dout c_hat only needs the pixels the perturbed Gaussian touches
    (the others do not move); it is taken only where no pair of that
    Gaussian changes side of the cut-off between theta - h and theta + h."""
    from oracle import pool
    from tests.configs import tuned_params
    from tests.parity import oracle_params
    g, pl, _ = synth.make_config(1)
    params = tuned_params(g, pl)
    op = oracle_params(params)
    X = oracle.plane_points(pl)
    rng = np.random.default_rng(4101)
    chosen, touched = [], []
    for i in rng.permutation(g.n):
        d2 = oracle.d2_points(g.subset(np.array([i])), X, op)[:, 0]
        t = np.nonzero(d2 <= op.chi2 * 1.01)[0]
        if 50 <= t.size <= 2000:
            chosen.append(int(i))
            touched.append(t)
        if len(chosen) == 12:
            break
    S = np.unique(np.concatenate(touched))
    _, _, k = pool.ambiguity_points(g, X[S], op)
    S = S[k == 0]
    dimg = np.zeros(pl.npix, dtype=np.float32)
    dimg[S] = rng.standard_normal(S.size).astype(np.float32)
    _, gg, _ = _fwd_bwd(R, g, pl, dimg, params)
    base = {f: np.array(getattr(g, f), dtype=np.float64) for f in ("means", "lraw", "intensity", "opacity")}
    fields = [("means", j) for j in range(3)] + [("lraw", j) for j in range(6)] + [("intensity", None),
                                                                                  ("opacity", None)]
    # Gaussians that can reach a point: |x - mu| <= sqrt(chi^2) sigma_max
    # (d^2 >= |x - mu|^2 / sigma_max^2), so the others add exact zeros there
    sig_max = np.sqrt(np.linalg.eigvalsh(oracle.covariance(g.lraw, op.beta))[:, -1])
    reach = np.sqrt(op.chi2) * sig_max * 1.001 + 1e-9
    mu = np.asarray(g.means, dtype=np.float64)
    checked = 0
    for i, t in zip(chosen, touched):
        f, j = fields[int(rng.integers(len(fields)))]
        x0 = base[f][i] if j is None else base[f][i, j]
        h = 1e-6 * max(1.0, abs(x0))
        moved = []
        for sgn in (1.0, -1.0):
            a = {kk: vv.copy() for kk, vv in base.items()}
            if j is None:
                a[f][i] += sgn * h
            else:
                a[f][i, j] += sgn * h
            moved.append(synth.Gaussians(**a))
        d2p = oracle.d2_points(moved[0].subset(np.array([i])), X, op)[:, 0]
        d2m = oracle.d2_points(moved[1].subset(np.array([i])), X, op)[:, 0]
        if np.any((d2p <= op.chi2) != (d2m <= op.chi2)):
            continue  # a pair of this Gaussian crosses the cut-off within the step
        P = np.nonzero(((d2p <= op.chi2) | (d2m <= op.chi2)) & (dimg != 0))[0]
        lo, hi = X[P].min(axis=0), X[P].max(axis=0)
        gap = np.linalg.norm(np.maximum(np.maximum(lo - mu, mu - hi), 0.0), axis=1)
        near = np.nonzero(gap <= reach)[0]
        assert i in near
        lp = oracle.render_points(moved[0].subset(near), X[P], op)[0] @ dimg[P].astype(np.float64)
        lm = oracle.render_points(moved[1].subset(near), X[P], op)[0] @ dimg[P].astype(np.float64)
        fd = (lp - lm) / (2 * h)
        got = gg[f][i] if j is None else gg[f][i, j]
        scale = float(np.abs(gg[f]).max())
        assert abs(got - fd) <= 1e-3 * abs(fd) + 1e-5 * scale, (i, f, j, got, fd, scale)
        checked += 1
    assert checked >= 8, f"only {checked} parameters were free of cut-off crossings"
    print(f"c1 finite differences: {checked} parameters, {S.size} upstream pixels")
