"""Image-quality scores (ug_image_quality) against the SSIM / PSNR
reference, and the synthetic reconstruction workload end to end."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_05643_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SSIM_TOL = 1e-9   # both sides sum float64 moments of the same float32 pixels
MSE_TOL = 1e-9    # relative


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05643_amd import raster
    return raster


def _check(R, wh, tile, img, ref, data_range=1.0):
    dev = torch.device("cuda", 0)
    plan = R.Plan(1, wh, R.Params(tile_w=tile[0], tile_h=tile[1]), device=dev)
    a = torch.from_numpy(img.astype(np.float32)).to(dev)
    b = torch.from_numpy(ref.astype(np.float32)).to(dev)
    s, m = plan.quality(a, b, data_range)
    s2, m2 = plan.quality(a, b, data_range)
    assert torch.equal(s, s2) or bool(torch.all(torch.isnan(s) == torch.isnan(s2)))
    assert torch.equal(m, m2)
    s, m = s.cpu().numpy(), m.cpu().numpy()
    rs, rm = oracle.quality.quality(img.astype(np.float32), ref.astype(np.float32), wh, data_range)
    assert np.array_equal(np.isnan(s), np.isnan(rs))
    ok = ~np.isnan(rs)
    assert np.max(np.abs(s[ok] - rs[ok])) <= SSIM_TOL, (s, rs)
    np.testing.assert_allclose(m, rm, rtol=MSE_TOL, atol=0)
    return s, m


@pytest.mark.parametrize("tile", [(8, 8), (16, 32), (32, 32)])
def test_quality_matches_reference_ragged(R, tile):
    """Ragged planes (one too narrow for a window, one exactly 11 x 11),
    every tile shape: per-plane SSIM and MSE against the float64 reference;
    two calls agree bit for bit."""
    wh = np.array([[37, 23], [8, 30], [11, 11], [64, 40], [161, 19]], dtype=np.int32)
    rng = np.random.default_rng(11)
    npx = int(np.sum(wh[:, 0] * wh[:, 1]))
    img = rng.random(npx)
    ref = np.clip(img + 0.15 * rng.standard_normal(npx), 0, 1)
    s, m = _check(R, wh, tile, img, ref)
    assert math.isnan(s[1]) and np.all(np.isfinite(s[[0, 2, 3, 4]]))
    _check(R, wh, tile, img, 2.0 * ref, data_range=2.0)
    # identical images: SSIM 1 and MSE 0
    s, m = _check(R, wh, tile, img, img)
    assert np.all(np.abs(s[[0, 2, 3, 4]] - 1.0) <= 1e-12) and np.all(m == 0.0)


def test_quality_on_rendered_slices(R):
    """Rendered slices of two different seeded volumes (smooth images with
    flat background, where E[x^2] - mu^2 cancels most)."""
    from paper_2505_05643_amd import recon
    setup = recon.ReconSetup(size=64, n_truth=3000)
    dev = torch.device("cuda", 0)
    pl = recon.eval_planes(setup)
    pd = R.to_device(pl, dev)
    imgs = []
    for seed in (0, 1):
        g = R.to_device(recon.truth_gaussians(recon.ReconSetup(**{**setup.__dict__, "seed": seed})), dev)
        plan = R.Plan(g.means.shape[0], pl.wh, R.Params(), device=dev)
        plan.fit(g, pd)
        imgs.append(plan.render(g, pd).cpu().numpy())
    _check(R, pl.wh, (16, 16), imgs[0], imgs[1])


def test_reconstruction_small(R):
    """A small full-coverage and a jittered half-coverage fit: the scores on
    all three views (coronal and sagittal never seen) rise from the
    initialisation, the loss falls, and the scores the workload reports are
    the reference's on the same images."""
    from paper_2505_05643_amd import recon
    setup = recon.ReconSetup(size=48, n_truth=3000, n_model=6000, steps=150, check_every=50)
    dev = torch.device("cuda", 0)
    truth = R.to_device(recon.truth_gaussians(setup), dev)
    scorer = recon.Scorer(setup, truth, R.Params(), dev)
    for case in ("full", "half_jitter"):
        out = recon.run_case(setup, case, dev, scorer=scorer)
        print(case, {k: out[k] for k in ("train_slices", "ms_per_step", "loss_first_check", "loss_last")},
              "init", out["init"], "trained", out["trained"])
        assert out["loss_last"] < 0.5 * out["loss_first_check"]
        for v in recon.VIEWS:
            assert out["trained"]["psnr"][v] > out["init"]["psnr"][v] + 3.0, (case, v)
            assert out["trained"]["ssim"][v] > out["init"]["ssim"][v] + 0.05, (case, v)
    # the workload's scores are the reference's on the images it scored
    model = R.to_device(synth.paper_init(setup.n_model, 7), dev)
    img = scorer.images(model).cpu().numpy()
    got = scorer.score(model)
    rs, rm = oracle.quality.quality(img, scorer.truth_images.cpu().numpy(), scorer.wh, 1.0)
    for k, v in enumerate(recon.VIEWS):
        sl = slice(k * setup.size, (k + 1) * setup.size)
        assert abs(got["ssim"][v] - float(np.mean(rs[sl]))) <= 1e-9
        assert abs(got["psnr"][v] - float(np.mean(10 * np.log10(1.0 / rm[sl])))) <= 1e-6
