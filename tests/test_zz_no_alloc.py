"""The forward that allocates nothing (ug_render_planes_noalloc): through the
C ABI it must give the image of ug_render_planes on the same plan and
inputs, bit for bit (same kernels, same workspace layout, only the
workspace's address differs), on two calls in a row with the second on a
smaller input, and it must refuse a plan whose workspace exceeds its static
array, enqueueing nothing."""
import ctypes

import numpy as np
import pytest

from paper_2505_05643_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05643_amd import raster
    return raster


def _pair(R, g, pl, params):
    """(image from ug_render_planes, image from ug_render_planes_noalloc)."""
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    plan = R.Plan(g.n, pl.wh, params, device=dev)
    plan.fit(gd, pd)
    assert plan.workspace_bytes <= R._lib.UG_NOALLOC_WORKSPACE_BYTES
    ref = plan.render(gd, pd)
    assert plan.status() == 0
    out = torch.full_like(ref, float("nan"))
    plan.render_noalloc(gd, pd, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_forward_equals_render_two_calls_second_smaller(R):
    # first call: 1,000 Gaussians on four 128^2 planes (several tiles per
    # plane, a ragged last plane); second: fewer Gaussians, fewer and smaller
    # planes, another tile shape -- the static workspace keeps the first
    # call's contents, which the second must not read
    g1 = synth.make_gaussians(1000, 71, (0, 0, 0), (1, 1, 1), (0.005, 0.05), opacity="random")
    pl1 = synth.random_planes(4, 72, (128, 128), 1 / 128, 0.25, 0.75)
    pl1.wh[3] = [97, 61]
    g2 = synth.make_gaussians(150, 73, (0, 0, 0), (1, 1, 1), (0.01, 0.08), opacity="random")
    pl2 = synth.random_planes(2, 74, (40, 24), 1 / 40, 0.3, 0.7)
    for g, pl, params in ((g1, pl1, R.Params()), (g2, pl2, R.Params(tile_w=32, tile_h=16, box_mode=1))):
        ref, out = _pair(R, g, pl, params)
        assert np.all(np.isfinite(out))
        assert np.array_equal(ref.view(np.uint32), out.view(np.uint32)), (
            f"noalloc image differs at {np.count_nonzero(ref != out)} pixels (max {np.abs(ref - out).max():.3e})")


def test_noalloc_rejects_workspace_beyond_static_array(R):
    g = synth.make_gaussians(100, 75, (0, 0, 0), (1, 1, 1), (0.01, 0.05))
    pl = synth.random_planes(2, 76, (32, 32), 1 / 32, 0.4, 0.6)
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    plan = R.Plan(g.n, pl.wh, R.Params(), device=dev)
    # key capacity alone past the limit: 56 bytes of workspace per key
    plan.reserve(1024, (R._lib.UG_NOALLOC_WORKSPACE_BYTES // 56) + 1024)
    assert plan.workspace_bytes > R._lib.UG_NOALLOC_WORKSPACE_BYTES
    img = torch.full((plan.num_pixels,), 7.0, device=dev)
    code = R._lib.lib.ug_render_planes_noalloc(plan._h, ctypes.byref(R._c_gauss(gd)), ctypes.byref(R._c_planes(pd)),
                                               img.data_ptr(), R._stream())
    assert code == R._lib.UG_ERR_SCRATCH_SIZE
    torch.cuda.synchronize()
    assert bool((img == 7.0).all()), "a refused call must enqueue nothing"
