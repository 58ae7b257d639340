"""The autotuner on a small workload: every candidate is timed and checked
(images, workload gradients and the cut-off-free probe's gradients against
the first tile shape's) and the pick is one of the candidates."""
import numpy as np
import pytest

from paper_2505_05643_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tune_checks_every_candidate():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05643_amd import autotune
    from paper_2505_05643_amd import raster as R
    dev = torch.device("cuda", 0)
    g = synth.make_gaussians(3000, 61, (0, 0, 0), (1, 1, 1), (0.005, 0.05), opacity="random")
    pl = synth.random_planes(3, 62, (96, 80), 1 / 96, 0.3, 0.7)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    shapes = ((8, 8, 1), (16, 16, 2), (32, 32, 4), (16, 32, 2))
    params, results = autotune.tune(gd, pd, pl.wh, steps=2, shapes=shapes, batches=(64, 128))
    assert len(results) == len(shapes) * len(autotune.BOXES) + 3 + 3  # + batches and splits of the best three
    assert sum(r["split_forward"] for r in results) == 3
    picked = (params.tile_w, params.tile_h, params.px_per_lane, params.lds_batch, params.box_mode,
              bool(params.flags & R._lib.UG_FLAG_SPLIT_FORWARD))
    assert picked in {(r["tile_w"], r["tile_h"], r["px_per_lane"], r["lds_batch"], r["box_mode"], r["split_forward"])
                      for r in results}
    for r in results:
        assert r["ms"] > 0
        for name, e in r["grad_vs_first_shape"].items():
            assert e["probe_max_by_largest"] <= autotune.GRAD_REL, (r, name)
            assert e["workload_normwise"] <= autotune.GRAD_REL_WORKLOAD, (r, name)
    # the first shape's candidates compare with themselves: exact
    first = [r for r in results if (r["tile_w"], r["tile_h"]) == shapes[0][:2] and not r["split_forward"]]
    assert all(e["probe_max_by_largest"] == 0.0 for r in first for e in r["grad_vs_first_shape"].values())
    assert np.isfinite([r["ms"] for r in results]).all()
