"""Host logic of the benchmark (no GPU): the stored HBM traffic is reported
only for the workload, launch configuration and kernel sources it was
measured with."""
import types

import bench


def _params(tw=16, th=32, ppl=2, batch=64, box=2, flags=0):
    return types.SimpleNamespace(tile_w=tw, tile_h=th, px_per_lane=ppl, lds_batch=batch, box_mode=box, flags=flags)


def test_stored_traffic_follows_the_committed_counters(monkeypatch):
    rec = bench.stored_traffic("accum_bwd", 1, _params(), None)
    assert rec is None or rec > 0
    # another launch configuration or workload has no stored figure
    assert bench.stored_traffic("accum_bwd", 1, _params(box=0), None) is None
    assert bench.stored_traffic("accum_bwd", 1, _params(flags=8), None) is None  # the split forward
    assert bench.stored_traffic("accum_bwd", 4, _params(), None) is None
    # any change to the kernel sources voids every stored figure
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 16)
    assert bench.stored_traffic("accum_bwd", 1, _params(), None) is None


def test_sources_digest_is_stable_and_covers_the_kernels():
    a = bench.sources_digest()
    assert a == bench.sources_digest() and len(a) == 16


def test_plan_ppl_default():
    assert bench.plan_ppl(_params(ppl=0, tw=32)) == 4
    assert bench.plan_ppl(_params(ppl=2)) == 2


def test_stored_traffic_is_calibrated_on_the_copy_probe():
    """The committed counter summaries scale FETCH_SIZE and WRITE_SIZE by what
    the same counters read for a plain copy of known size; on this GPU that is
    about 2 and 1.  A summary calibrated on some other kernel would carry
    factors thousands of times larger and per-launch bytes beyond any HBM."""
    import json
    for k in (1, 4):
        with open(bench.traffic_file(k)) as f:
            line = next(ln for ln in f if ln.startswith("traffic-json: "))
        rec = json.loads(line[len("traffic-json: "):])
        assert 1.5 < rec["fetch_scale"] < 2.5 and 0.75 < rec["write_scale"] < 1.5, rec
        assert rec["bytes_per_launch"] and max(rec["bytes_per_launch"].values()) < 64e9


def test_cull_group_rule():
    """The benchmark's restatement of when the Phase-1 cull searches plane
    groups: planes sharing the normal row of R^-1 and the origin's x and y,
    eight or more of them, at most 256 planes, one lane per Gaussian, and
    the per-plane flag unset."""
    import numpy as np
    from paper_2505_05643_amd import synth
    from paper_2505_05643_amd._lib import UG_FLAG_CULL_EACH_PLANE
    p4 = synth.config_planes(4)
    assert bench.cull_searches_groups(p4, _params(flags=0), 1_000_000)
    assert not bench.cull_searches_groups(p4, _params(flags=UG_FLAG_CULL_EACH_PLANE), 1_000_000)
    assert not bench.cull_searches_groups(p4, _params(flags=0), 50_000)  # several lanes per Gaussian
    for k in (0, 1, 2, 3):
        assert not bench.cull_searches_groups(synth.config_planes(k), _params(flags=0), 1_000_000)
    # same normal, in-plane rotations differing: still one group
    frames = [synth.frame_from_normal((0.0, 0.0, 1.0), a) for a in np.linspace(0.0, 3.0, 10)]
    pl = synth.pack_planes(frames, [(0.5, 0.5, z) for z in np.linspace(0.1, 0.9, 10)], [(0.01, 0.01)] * 10,
                           [(32, 32)] * 10)
    assert bench.cull_searches_groups(pl, _params(flags=0), 1_000_000)
    # origins differing in x: no group
    pl.origin[:, 0] = np.linspace(0.1, 0.9, 10)
    assert not bench.cull_searches_groups(pl, _params(flags=0), 1_000_000)
