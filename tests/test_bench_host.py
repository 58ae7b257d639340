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
