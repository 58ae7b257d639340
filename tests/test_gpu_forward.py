"""Forward parity: HIP render vs the FP64 oracle, element by element."""
import math

import numpy as np
import pytest

from paper_2505_05643_amd import synth
from tests.parity import check_image

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05643_amd import raster
    return raster


def _render(R, g, pl, params=None, fit=True):
    params = params or R.Params()
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    plan = R.Plan(g.n, pl.wh, params, device=dev)
    if fit:
        plan.fit(gd, pd)
    img = plan.render(gd, pd)
    torch.cuda.synchronize()
    return img.cpu().numpy(), plan


def test_config0_full_image(R):
    g, pl, _ = synth.make_config(0)
    img, plan = _render(R, g, pl)
    st = check_image(img, g, pl, plan.params)
    print("c0", st)


def test_small_ragged_planes_several_tiles(R):
    g = synth.make_gaussians(300, 41, (0, 0, 0), (1, 1, 1), (0.02, 0.12), opacity="random")
    pl = synth.random_planes(3, 42, (8, 8), 1 / 40, 0.3, 0.7)
    pl.wh[:] = [[37, 23], [8, 8], [50, 41]]
    for bm in (0, 1, 2):
        img, plan = _render(R, g, pl, R.Params(box_mode=bm))
        check_image(img, g, pl, plan.params)


def test_no_gaussians_is_background(R):
    g = synth.make_gaussians(0, 1)
    pl = synth.random_planes(2, 3, (20, 12), 0.05)
    params = R.Params(bg_color=0.25)
    img, _ = _render(R, g, pl, params, fit=False)
    assert np.all(img == np.float32(0.25))


def test_chi2_infinite_and_bright_background(R):
    g = synth.make_gaussians(40, 5, (0.3, 0.3, 0.3), (0.7, 0.7, 0.7), (0.05, 0.2), opacity="random")
    pl = synth.random_planes(2, 6, (24, 20), 1 / 24, 0.45, 0.55)
    for params in (R.Params(chi2=math.inf), R.Params(bg_alpha=1.0, bg_color=0.5)):
        img, plan = _render(R, g, pl, params)
        check_image(img, g, pl, plan.params)


def test_one_pixel_planes_and_far_planes(R):
    g = synth.make_gaussians(64, 7, (0, 0, 0), (1, 1, 1), (0.05, 0.3))
    pl = synth.pack_planes([np.eye(3), synth.axis_angle((1, 1, 0), 0.4), np.eye(3)],
                           [(0.5, 0.5, 0.5), (0.4, 0.6, 0.5), (10.0, 10.0, 10.0)],
                           [(0.1, 0.1), (0.02, 0.05), (0.1, 0.1)], [(1, 1), (3, 70), (16, 16)])
    img, plan = _render(R, g, pl)
    check_image(img, g, pl, plan.params)
    assert np.all(img[-256:] == 0.0)  # the far plane sees background only


def test_in_plane_rotation_gives_rot90(R):
    """Rotating a plane's in-plane axes by 90 degrees about its normal
    (e1' = e2, e2' = -e1) on a centred square grid samples the same 3D
    points, so the image rotates: image'[v, u] = image[u, W-1-v], which is
    numpy's rot90.  Both renders are also checked against the oracle; the
    two may differ by more than the tolerance only where a pair sits on the
    cut-off (rare)."""
    g = synth.make_gaussians(400, 51, (0.2, 0.2, 0.2), (0.8, 0.8, 0.8), (0.02, 0.1), opacity="random")
    base = synth.axis_angle((1, 2, 3), 0.7)
    e1, e2, n = base[:, 0], base[:, 1], base[:, 2]
    turned = np.stack([e2, -e1, n], axis=1)
    W = 48
    pl = synth.pack_planes([base, turned], [(0.5, 0.5, 0.5)] * 2, [(1 / W, 1 / W)] * 2, [(W, W)] * 2)
    assert np.array_equal(pl.rot[1].reshape(3, 3)[:, 0], pl.rot[0].reshape(3, 3)[:, 1])  # exact in float32
    for bm in (0, 1, 2):
        img, plan = _render(R, g, pl, R.Params(box_mode=bm))
        st = check_image(img, g, pl, plan.params)
        a, b = img[:W * W].reshape(W, W), img[W * W:].reshape(W, W)
        diff = np.abs(b.astype(np.float64) - np.rot90(a).astype(np.float64))
        off = int(np.sum(diff > 2e-4 * st["peak"]))
        assert off <= max(1, 1e-3 * W * W), f"box {bm}: {off} pixels differ from rot90"
        print("rot90 box", bm, "max diff / peak", float(diff.max() / st["peak"]), "off", off)


def test_paper_phase2_atomic_scatter(R):
    """UG_FLAG_SCATTER, the paper's Phase 2: each record adds to per-pixel
    sums with atomic adds over its box.  Same per-pair test as the gather,
    so the oracle's image within the parity tolerance and the gather's to
    float rounding (pairs on the cut-off aside); such plans refuse the
    backward."""
    from paper_2505_05643_amd._lib import UG_FLAG_SCATTER, UgError
    cases = [synth.make_config(0)[:2]]
    g1 = synth.make_gaussians(300, 41, (0, 0, 0), (1, 1, 1), (0.02, 0.12), opacity="random")
    p1 = synth.random_planes(3, 42, (8, 8), 1 / 40, 0.3, 0.7)
    p1.wh[:] = [[37, 23], [8, 8], [50, 41]]
    cases.append((g1, p1))
    for g, pl in cases:
        for bm in (0, 1, 2):
            img_s, plan_s = _render(R, g, pl, R.Params(box_mode=bm, flags=UG_FLAG_SCATTER))
            st = check_image(img_s, g, pl, plan_s.params)
            img_g, _ = _render(R, g, pl, R.Params(box_mode=bm))
            diff = np.abs(img_s.astype(np.float64) - img_g.astype(np.float64))
            off = int(np.sum(diff > 2e-5 * st["peak"]))
            assert off <= max(1, 1e-3 * img_s.size), f"box {bm}: {off} pixels differ from the gather"
    g, pl = cases[1]
    img, plan = _render(R, g, pl, R.Params(chi2=math.inf, flags=UG_FLAG_SCATTER))
    check_image(img, g, pl, plan.params)
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    with pytest.raises(UgError):
        plan.backward(gd, pd, torch.from_numpy(img).to(dev), torch.zeros(plan.num_pixels, device=dev))


def test_tile_shapes_box_modes_batches(R):
    """Within one tile shape, every LDS batch and binning box gives the same
    image bit for bit (each pixel sums its in-support Gaussians in record
    order; a binned pair outside the support adds exactly zero, and the
    sub-block masks do not depend on the box).  Across tile shapes only the
    tile-relative coordinates round differently."""
    g = synth.make_gaussians(500, 43, (0, 0, 0), (1, 1, 1), (0.02, 0.12), aniso_max=8.0, opacity="random")
    pl = synth.random_planes(3, 44, (8, 8), 1 / 48, 0.35, 0.65)
    pl.wh[:] = [[61, 47], [32, 32], [48, 17]]
    base, plan = _render(R, g, pl)
    check_image(base, g, pl, plan.params)
    shapes = {(8, 8): (0, 1), (16, 8): (2,), (8, 16): (1,), (16, 16): (0,), (32, 8): (4,), (32, 16): (4,),
              (16, 32): (2,), (32, 32): (0,)}
    for (tw, th), ppls in shapes.items():
        first = None
        for ppl in ppls:
            for bg in (32, 64, 128, 256):
                for bm in (0, 1, 2):
                    if bm != 0 and bg != 64:
                        continue
                    img, _ = _render(R, g, pl, R.Params(tile_w=tw, tile_h=th, px_per_lane=ppl, lds_batch=bg,
                                                        box_mode=bm))
                    if first is None:
                        first = img
                        check_image(img, g, pl, R.Params(tile_w=tw, tile_h=th))
                    assert np.array_equal(img, first), (tw, th, ppl, bg, bm)


@pytest.mark.parametrize("k,count", [(1, 1500), (2, 800), (3, 600), (4, 600)])
def test_configs_sampled_pixels(R, k, count):
    """Full-size workloads in the library's default launch configuration and
    in the autotuner's stored pick (the one the benchmark times); the oracle
    evaluates a seeded sample of pixels against every Gaussian."""
    from tests.configs import launch_configs
    from tests.parity import reference_points
    import oracle
    g, pl, _ = synth.make_config(k)
    pix = synth.sample_pixels(pl, count, 500 + k)
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    ref = None
    for name, params in launch_configs(R, g, pl):
        img, plan = _render(R, g, pl, params)
        if ref is None:
            ref, _ = reference_points(g, oracle.plane_points(pl, pix), plan.params)
        st = check_image(img[flat], g, pl, plan.params, pix=pix, ref=ref)
        print(f"c{k} {name} {params.tile_w}x{params.tile_h} batch {params.lds_batch} box {params.box_mode}", st,
              "records/keys", plan.status(counts=True))


def test_run_to_run_bitwise_forward(R):
    """The gather forward is deterministic: two renders of the 200k
    anisotropic workload (tuned configuration), and a render by a second
    plan, give the same image bit for bit."""
    from tests.configs import tuned_params
    g, pl, _ = synth.make_config(2)
    params = tuned_params(g, pl)
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    plan = R.Plan(g.n, pl.wh, params, device=dev)
    plan.fit(gd, pd)
    a = plan.render(gd, pd).clone()
    b = plan.render(gd, pd).clone()
    plan2 = R.Plan(g.n, pl.wh, params, device=dev)
    plan2.fit(gd, pd, headroom=2.0)
    c = plan2.render(gd, pd)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_binning_keys_and_ranges(R):
    """Sections 4.3-4.4 binning, checked from the sorted keys (debug hook):
    the emission positions are a permutation; keys are emitted record by
    record; numpy's stable argsort of the emitted tile ids gives exactly the
    sorted order; the tile ranges are the first key of each tile; every key's
    tile lies in its record's tile rectangle.  Independently of the GPU,
    every (Gaussian, pixel) pair inside the Eq. 12 support (FP64 oracle
    distance, with a 1e-4 relative margin below chi^2) has a record, a key
    for the pixel's tile and that key's sub-block bit set."""
    import oracle
    from tests.parity import oracle_params
    g = synth.make_gaussians(400, 81, (0, 0, 0), (1, 1, 1), (0.02, 0.12), aniso_max=8.0, opacity="random")
    pl = synth.random_planes(3, 82, (8, 8), 1 / 48, 0.35, 0.65)
    pl.wh[:] = [[61, 47], [32, 32], [48, 17]]
    for tw, th in ((16, 16), (32, 32), (8, 8), (16, 32)):
        for bm in (0, 1, 2):
            params = R.Params(tile_w=tw, tile_h=th, box_mode=bm)
            img, plan = _render(R, g, pl, params)
            key, eidx, rec, ranges = plan.debug_keys()
            recs = plan.debug_records()
            n = key.size
            q = (tw // 8) * (th // 8)
            shift = 32 - q
            tile = (key & np.uint32((1 << shift) - 1)).astype(np.int64)
            mask = (key >> np.uint32(shift)).astype(np.int64)
            assert np.array_equal(np.sort(eidx), np.arange(n, dtype=np.uint32))
            emitted_tile = np.empty(n, dtype=np.int64)
            emitted_rec = np.empty(n, dtype=np.int64)
            emitted_tile[eidx] = tile
            emitted_rec[eidx] = rec
            assert np.all(np.diff(emitted_rec) >= 0), "keys are emitted record by record"
            assert np.array_equal(np.argsort(emitted_tile, kind="stable"), eidx.astype(np.int64))
            assert np.all(np.diff(tile) >= 0)
            T = plan.num_tiles
            assert np.array_equal(ranges.astype(np.int64), np.searchsorted(tile, np.arange(T + 1), side="left"))
            # tile rectangle of each key's record
            tile_off = np.concatenate([[0], np.cumsum(-(-pl.wh[:, 0] // tw) * -(-pl.wh[:, 1] // th))])
            ntx = -(-pl.wh[:, 0] // tw)
            r = recs[rec]
            lt = tile - tile_off[r["plane"]]
            tx, ty = lt % ntx[r["plane"]], lt // ntx[r["plane"]]
            assert np.all((tx >= r["tx0"]) & (tx <= r["tx1"]) & (ty >= r["ty0"]) & (ty <= r["ty1"]))
            # coverage of the FP64 support
            op = oracle_params(plan.params)
            rec_of = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(recs["gaussian"], recs["plane"]))}
            keyset = {}
            for j in range(n):
                keyset[(int(rec[j]), int(tile[j]))] = int(mask[j])
            for p in range(pl.p):
                W, H = (int(x) for x in pl.wh[p])
                uu, vv = np.meshgrid(np.arange(W), np.arange(H))
                pix = np.stack([np.full(W * H, p), uu.ravel(), vv.ravel()], axis=1)
                d2 = oracle.d2_points(g, oracle.plane_points(pl, pix), op)
                inside = np.argwhere(d2 <= op.chi2 * (1 - 1e-4))
                for pi, gi in inside:
                    u, v = int(pix[pi, 1]), int(pix[pi, 2])
                    ri = rec_of.get((int(gi), p))
                    assert ri is not None, f"pair (g{gi}, plane {p}) in support has no record"
                    t = int(tile_off[p]) + (v // th) * int(ntx[p]) + u // tw
                    m = keyset.get((ri, t))
                    assert m is not None, f"record {ri} has no key for tile {t} at pixel ({u}, {v})"
                    b = ((v % th) // 8) * (tw // 8) + (u % tw) // 8
                    assert (m >> b) & 1, f"record {ri} tile {t}: sub-block {b} of pixel ({u}, {v}) not marked"
            print((tw, th, bm), "keys", n, "records", len(recs))


def test_cull_plane_groups_equal_per_plane_cull(R):
    """Planes that differ only in the origin's third coordinate are culled by
    searching each group for the window of planes the pre-test can accept;
    the records, the sorted keys and the image equal those of the per-plane
    cull (UG_FLAG_CULL_EACH_PLANE) bit for bit.  Planes: an axial stack in
    shuffled order with repeated heights, a tilted stack (one rotation and
    origin x, y; heights varied), a stack of one normal turned to different
    in-plane angles, and single oblique planes; with a cut-off
    in both box modes and without one.  The grouped image is also checked
    against the oracle on sampled pixels."""
    from tests.parity import reference_points
    import oracle
    g = synth.make_gaussians(3000, 95, (0, 0, 0), (1, 1, 1), (0.005, 0.05), aniso_max=6.0, opacity="random")
    rng = np.random.default_rng(96)
    frames, origins = [], []
    for zz in rng.permutation(np.concatenate([np.linspace(0.02, 0.98, 40), [0.5, 0.5, 0.25]])):
        frames.append(np.eye(3))
        origins.append((0.5, 0.5, zz))
    tilt = synth.axis_angle((1.0, 0.3, 0.0), 0.5)
    for zz in rng.uniform(0.1, 0.9, 20):
        frames.append(tilt)
        origins.append((0.45, 0.55, zz))
    for zz, ang in zip(rng.uniform(0.1, 0.9, 12), np.linspace(0.1, 3.0, 12)):  # one normal, turned in-plane
        frames.append(synth.frame_from_normal((0.0, 0.0, 1.0), ang))
        origins.append((0.52, 0.48, zz))
    for _ in range(5):
        frames.append(synth.axis_angle(rng.standard_normal(3), rng.uniform(0.2, 3.0)))
        origins.append(rng.uniform(0.3, 0.7, 3))
    P = len(frames)
    pl = synth.pack_planes(frames, origins, [(1 / 48, 1 / 48)] * P, [(48, 48)] * P)
    each = R._lib.UG_FLAG_CULL_EACH_PLANE
    for kw in (dict(box_mode=1), dict(box_mode=2), dict(box_mode=1, chi2=math.inf)):
        img_g, plan_g = _render(R, g, pl, R.Params(**kw))
        img_e, plan_e = _render(R, g, pl, R.Params(flags=each, **kw))
        rg, re_ = plan_g.debug_records(), plan_e.debug_records()
        assert rg.size == re_.size and rg.tobytes() == re_.tobytes()
        for a, b in zip(plan_g.debug_keys(), plan_e.debug_keys()):
            assert np.array_equal(a, b)
        assert np.array_equal(img_g.view(np.uint32), img_e.view(np.uint32))
        print(kw, "records", rg.size)
        if kw.get("chi2") is None:
            pix = synth.sample_pixels(pl, 1500, 97)
            offs = pl.pixel_offsets()
            flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
            ref, _ = reference_points(g, oracle.plane_points(pl, pix), plan_g.params)
            check_image(img_g[flat], g, pl, plan_g.params, pix=pix, ref=ref)


def test_emission_layout_small_and_whole_plane_records(R):
    """Key emission for rounds of 256 records of a few keys each (512 small
    Gaussians) and rounds of tens of thousands (256 that cover the whole
    plane): the keys are laid out record by record, each record's tiles
    row-major inside its tile rectangle (all of it for conic boxes), the
    sort is numpy's stable argsort, and the image matches the oracle."""
    small = synth.make_gaussians(512, 91, (0.05, 0.05, 0.49), (0.95, 0.95, 0.51), (0.004, 0.01), opacity="random")
    big = synth.make_gaussians(256, 92, (0.4, 0.4, 0.45), (0.6, 0.6, 0.55), (0.2, 0.3), opacity="random")
    g = synth.Gaussians(*(np.concatenate([getattr(small, f), getattr(big, f)])
                          for f in ("means", "lraw", "intensity", "opacity")))
    pl = synth.pack_planes([np.eye(3)], [(0.5, 0.5, 0.5)], [(1 / 96, 1 / 96)], [(96, 96)])
    for bm in (1, 2):
        params = R.Params(tile_w=8, tile_h=8, box_mode=bm)
        img, plan = _render(R, g, pl, params)
        check_image(img, g, pl, plan.params)
        key, eidx, rec, _ = plan.debug_keys()
        recs = plan.debug_records()
        n = key.size
        tile = (key & np.uint32((1 << 31) - 1)).astype(np.int64)
        emitted_tile = np.empty(n, dtype=np.int64)
        emitted_rec = np.empty(n, dtype=np.int64)
        emitted_tile[eidx] = tile
        emitted_rec[eidx] = rec
        assert np.array_equal(np.sort(eidx), np.arange(n, dtype=np.uint32))
        assert np.all(np.diff(emitted_rec) >= 0), "keys are emitted record by record"
        assert np.array_equal(np.argsort(emitted_tile, kind="stable"), eidx.astype(np.int64))
        # within a record: its tiles in row-major order inside its rectangle
        r = recs[emitted_rec]
        tx, ty = emitted_tile % 12, emitted_tile // 12
        assert np.all((tx >= r["tx0"]) & (tx <= r["tx1"]) & (ty >= r["ty0"]) & (ty <= r["ty1"]))
        same = emitted_rec[1:] == emitted_rec[:-1]
        assert np.all(emitted_tile[1:][same] > emitted_tile[:-1][same])
        if bm == 1:  # conic boxes: every tile of the rectangle
            area = (recs["tx1"].astype(np.int64) - recs["tx0"] + 1) * (recs["ty1"].astype(np.int64) - recs["ty0"] + 1)
            assert np.array_equal(np.bincount(emitted_rec, minlength=len(recs)), area)
        per_round = np.bincount(emitted_rec // 256)
        assert per_round.max() > 16 * 256 and per_round.min() < 4 * 256, per_round
        print("box", bm, "keys per round of 256 records", per_round)


@pytest.mark.parametrize("k,count", [(1, 1500), (4, 300)])
def test_configs_sampled_pixels_phase2_scatter(R, k, count):
    """The Phase-2 atomic scatter on full-size workloads: a seeded sample of
    pixels against the oracle."""
    from paper_2505_05643_amd._lib import UG_FLAG_SCATTER
    g, pl, _ = synth.make_config(k)
    img, plan = _render(R, g, pl, R.Params(flags=UG_FLAG_SCATTER))
    pix = synth.sample_pixels(pl, count, 700 + k)
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    st = check_image(img[flat], g, pl, plan.params, pix=pix)
    print(f"scatter c{k}", st)


def test_paper_phase2_box_support(R):
    """UG_FLAG_SCATTER | UG_FLAG_BOX_SUPPORT, the paper-literal Phase 2:
    every pixel whose centre lies in a kept pair's Eq. 13 box takes the Eq. 8
    weight.  Parity with the box-support reference; the image departs from
    the ellipsoid support (box corners count); with chi^2 = inf both supports
    are the plain sum; the flag needs the scatter; no backward."""
    from paper_2505_05643_amd._lib import UG_FLAG_BOX_SUPPORT, UG_FLAG_SCATTER, UgError
    from tests.parity import check_image_box_support
    fl = UG_FLAG_SCATTER | UG_FLAG_BOX_SUPPORT
    cases = [synth.make_config(0)[:2]]
    g1 = synth.make_gaussians(300, 41, (0, 0, 0), (1, 1, 1), (0.02, 0.12), aniso_max=8.0, opacity="random")
    p1 = synth.random_planes(3, 42, (8, 8), 1 / 40, 0.3, 0.7)
    p1.wh[:] = [[37, 23], [8, 8], [50, 41]]
    cases.append((g1, p1))
    for g, pl in cases:
        for bm in (0, 2):  # the binning box is ignored under the box support
            img, plan = _render(R, g, pl, R.Params(box_mode=bm, flags=fl))
            st = check_image_box_support(img, g, pl, plan.params)
            ell, _ = _render(R, g, pl, R.Params(box_mode=bm, flags=UG_FLAG_SCATTER))
            change = float(np.abs(img.astype(np.float64) - ell).max()) / st["peak"]
            assert change > 100 * 1e-4, f"box support changed the image by only {change:.3g} of peak"
            print("box support", st, "change vs ellipsoid", change)
    g, pl = cases[1]
    img, plan = _render(R, g, pl, R.Params(chi2=math.inf, flags=fl))
    check_image_box_support(img, g, pl, plan.params)
    check_image(img, g, pl, plan.params)  # the ellipsoid reference at chi^2 = inf
    with pytest.raises(UgError):
        R.Plan(g.n, pl.wh, R.Params(flags=UG_FLAG_BOX_SUPPORT), device=torch.device("cuda", 0))
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    with pytest.raises(UgError):
        plan.backward(gd, pd, torch.from_numpy(img).to(dev), torch.zeros(plan.num_pixels, device=dev))


@pytest.mark.parametrize("k", [1, 4])
def test_configs_sampled_pixels_box_support(R, k):
    """The box-support Phase 2 on full workloads (c1: 50k Gaussians, 16
    planes of 160^2, 1500 pixels over all planes; c4: 1M Gaussians, 256
    planes of 256^2, 300 pixels over three planes, which keeps the
    reference's boxes to those planes): seeded pixels against the
    reference."""
    from paper_2505_05643_amd._lib import UG_FLAG_BOX_SUPPORT, UG_FLAG_SCATTER
    from tests.parity import check_image_box_support
    g, pl, _ = synth.make_config(k)
    img, plan = _render(R, g, pl, R.Params(flags=UG_FLAG_SCATTER | UG_FLAG_BOX_SUPPORT))
    if k == 1:
        pix = synth.sample_pixels(pl, 1500, 801)
    else:
        planes = np.random.default_rng(5).choice(pl.p, 3, replace=False)
        pix = synth.sample_pixels(pl.subset(planes), 300, 804)
        pix[:, 0] = planes[pix[:, 0]]
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    st = check_image_box_support(img[flat], g, pl, plan.params, pix=pix)
    print(f"box support c{k}", st)


def test_records_are_the_inplane_conic(R):
    """ug_debug_records: every record's float conic against the float64
    restriction of Eq. 8 to the plane (centre, 2x2 precision, offset r^2):
    T^T T = log2(e)/2 diag(s) A diag(s) in pixel units, the centre at the
    pixel coordinates of c, e0 and emin from r^2 and chi^2 (relative 1e-5)."""
    import math

    import oracle
    from tests.parity import oracle_params
    g = synth.make_gaussians(300, 71, (0, 0, 0), (1, 1, 1), (0.02, 0.12), aniso_max=8.0, opacity="random")
    pl = synth.random_planes(3, 72, (8, 8), 1 / 40, 0.3, 0.7)
    pl.wh[:] = [[37, 23], [48, 48], [50, 41]]
    img, plan = _render(R, g, pl)
    allrec = plan.debug_records()
    n_rec = plan.status(counts=True)[1]
    assert allrec.shape[0] == n_rec > 50
    # a pair whose footprint misses the image keeps a zeroed record with an
    # empty rectangle; the conic is compared on the others
    on = (allrec["tx0"] <= allrec["tx1"]) & (allrec["ty0"] <= allrec["ty1"])
    assert np.all(allrec["t11"][~on] == 0) and on.sum() > 50
    rec = allrec[on]
    op = oracle_params(plan.params)
    cen, A, r2 = oracle.inplane_conic(g, pl, op)
    k = 0.5 * math.log2(math.e)
    alpha = oracle.sigmoid(g.opacity)
    gi, pi = rec["gaussian"].astype(int), rec["plane"].astype(int)
    assert np.all(np.diff(gi) >= 0)  # Gaussian-major
    sx, sy = pl.spacing[pi, 0].astype(np.float64), pl.spacing[pi, 1].astype(np.float64)
    W, H = pl.wh[pi, 0].astype(np.float64), pl.wh[pi, 1].astype(np.float64)
    t11, t12, t22 = (rec[f].astype(np.float64) for f in ("t11", "t12", "t22"))
    Ap = A[gi, pi]
    want = np.stack([k * Ap[:, 0, 0] * sx * sx, k * Ap[:, 0, 1] * sx * sy, k * Ap[:, 1, 1] * sy * sy], axis=1)
    got = np.stack([t11 * t11, t11 * t12, t12 * t12 + t22 * t22], axis=1)
    scale = np.abs(want).max(axis=1, keepdims=True)
    assert np.max(np.abs(got - want) / scale) <= 1e-5
    cu = rec["ub"] + rec["fu"].astype(np.float64)
    cv = rec["vb"] + rec["fv"].astype(np.float64)
    np.testing.assert_allclose(cu, cen[gi, pi, 0] / sx + W / 2 - 0.5, rtol=0, atol=1e-4)
    np.testing.assert_allclose(cv, cen[gi, pi, 1] / sy + H / 2 - 0.5, rtol=0, atol=1e-4)
    la = np.log2(alpha[gi])
    np.testing.assert_allclose(rec["e0"], la - k * r2[gi, pi], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(rec["emin"], la - k * op.chi2, rtol=1e-5, atol=1e-5)
    np.testing.assert_array_equal(rec["c"], g.intensity[gi])
    # every pair whose plane meets the ellipsoid has a record (the float cull
    # may add a few that narrowly miss, whose support is empty)
    meets = set(zip(*np.nonzero(r2 <= op.chi2)))
    assert meets <= set(zip(allrec["gaussian"].tolist(), allrec["plane"].tolist()))


def test_widest_planes_gather_and_box_support(R):
    """Planes at the widest size the plan accepts (32,767 pixels): the
    16-bit tile and pixel rectangles and the pixel offsets near their
    limits, for the gather (every binning) and the box-support scatter."""
    from paper_2505_05643_amd._lib import UG_FLAG_BOX_SUPPORT, UG_FLAG_SCATTER
    from tests.parity import check_image_box_support
    W = 32767
    frames = [np.eye(3), synth.axis_angle((1, 0, 0), 0.3)]
    pl = synth.pack_planes(frames, [(0.5, 0.5, 0.5), (0.5, 0.5, 0.52)], [(1.0 / 8192, 1.0 / 256)] * 2,
                           [(W, 3), (W, 5)])
    rng = np.random.default_rng(81)
    g = synth.make_gaussians(120, 82, (0.0, 0.49, 0.45), (1.0, 0.51, 0.55), (0.001, 0.01), opacity="random")
    # a few Gaussians right at the far end of the planes
    # (pixel u sits at x = 0.5 + (u + 1/2 - W/2) / 8192: x in [-1.5, 2.5])
    g.means[:6, 0] = (2.47 + 0.02 * rng.random(6)).astype(np.float32)
    g.means[:6, 1] = (0.5 + 0.002 * rng.standard_normal(6)).astype(np.float32)   # on the tilted plane
    g.means[:6, 2] = (0.52 + 0.002 * rng.standard_normal(6)).astype(np.float32)
    pix = np.concatenate([np.stack([np.zeros(300, int), rng.integers(12000, 20600, 300), rng.integers(0, 3, 300)], 1),
                          np.stack([np.zeros(100, int), rng.integers(0, W, 100), rng.integers(0, 3, 100)], 1),
                          np.stack([np.ones(400, int), rng.integers(W - 400, W, 400), rng.integers(0, 5, 400)], 1)])
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    for bm in (0, 1, 2):
        img, plan = _render(R, g, pl, R.Params(box_mode=bm))
        check_image(img[flat], g, pl, plan.params, pix=pix)
    img, plan = _render(R, g, pl, R.Params(flags=UG_FLAG_SCATTER | UG_FLAG_BOX_SUPPORT))
    check_image_box_support(img[flat], g, pl, plan.params, pix=pix)
    assert img.shape[0] == W * 8


@pytest.mark.parametrize("k,count", [(1, 1200), (2, 600)])
def test_split_forward_parity_and_determinism(R, k, count):
    """UG_FLAG_SPLIT_FORWARD (two waves per band, alternate record rounds):
    every tile shape and LDS batch on small ragged planes and the full c1 /
    c2 workloads on sampled pixels against the oracle; run to run bitwise;
    within 2e-5 of the peak of the one-wave image (the two halves' sums are
    grouped differently), except for pixels with a pair on the cut-off."""
    from tests.parity import reference_points
    import oracle
    flag = R._lib.UG_FLAG_SPLIT_FORWARD
    g = synth.make_gaussians(500, 91, (0, 0, 0), (1, 1, 1), (0.02, 0.12), aniso_max=8.0, opacity="random")
    pl = synth.random_planes(3, 92, (8, 8), 1 / 48, 0.35, 0.65)
    pl.wh[:] = [[61, 47], [32, 32], [48, 17]]
    for tw, th in ((8, 8), (16, 16), (32, 32), (16, 32), (32, 8)):
        for bg in (32, 64, 128):
            img, plan = _render(R, g, pl, R.Params(tile_w=tw, tile_h=th, lds_batch=bg, flags=flag))
            check_image(img, g, pl, plan.params)
    g, pl, _ = synth.make_config(k)
    from tests.configs import tuned_params
    base = tuned_params(g, pl)
    params = R.Params(**{**base.__dict__, "flags": flag})
    dev = torch.device("cuda", 0)
    gd, pd = R.to_device(g, dev), R.to_device(pl, dev)
    plan = R.Plan(g.n, pl.wh, params, device=dev)
    plan.fit(gd, pd)
    a = plan.render(gd, pd).clone()
    b = plan.render(gd, pd).clone()
    one = R.Plan(g.n, pl.wh, base, device=dev)
    one.fit(gd, pd)
    c = one.render(gd, pd)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    peak = float(c.abs().max())
    assert int(((a - c).abs() > 2e-5 * peak).sum()) <= max(1, 1e-4 * a.numel())
    pix = synth.sample_pixels(pl, count, 700 + k)
    offs = pl.pixel_offsets()
    flat = offs[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
    ref, _ = reference_points(g, oracle.plane_points(pl, pix), params)
    print(f"c{k} split", check_image(a.cpu().numpy()[flat], g, pl, params, pix=pix, ref=ref))
