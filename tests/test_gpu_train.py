"""Training step: the device-step Adam against a float64 reference of the
update rule, hipGraph replay against eager steps, the overflow guard, and a
short fit."""
import numpy as np
import pytest

from paper_2505_05643_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_05643_amd import raster, step
    return raster, step


def _adam_ref(p, g_seq, cfg, seg_lr):
    """Adam in float64 for a list of gradients; seg_lr(t) -> learning rate."""
    p = p.astype(np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t, g in enumerate(g_seq, start=1):
        g = g.astype(np.float64)
        m = cfg.beta1 * m + (1 - cfg.beta1) * g
        v = cfg.beta2 * v + (1 - cfg.beta2) * g * g
        mh = m / (1 - cfg.beta1 ** t)
        vh = v / (1 - cfg.beta2 ** t)
        p -= seg_lr(t) * mh / (np.sqrt(vh) + cfg.eps)
    return p


@pytest.mark.parametrize("m,offset", [(1, 0), (7, 0), (1023, 0), (12293, 0), (409_600, 0), (409_603, 1),
                                      (2_000_001, 0)])
def test_mse_grad_matches_numpy(M, m, offset):
    """d_image = 2 (image - target) / m and the mean squared error, against
    float64 numpy; offset 1 makes the arrays 4-byte (not 16-byte) aligned,
    so the single-pixel path runs.  Called twice on the same scratch
    buffer: the block counter must be left at zero."""
    R, _ = M
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(m)
    img = rng.standard_normal(m + offset).astype(np.float32)
    tgt = rng.standard_normal(m + offset).astype(np.float32)
    a = torch.from_numpy(img).to(dev)[offset:]
    b = torch.from_numpy(tgt).to(dev)[offset:]
    d = torch.empty(m + offset, dtype=torch.float32, device=dev)[offset:]
    buf = torch.zeros(R._lib.UG_MSE_SCRATCH_FLOATS, dtype=torch.float32, device=dev)
    diff = img[offset:].astype(np.float64) - tgt[offset:].astype(np.float64)
    ref_d = 2.0 * diff / m
    ref_loss = float(np.mean(diff * diff))
    for _ in range(2):
        loss, dimg = R.mse_grad(a, b, d, buf)
        torch.cuda.synchronize()
        got = dimg.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref_d)) <= 1e-6 * np.max(np.abs(ref_d))
        assert abs(float(loss.item()) - ref_loss) <= 1e-5 * ref_loss


def test_adam_gaussians_matches_reference(M):
    R, S = M
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(0)
    n = 777
    cfg = S.AdamConfig(lr_means=1e-2, lr_means_final=1e-4, decay_steps=4, lr=0.05)
    p0 = [rng.standard_normal((n, 3)), rng.standard_normal((n, 6)), rng.random(n), rng.standard_normal(n)]
    params = R.GaussianTensors(*(torch.tensor(x, dtype=torch.float32, device=dev) for x in p0))
    z = lambda t: torch.zeros_like(t)  # noqa: E731
    m1 = R.GaussianTensors(*(z(t) for t in params))
    m2 = R.GaussianTensors(*(z(t) for t in params))
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    gseq = []
    for _ in range(6):
        gs = [rng.standard_normal(x.shape).astype(np.float32) for x in p0]
        gseq.append(gs)
        grads = R.GaussianTensors(*(torch.tensor(x, device=dev) for x in gs))
        S.adam_gaussians(params, grads, m1, m2, cfg, step)
    torch.cuda.synchronize()
    assert int(step.item()) == 6
    lr_mu = lambda t: cfg.lr_means * (cfg.lr_means_final / cfg.lr_means) ** min((t - 1) / cfg.decay_steps, 1.0)  # noqa: E731
    for k in range(4):
        ref = _adam_ref(p0[k].astype(np.float32), [gs[k] for gs in gseq], cfg,
                        lr_mu if k == 0 else (lambda t: cfg.lr))
        got = params[k].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)


def _problem(R, n=300, seed=81):
    g = synth.make_gaussians(n, seed, (0, 0, 0), (1, 1, 1), (0.03, 0.12), opacity="random")
    t = synth.make_gaussians(n, seed + 1, (0, 0, 0), (1, 1, 1), (0.03, 0.12))
    pl = synth.random_planes(4, seed + 2, (48, 40), 1 / 40, 0.35, 0.65)
    dev = torch.device("cuda", 0)
    gt, pt, tt = R.to_device(g, dev), R.to_device(pl, dev), R.to_device(t, dev)
    tplan = R.Plan(t.n, pl.wh, device=dev)
    tplan.fit(tt, pt)
    target = tplan.render(tt, pt).clone()
    return gt, pt, pl.wh, target


def test_graph_replay_equals_eager_steps(M):
    R, S = M
    gt, pt, wh, target = _problem(R)
    a = R.GaussianTensors(*(x.clone() for x in gt))
    b = R.GaussianTensors(*(x.clone() for x in gt))
    ea = S.TrainStep(a, pt, wh, target)
    eb = S.TrainStep(b, pt, wh, target)
    la = ea.run(8, use_graph=False)
    lb = eb.run(8, use_graph=True)
    torch.cuda.synchronize()
    assert ea.step_count == eb.step_count == 8
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert la == lb


def test_native_step_graph_equals_torch_graph_and_eager(M):
    """ug_step_capture / ug_step_replay: each replay (with eager work between
    them) leaves the same parameters, statistic and loss as the torch-captured
    graph and the eager steps, bit for bit; a reserve drops the capture."""
    R, S = M
    gt, pt, wh, target = _problem(R, seed=97)
    sets = [R.GaussianTensors(*(x.clone() for x in gt)) for _ in range(3)]
    native = S.TrainStep(sets[0], pt, wh, target, native_graph=True)
    graph = S.TrainStep(sets[1], pt, wh, target)
    eager = S.TrainStep(sets[2], pt, wh, target)
    for k in range(5):
        native.replay()
        graph.replay()
        eager.enqueue()
        junk = torch.randn(1000, device=pt.rot.device).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for x, y, z in zip(native.params, graph.params, eager.params):
            assert torch.equal(x, y) and torch.equal(x, z), k
        assert torch.equal(native.grad_acc, eager.grad_acc) and torch.equal(native.grad_cnt, eager.grad_cnt)
        assert float(native.loss_buf[0]) == float(eager.loss_buf[0]) == float(graph.loss_buf[0])
    assert native.step_count == 5 and native.plan.status() == 0
    from paper_2505_05643_amd._lib import UgError
    native.plan.reserve(native.plan.record_capacity + 64, native.plan.key_capacity)
    with pytest.raises(UgError):
        S.check(S.lib.ug_step_replay(native.plan._h, R._stream()), "ug_step_replay")
    native.graph = None  # re-captured on the next replay, against the new layout
    losses = native.run(3, check_every=1)
    assert native.step_count == 8 and len(losses) == 3


def test_training_reduces_loss(M):
    R, S = M
    gt, pt, wh, target = _problem(R, seed=91)
    st = S.TrainStep(gt, pt, wh, target, adam=S.AdamConfig(lr_means=2e-3, lr_means_final=2e-4, decay_steps=60,
                                                            lr=0.02))
    losses = st.run(60, use_graph=True, check_every=10)
    assert losses[-1] < 0.7 * losses[0], losses


def test_overflow_skips_update_and_run_recovers(M):
    R, S = M
    gt, pt, wh, target = _problem(R, seed=95)
    st = S.TrainStep(gt, pt, wh, target)
    st.run(2, use_graph=True)
    before = [x.clone() for x in st.params]
    st.plan.reserve(4, 8)          # far too small for this scene
    st.graph = None
    st.replay()
    torch.cuda.synchronize()
    assert st.plan.status() == R._lib.UG_ERR_CAPACITY
    assert st.step_count == 2      # the Adam launch skipped itself
    for x, y in zip(before, st.params):
        assert torch.equal(x, y)
    st.run(3, use_graph=True)      # re-sizes, re-captures, redoes the step
    assert st.step_count == 5


def test_training_with_densify(M):
    """The gradient statistic accumulates inside the captured step (and not
    for a step whose render overflowed); densify clones, splits and prunes by
    it, re-plans for the new number of Gaussians and training continues."""
    R, S = M
    from paper_2505_05643_amd import densify as Dn
    gt, pt, wh, target = _problem(R, seed=97)
    st = S.TrainStep(gt, pt, wh, target, adam=S.AdamConfig(lr_means=2e-3, lr_means_final=2e-4, decay_steps=60,
                                                            lr=0.02))
    l0 = st.run(20, use_graph=True, check_every=10)
    torch.cuda.synchronize()
    assert int(st.grad_cnt.min().item()) == 20 and float(st.grad_acc.max().item()) > 0.0
    # an overflowed render leaves the statistic alone
    acc0, cnt0 = st.grad_acc.clone(), st.grad_cnt.clone()
    st.plan.reserve(4, 8)
    st.graph = None
    st.replay()
    torch.cuda.synchronize()
    assert torch.equal(st.grad_acc, acc0) and torch.equal(st.grad_cnt, cnt0)
    st.plan.fit(st.params, st.planes, st.headroom)
    st.graph = None
    n0 = st.params.means.shape[0]
    med = float(st.grad_acc.median().item()) / 20.0
    prm = Dn.DensifyParams(grad_thresh=med, split_size=0.05, min_opacity=0.3)
    n1 = st.densify(prm, seed=3)
    assert n1 != n0 and st.plan.n == n1
    assert int(st.grad_cnt.sum().item()) == 0
    l1 = st.run(20, use_graph=True, check_every=10)
    assert all(np.isfinite(l1)) and l1[-1] < l0[0], (l0, l1)
