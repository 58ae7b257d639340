"""Benchmark: forward + backward planes/s of the probe-plane rasterizer.

One step = one pass of the whole hot path over one batch of planes: the
culling/record pass, key emission, the radix sort by tile, the per-tile
accumulation (forward), the MSE gradient against a target image, the
per-key adjoint, the per-record reduction and the per-Gaussian adjoint.
Inputs are seeded synthetic workloads already resident in device memory.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1]

Prints ONE JSON line.  Extra keys: in-support pair evaluations per second,
the plain per-plane form on the same GPU, per-stage times, a roofline for
the dominant kernel (timed with HIP events on its launch stream inside the
timed region) and the FP64 oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd planes/s and Gaussian-pixel evals/s vs plain per-plane, at 1e-4 err"

# Algorithmic FP32 work per in-support (Gaussian, pixel) pair, counted on
# the conic form of Eq. 8 restricted to the plane:
#   forward: du, dv (2), t1 = T11 du + T12 dv (3), t2 = T22 dv (1),
#            s = t1^2 + t2^2 (3), e = e0 - s (1), cut-off compare (1),
#            exp2 (1), D += w (1), N += w c (2)                        = 16
#   adjoint: the forward's first 13 plus dL/dw = gamma (c - c_hat) (2),
#            w dL/dw (1), dc += gamma w (2), de0 (1), dT11 (3), dT12 (2),
#            dT22 (3), du0 (1), dv0 (4)                                = 32
FLOPS_PER_PAIR = {"accum": 16, "accum_bwd": 32}
# The Phase-1 test of one (Gaussian, plane) pair: m3 = r3 . (mu - o) (3 sub,
# 3 mul, 2 add), forward substitution L g = r3 with the Gaussian's reciprocal
# diagonal (9), Sigma'_33 = |g|^2 (5), m3^2 <= chi^2 Sigma'_33 (3)      = 25
FLOPS_PER_CULL_TEST = 25
# MI355X's published FP32 vector peak (256 CUs x 2.4 GHz x 256 flop per CU
# and clock; it needs packed FP32 instructions) and the peak of the scalar
# FP32 forms these kernels are compiled to (packed FP32 stays disabled):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 157.3
ALU_PEAK_SCALAR_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


_T0 = time.perf_counter()


def progress(what: str) -> None:
    """One line on stderr as each leg of the run ends."""
    print(f"bench: {what} ({time.perf_counter() - _T0:.1f} s)", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, pl, n_px: int, workers: int) -> dict:
    """The FP64 oracle, forward + adjoint, on a seeded sample of pixels spread
    over all planes of the workload, against every Gaussian, on ``workers``
    host processes (one chunk of the sample each)."""
    import oracle
    from oracle import pool
    from paper_2505_05643_amd import synth
    pix = synth.sample_pixels(pl, n_px, 901)
    X = oracle.plane_points(pl, pix)
    dout = np.random.default_rng(902).standard_normal(X.shape[0])
    t0 = time.perf_counter()
    out, _ = pool.render_points(g, X, workers=workers)
    pool.grad_points(g, X, dout, workers=workers)
    dt = time.perf_counter() - t0
    return {"seconds": dt, "pix": pix, "values": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=4,
                    help="workload 0-4 (default 4: 1M Gaussians, 256 planes of 256^2, the largest)")
    ap.add_argument("--tile", type=str, default=None, help="WxH[xPPL], e.g. 16x16x1")
    ap.add_argument("--lds-batch", type=int, default=None)
    ap.add_argument("--box", type=int, default=None, help="0 paper, 1 conic, 2 rows")
    ap.add_argument("--split", type=int, default=None, choices=(0, 1),
                    help="forward with two waves per 8-row band (UG_FLAG_SPLIT_FORWARD)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-plane comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-scatter", action="store_true", help="skip timing the Phase-2 atomic scatter forward")
    ap.add_argument("--no-densify", action="store_true", help="skip timing the densify / prune pass")
    ap.add_argument("--no-recon", action="store_true",
                    help="skip the synthetic reconstruction-quality workload (run with the default workload)")
    ap.add_argument("--recon-steps", type=int, default=300, help="training steps per reconstruction case")
    ap.add_argument("--train-steps", type=int, default=2000,
                    help="steps of the 1M-Gaussian training run on pool planes (workload 4; 0 skips it)")
    ap.add_argument("--no-param-study", action="store_true",
                    help="skip the covariance parameterisation study (run with the default workload)")
    ap.add_argument("--cpu-px", type=int, default=0,
                    help="oracle baseline sample in pixels (default: sized for about 20 s on the host cores)")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches only")
    ap.add_argument("--no-autotune", action="store_true", help="use the default launch configuration")
    ap.add_argument("--retune", action="store_true",
                    help="search launch configurations even if the autotune cache has this workload")
    ap.add_argument("--tune-cache", type=str, default=None,
                    help="autotune cache file (default: the package's autotune_cache.json); a search stores its "
                         "pick there")
    ap.add_argument("--peaks", action="store_true", help="print the chip's measured throughput probes and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="finish with 5 elementwise copies (dst = -src) of MIB MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; the multi-GPU (plane-sharded) path is a design, "
              "not an implementation. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2505_05643_amd import synth
    from paper_2505_05643_amd import raster as R

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.peaks:
        print(json.dumps(measured_peaks(dev)), flush=True)
        return
    k = args.config
    g, pl, tg = synth.make_config(k)
    gd, pd, tgd = R.to_device(g, dev), R.to_device(pl, dev), R.to_device(tg, dev)

    params = R.Params()
    tuned = None
    if not (args.tile or args.lds_batch or args.box is not None or args.split is not None or args.no_autotune):
        from paper_2505_05643_amd import autotune
        cache = args.tune_cache or autotune.CACHE
        sig = autotune.signature(g.n, pl.wh)
        cached = None if args.retune else autotune.cached_params(sig, cache)
        if cached is not None:
            params = cached
            tuned = {"source": "cache", "signature": sig}
        else:
            params, results = autotune.tune(gd, pd, pl.wh, steps=3)
            default = next((r for r in results if (r["tile_w"], r["tile_h"], r["px_per_lane"], r["lds_batch"],
                                                   r["box_mode"]) == (16, 16, 2, 64, 0)), None)
            best = min(results, key=lambda r: r["ms"])
            tuned = {"source": "search", "signature": sig, "candidates": len(results), "best_ms": best["ms"],
                     "default_16x16_paper_ms": default["ms"] if default else None}
            autotune.store(sig, params, best["ms"], cache)
    if args.tile:
        parts = [int(x) for x in args.tile.lower().split("x")]
        params.tile_w, params.tile_h = parts[0], parts[1]
        params.px_per_lane = parts[2] if len(parts) > 2 else 0
    if args.lds_batch:
        params.lds_batch = args.lds_batch
    if args.box is not None:
        params.box_mode = args.box
    if args.split is not None:
        params.flags = (params.flags | R._lib.UG_FLAG_SPLIT_FORWARD) if args.split else (
            params.flags & ~R._lib.UG_FLAG_SPLIT_FORWARD)

    # target image: the second seeded Gaussian set rendered on the same planes
    tplan = R.Plan(tg.n, pl.wh, params, device=dev)
    tplan.fit(tgd, pd)
    target = tplan.render(tgd, pd).clone()
    del tplan

    plan = R.Plan(g.n, pl.wh, params, device=dev)
    n_rec, n_key = plan.fit(gd, pd)
    image = torch.empty(plan.num_pixels, device=dev)
    d_image = torch.empty_like(image)
    loss_buf = torch.zeros(1026, device=dev)
    grads = R.GaussianTensors(torch.empty_like(gd.means), torch.empty_like(gd.lraw),
                              torch.empty_like(gd.intensity), torch.empty_like(gd.opacity))

    def step(p=plan, gg=gd, pp=pd, img=image, gr=grads, tgt=target):
        p.render(gg, pp, img, check_status=False)
        p.backward_mse(gg, pp, img, tgt, gr, loss_buf=loss_buf)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    code = plan.status()
    assert code == 0, f"render status {code}"

    # ---- timed region (per-stage events on the launch stream) ----
    plan.profile_begin(max_launches=args.steps * 32 + 16)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms_total = t0.elapsed_time(t1)
    stages = plan.profile_read()
    progress("eager steps timed")
    eager_ms_step = ms_total / args.steps
    eager_image = image.clone()

    # ---- the same step captured once as a hipGraph and replayed ----
    graph_ms_step = None
    if not args.no_graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(image, eager_image), "graph replay must match the eager step"
        t0.record()
        for _ in range(args.steps):
            graph.replay()
        t1.record()
        torch.cuda.synchronize()
        graph_ms_step = t0.elapsed_time(t1) / args.steps
        progress("graph steps timed")
        assert torch.equal(image, eager_image), "graph replay must match the eager step"
        del graph
    ms_step = graph_ms_step if graph_ms_step is not None else eager_ms_step
    ms_total = ms_step * args.steps
    planes_s = pl.p * args.steps / (ms_total / 1e3)

    # ---- context figures: the forward alone, and the full training step ----
    fwd_ms = None
    train_ms = None
    if not args.no_graph:
        fwd_ms = replay_ms(lambda: plan.render(gd, pd, image, check_status=False), args.warmup, args.steps)
        fwd_img = image.clone()
        assert torch.equal(fwd_img, eager_image), "the forward alone must render the same image"
        from paper_2505_05643_amd.step import AdamConfig, TrainStep
        tparams = R.GaussianTensors(*(t.clone() for t in gd))
        # the cost of one full step at the workload's Gaussians: every kernel
        # runs, with learning rates too small to move them
        tiny = AdamConfig(lr_means=1e-12, lr_means_final=1e-12, lr=1e-12)
        ts = TrainStep(tparams, pd, pl.wh, target, plan.params, adam=tiny)
        ts.run(max(args.warmup, 1))  # captures the step as a hipGraph and replays it
        torch.cuda.synchronize()
        n_train = args.steps
        t0.record()
        for _ in range(n_train):
            ts.replay()
        t1.record()
        torch.cuda.synchronize()
        train_ms = t0.elapsed_time(t1) / n_train
        if ts.plan.status() != 0:  # a step that overflowed skipped its update: no valid time
            train_ms = None
        del ts, tparams
        progress("forward alone and training step timed")

    # the paper's own accumulation (Phase 2 atomic scatter) on the same
    # records, for comparison with the gather forward above
    scatter = None
    if not args.no_graph and not args.no_scatter:
        sparams = R.Params(**{**params.__dict__, "flags": R._lib.UG_FLAG_SCATTER})
        splan = R.Plan(g.n, pl.wh, sparams, device=dev)
        splan.fit(gd, pd)
        simg = torch.empty_like(image)
        s_ms = replay_ms(lambda: splan.render(gd, pd, simg, check_status=False), 1, max(2, args.steps // 10))
        ok = splan.status() == 0
        # the two agree to float rounding except where a pair sits on the
        # cut-off (their exponents round differently): count those pixels
        peak = max(float(image.abs().max()), 1e-30)
        off = int(((simg - image).abs() > 1e-4 * peak).sum())
        scatter = {"forward_ms": s_ms if ok else None, "gather_forward_ms": fwd_ms,
                   "gather_speedup": (s_ms / fwd_ms) if (ok and fwd_ms) else None,
                   "pixels_off_gather_by_1e-4_peak": off, "pixels": int(image.numel())}
        del splan
        # the paper-literal support: every pixel of the Eq. 13 box counts
        bparams = R.Params(**{**params.__dict__,
                              "flags": R._lib.UG_FLAG_SCATTER | R._lib.UG_FLAG_BOX_SUPPORT})
        bplan = R.Plan(g.n, pl.wh, bparams, device=dev)
        bplan.fit(gd, pd)
        b_ms = replay_ms(lambda: bplan.render(gd, pd, simg, check_status=False), 1, max(2, args.steps // 10))
        bok = bplan.status() == 0
        scatter["box_support_forward_ms"] = b_ms if bok else None
        # how far the box support moves the image from the ellipsoid support
        scatter["box_support_max_change_by_peak"] = float((simg - image).abs().max()) / peak
        del bplan, simg
        progress("Phase-2 scatter forms timed")

    # in-support pairs of one forward, counted by the kernel itself
    cparams = R.Params(**{**params.__dict__, "flags": params.flags | R._lib.UG_FLAG_COUNT_EVALS})
    cplan = R.Plan(g.n, pl.wh, cparams, device=dev)
    cplan.fit(gd, pd)
    cimg = cplan.render(gd, pd)
    _, _, _, n_eval, n_exec = cplan.status(counts=True)
    assert torch.equal(cimg, image), "counting variant must render the same image"
    del cplan
    tpx = params.tile_w * params.tile_h
    evals_s = n_eval * args.steps / (ms_total / 1e3)

    # ---- plain per-plane form: the same library, one plan per plane ----
    plain = None
    if not args.no_plain:
        per = []
        for i in range(pl.p):
            one = pl.subset(i)
            pdi = R.to_device(one, dev)
            pli = R.Plan(g.n, one.wh, params, device=dev)
            pli.fit(gd, pdi)
            off = int(pl.pixel_offsets()[i])
            npx = int(one.wh[0, 0] * one.wh[0, 1])
            per.append((pli, pdi, image[off:off + npx], d_image[off:off + npx], target[off:off + npx]))
        gsum = R.GaussianTensors(*(torch.zeros_like(t) for t in grads))

        def plain_step():
            for j, (pli, pdi, img, dimg, tgt) in enumerate(per):
                pli.render(gd, pdi, img, check_status=False)
            R.mse_grad(image, target, d_image, loss_buf)
            for j, (pli, pdi, img, dimg, tgt) in enumerate(per):
                pli.backward(gd, pdi, img, dimg, gsum, accumulate=j > 0)

        for _ in range(max(2, args.warmup // 2)):
            plain_step()
        torch.cuda.synchronize()
        run = plain_step
        if graph_ms_step is not None:  # same launch mode as the batched figure
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                plain_step()
            torch.cuda.current_stream().wait_stream(side)
            pgraph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(pgraph):
                plain_step()
            run = pgraph.replay
            run()
            torch.cuda.synchronize()
        psteps = max(3, args.steps // 4)
        t0.record()
        for _ in range(psteps):
            run()
        t1.record()
        torch.cuda.synchronize()
        pms = t0.elapsed_time(t1) / psteps
        plain = {"planes_per_s": pl.p / (pms / 1e3), "ms_per_step": pms,
                 "launch": "hipGraph replay" if graph_ms_step is not None else "eager",
                 "batched_speedup": pms / ms_step}
        del per
        progress("plain per-plane form timed")

    # ---- roofline of every kernel; the dominant one is the headline ----
    # sort passes as launched (one histogram launch per pass); digit slots
    # per block histogram: 2^ceil(bits / passes) rounded up to 256 or 1024
    passes = max(1, round(stages["sort_hist"][1] / args.steps)) if "sort_hist" in stages else 1
    g_sort = min(2048, max(1, (plan.key_capacity + 2047) // 2048))
    dslots = 1024 if -(-plan_bits(plan) // passes) > 8 else 256
    sizes = dict(n=g.n, p=pl.p, r=n_rec, k=n_key, t=plan.num_tiles, m=int(pl.npix), passes=passes,
                 w=(pl.p + 63) // 64, rows=params.box_mode == 2, g_sort=g_sort, dslots=dslots)
    kernels = {}
    cull_grouped = cull_searches_groups(pl, params, g.n)
    for nm, (ms, n) in stages.items():
        avg = ms / max(n, 1)
        row = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps, "avg_launch_ms": avg}
        if nm in FLOPS_PER_PAIR or (nm == "cull_count" and not cull_grouped):
            if nm == "cull_count":
                flop = FLOPS_PER_CULL_TEST * g.n * pl.p
                work = f"{FLOPS_PER_CULL_TEST} flop x {g.n} x {pl.p} (Gaussian, plane) tests per launch"
            else:
                flop = FLOPS_PER_PAIR[nm] * n_eval
                work = f"{FLOPS_PER_PAIR[nm]} flop x {n_eval} in-support pairs per launch"
            ach = flop / (avg / 1e3) / 1e12
            row.update(bound="alu", achieved=ach, peak=ALU_PEAK_TFLOPS, unit="TFLOP/s", frac=ach / ALU_PEAK_TFLOPS,
                       frac_scalar_fp32_peak=ach / ALU_PEAK_SCALAR_TFLOPS, work=work)
            if nm in FLOPS_PER_PAIR:
                row["evaluated_pairs"] = n_exec
        else:
            nbytes = kernel_bytes(nm, **sizes)
            ach = nbytes / (avg / 1e3) / 1e9
            row.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                       work=f"{nbytes} algorithmic bytes per launch")
            if nm == "cull_count":
                row["work"] += " (grouped search over parallel slices: not N x P tests)"
        kernels[nm] = row
    dom_name = max(kernels, key=lambda nm: kernels[nm]["ms_per_step"])
    d = kernels[dom_name]
    roof = {"bound": d["bound"], "kernel": dom_name, "achieved": d["achieved"], "peak": d["peak"],
            "unit": d["unit"], "frac": d["frac"], "traffic": stored_traffic(dom_name, k, params, plan),
            "work": d["work"], "avg_launch_ms": d["avg_launch_ms"]}
    if d["bound"] == "alu":
        roof["peak_scalar_fp32"] = ALU_PEAK_SCALAR_TFLOPS
        roof["frac_scalar_fp32_peak"] = d["frac_scalar_fp32_peak"]
    acc = {nm: kernels[nm] for nm in ("accum", "accum_bwd") if nm in kernels}

    out = {
        "metric": METRIC,
        "value": planes_s,
        "unit": "planes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": synth.CONFIG_NAMES[k], "gaussians": g.n, "planes": pl.p,
                   "pixels": int(pl.npix), "tile": f"{params.tile_w}x{params.tile_h}",
                   "px_per_lane": plan_ppl(params), "lds_batch": params.lds_batch, "box_mode": params.box_mode,
                   "split_forward": bool(params.flags & R._lib.UG_FLAG_SPLIT_FORWARD),
                   "step": "render + MSE adjoint (gradient of the loss formed in the first adjoint kernel)",
                   "launch": "hipGraph replay" if graph_ms_step is not None else "eager"},
        "autotune": tuned,
        "eager_ms_per_step": eager_ms_step,
        "graph_ms_per_step": graph_ms_step,
        "forward_only_ms": fwd_ms,
        "train_step_ms": train_ms,
        "paper_phase2_scatter": scatter,
        "densify": densify_ms(R, gd, dev, args.warmup, args.steps) if not args.no_densify else None,
        "evals_per_s": evals_s,
        "in_support_pairs": n_eval,
        "records": n_rec,
        "keys": n_key,
        "evaluated_pairs": n_exec,
        "tile_efficiency": n_eval / max(n_key * tpx, 1),
        "subblock_efficiency": n_eval / max(n_exec, 1),
        "plain_per_plane": plain,
        "accumulate_kernels": acc,
        "kernels": kernels,
        "roofline": roof,
        "measured_peaks": measured_peaks(dev),
    }
    progress("kernel table and probes done")
    if k == 4 and args.train_steps > 0 and not args.no_graph:
        out["config4_training"] = config4_training(dev, params, args.train_steps)
        progress("1M-Gaussian training run and extraction done")
    if k == 1 and not args.no_recon and not args.no_graph:
        out["reconstruction"] = reconstruction(dev, args.recon_steps)
    if k == 1 and not args.no_param_study:
        from paper_2505_05643_amd import paramstudy
        out["parameterization"] = {"float32_error": paramstudy.study(device=dev),
                                   "throughput": paramstudy.throughput(device=dev)}

    if not args.no_cpu_baseline:
        from oracle import pool
        workers = pool.default_workers()
        # about 20 s of host time: the oracle costs about 5.6e-7 s per
        # (Gaussian, pixel) pair for forward + adjoint on one core
        n_px = args.cpu_px or int(max(workers, min(pl.npix, 20.0 * workers / (5.6e-7 * g.n))))
        cb = cpu_baseline(g, pl, n_px, workers)
        pix = cb["pix"]
        flat = pl.pixel_offsets()[pix[:, 0]] + pix[:, 2] * pl.wh[pix[:, 0], 0] + pix[:, 1]
        gpu_vals = image.cpu().numpy().astype(np.float64)[flat]
        ref = np.asarray(cb["values"])
        planes_equiv = len(pix) * pl.p / pl.npix  # the sample as a fraction of one step's planes
        out["cpu_baseline"] = {"value": planes_equiv / cb["seconds"], "unit": "planes/s", "cores": workers,
                               "kind": "oracle", "cpu": cpu_model(),
                               "sample": f"{len(pix)} seeded pixels over all {pl.p} planes x all {g.n} Gaussians, "
                                         f"FP64 forward + adjoint, {cb['seconds']:.1f} s on {workers} worker "
                                         f"processes, scaled to planes of the workload's mean size"}
        out["parity_sample_max_rel"] = float(np.abs(gpu_vals - ref).max() / max(np.abs(ref).max(), 1e-30))
        progress("oracle baseline done")
    print(json.dumps(out), flush=True)

    if args.copy_probe:
        src = torch.ones(args.copy_probe << 18, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()


def reconstruction(dev, steps):
    """The synthetic reconstruction-quality workload: each case (full axial
    coverage, half, half with +-5 degree tilts) trained from the Section 4.5
    initialisation for ``steps`` graph-replayed steps over all its slices,
    then scored by SSIM / PSNR on 160 axial, coronal and sagittal slices."""
    from paper_2505_05643_amd import raster as R
    from paper_2505_05643_amd import recon, synth
    setup = recon.ReconSetup(steps=steps)
    truth = R.to_device(recon.truth_gaussians(setup), dev)
    scorer = recon.Scorer(setup, truth, R.Params(), dev)
    cases = [recon.run_case(setup, c, dev, scorer=scorer) for c in recon.CASES]
    # the scoring kernel alone over all evaluation slices: it reads two
    # float32 images (8 B per pixel); its FP64 window sums bound it (row
    # pass 10 flop per tap x 11 taps, once per row; column pass 5 x 2 flop
    # x 11 taps; the score about 20: about 240 flop per pixel)
    img = scorer.images(R.to_device(synth.paper_init(setup.n_model, 6000), dev))
    q_ms = scorer.quality_ms(img)
    npx = img.numel()
    return {"setup": {"volume": f"phantom in the unit cube, {setup.n_truth} seeded ground-truth Gaussians",
                      "slices": f"{setup.size}^2", "gaussians": setup.n_model, "steps": steps},
            "cases": cases,
            "quality_kernel": {"ms": q_ms, "pixels": npx, "gpix_per_s": npx / (q_ms * 1e6),
                               "hbm_gbs": 8 * npx / (q_ms * 1e6),
                               "fp64_tflops": 240 * npx / (q_ms * 1e9)}}


def config4_training(dev, params, steps: int, seed: int = 404, check_every: int = 20) -> dict:
    """The 1M-Gaussian workload trained as stated: every step draws 256
    distinct planes of 256^2 (seeded) from the pool of 2,048 planes of 8
    interleaved oblique sweeps, gathers their poses and target images (the
    seed-204 Gaussian set rendered once on the whole pool) into the step's
    fixed buffers, and replays the captured step (render, MSE adjoint, Adam).
    The scene is expressed in the unit cube (the 256-voxel domain scaled by
    1/256; images unchanged), the frame in which the Section 4.5 learning
    rates are stated.  Every ``check_every`` steps the device step counter
    recorded after each step is read: a step whose render overflowed its
    capacity skipped its update on the device, so the plan is re-sized for the
    current Gaussians on those draws, the step captured again and those steps
    redone.  Then the trained Gaussians are extracted
    as the 256 axial planes of the 256^3 volume in one forward launch."""
    import torch
    from paper_2505_05643_amd import raster as R
    from paper_2505_05643_amd import synth
    from paper_2505_05643_amd.step import AdamConfig, TrainStep
    unit = 1.0 / 256.0
    _, pool = synth.rescale(None, synth.config4_training_pool(), unit)
    P, per = pool.p, 256
    wh = pool.wh[:per]
    pool_d = R.to_device(pool, dev)
    tg = R.to_device(synth.rescale(synth.config_gaussians(4, target=True), None, unit)[0], dev)
    tplan = R.Plan(tg.means.shape[0], wh, params, device=dev)
    npx = int(wh[0, 0] * wh[0, 1])
    targets = torch.empty(P, npx, device=dev)
    for c in range(0, P, per):
        sub = R.PlaneTensors(*(t[c:c + per] for t in pool_d))
        tplan.fit(tg, sub)
        tplan.render(tg, sub, targets[c:c + per].view(-1))
    del tplan, tg
    rng = np.random.default_rng(seed)
    draws = np.stack([rng.choice(P, size=per, replace=False) for _ in range(steps)]).astype(np.int64)
    idx = torch.from_numpy(draws).to(dev)
    planes = R.PlaneTensors(*(t.index_select(0, idx[0]).contiguous() for t in pool_d))
    target = targets.index_select(0, idx[0]).reshape(-1).contiguous()
    gauss = R.to_device(synth.rescale(synth.config_gaussians(4), None, unit)[0], dev)
    ts = TrainStep(gauss, planes, wh, target, params, adam=AdamConfig(decay_steps=steps), headroom=1.3)
    loss = torch.zeros(steps, device=dev)
    done_after = torch.zeros(steps, dtype=torch.int32, device=dev)  # device step counter after each step

    def gather(i):
        for dst, src in zip(planes, pool_d):
            torch.index_select(src, 0, idx[i], out=dst)
        torch.index_select(targets, 0, idx[i], out=target.view(per, npx))

    gather(0)
    ts.capture()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    refits = redone = 0
    t0.record()
    todo = list(range(steps))
    count = 0  # the device step counter before the window
    while todo:
        window, todo = todo[:check_every], todo[check_every:]
        for i in window:
            gather(i)
            ts.replay()
            loss[i:i + 1].copy_(ts.loss_buf[:1])
            done_after[i:i + 1].copy_(ts.step_dev)
        # the steps of this window whose Adam launch skipped itself (their
        # render overflowed): the device counter did not advance
        after = done_after[window].cpu().numpy().astype(np.int64)
        before = np.concatenate([[count], after[:-1]])
        skipped = [w for w, a, b0 in zip(window, after, before) if a == b0]
        count = int(after[-1])
        if skipped:
            if refits >= 100:  # the Gaussians keep outgrowing every re-size: stop here
                break
            for w in skipped:  # capacities for the largest of the skipped draws
                gather(w)
                ts.plan.fit(ts.params, planes, 1.5)
            ts.capture()
            refits += 1
            redone += len(skipped)
            todo = skipped + todo
    t1.record()
    torch.cuda.synchronize()
    done = ts.step_count
    ms = t0.elapsed_time(t1) / max(done, 1)
    lh = loss.cpu().numpy().astype(float)
    # extraction: the 256 axial planes of the volume, one forward launch
    _, ext = synth.rescale(None, synth.config_planes(4), unit)
    ext_d = R.to_device(ext, dev)
    eplan = R.Plan(ts.params.means.shape[0], ext.wh, params, device=dev)
    eplan.fit(ts.params, ext_d)
    vol = torch.empty(eplan.num_pixels, device=dev)
    ext_ms = replay_ms(lambda: eplan.render(ts.params, ext_d, vol, check_status=False), 2, 10)
    ok = eplan.status() == 0
    marks = sorted({0, 1, 10, 100, steps // 2, steps - 1} & set(range(steps)))
    return {"steps": steps, "planes_per_step": per, "pool_planes": P, "ms_per_step": ms,
            "planes_per_s": per / (ms / 1e3), "adam_updates_done": done, "capacity_refits": refits,
            "steps_redone_after_overflow": redone,
            "loss_at_step": {str(m): lh[m] for m in marks},
            "loss_mean_first_100": float(np.mean(lh[:100])), "loss_mean_last_100": float(np.mean(lh[-100:])),
            "frame": "unit cube (256-voxel domain scaled by 1/256)",
            "launch": "gather (torch index_select) + captured step replay per step; step counter read every "
                      f"{check_every} steps; ms_per_step = wall time incl. re-sizing and redone steps / updates done",
            "extraction_ms": ext_ms if ok else None, "extraction_planes": ext.p,
            "extraction_voxels_per_s": (eplan.num_pixels / (ext_ms / 1e3)) if ok else None}


def densify_ms(R, gd, dev, warmup, steps):
    """The densify / prune pass over the workload's Gaussians with seeded
    gradient statistics (about a tenth cloned or split, a few pruned):
    average ms per call and its rate against HBM.  Algorithmic bytes: the
    decision pass reads lraw, opacity and the statistics (36 B per
    Gaussian), the write pass reads them again with means and intensity
    (52 B) and writes 44 B per output (the 24 B of z a split reads are not
    counted, so the rate is a lower bound)."""
    import ctypes
    import numpy as np
    import torch
    from paper_2505_05643_amd import _lib
    n = gd.means.shape[0]
    rng = np.random.default_rng(77)
    cnt = torch.from_numpy(rng.integers(1, 20, n).astype(np.int32)).to(dev)
    acc = torch.from_numpy((rng.uniform(0.0, 2.2e-4, n) * cnt.cpu().numpy()).astype(np.float32)).to(dev)
    z = torch.from_numpy(rng.standard_normal((n, 2, 3)).astype(np.float32)).to(dev)
    cap = 2 * n
    out = [torch.empty((cap,) + sh, device=dev) for sh in ((3,), (6,), (), ())]
    ws = torch.empty((_lib.lib.ug_densify_workspace_bytes(n) + 3) // 4 + 1, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    cg = R._c_gauss(gd)
    co = _lib.UgGaussiansMut(*(t.data_ptr() for t in out), cap)
    dp = _lib.UgDensifyParams()
    _lib.lib.ug_densify_params_default(ctypes.byref(dp))

    def call():
        R.check(_lib.lib.ug_densify(ctypes.byref(cg), acc.data_ptr(), cnt.data_ptr(), z.data_ptr(), ctypes.byref(dp),
                                    ctypes.byref(co), cap, count.data_ptr(), ws.data_ptr(), R._stream()), "ug_densify")

    for _ in range(max(1, warmup)):
        call()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(3, steps)
    t0.record()
    for _ in range(reps):
        call()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    m = int(count.item())
    nbytes = 36 * n + 52 * n + 44 * m
    return {"ms": ms, "gaussians_in": n, "gaussians_out": m, "algorithmic_bytes": nbytes,
            "achieved_gbs": nbytes / (ms / 1e3) / 1e9, "frac_hbm": nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def measured_peaks(dev) -> dict:
    """The library's throughput probes (best of three launches each): FMA
    chains (scalar FP32 VALU), v_exp_f32 chains, the forward's pair
    evaluation on registers, and a 512 MiB device copy (HBM read + write)."""
    import ctypes
    import torch
    from paper_2505_05643_amd import _lib
    blocks, iters = 2048, 16384
    out = torch.empty(blocks * 256, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    ms = ctypes.c_float()

    def best(kind, b, it, src, dst, n):
        t = []
        for _ in range(3):
            _lib.check(_lib.lib.ug_probe(kind, b, it, src, dst, n, ctypes.byref(ms), stream), "ug_probe")
            t.append(ms.value)
        return min(t)

    res = {}
    t = best(_lib.UG_PROBE_FMA, blocks, iters, None, out.data_ptr(), out.numel())
    res["fma_tflops"] = 16.0 * iters * 256 * blocks / (t / 1e3) / 1e12
    t = best(_lib.UG_PROBE_EXP, blocks, iters, None, out.data_ptr(), out.numel())
    res["exp_per_s"] = 8.0 * iters * 256 * blocks / (t / 1e3)
    t = best(_lib.UG_PROBE_PAIRS, blocks, iters, None, out.data_ptr(), out.numel())
    res["forward_pairs_per_s"] = 8.0 * iters * 256 * blocks / (t / 1e3)
    n = 128 << 20
    src = torch.ones(n, device=dev)
    dst = torch.empty_like(src)
    t = best(_lib.UG_PROBE_COPY, 8192, 1, src.data_ptr(), dst.data_ptr(), n)
    res["copy_gbs"] = 8.0 * n / (t / 1e3) / 1e9
    res["scalar_fp32_peak_tflops"] = ALU_PEAK_SCALAR_TFLOPS
    res["published_fp32_peak_tflops"] = ALU_PEAK_TFLOPS
    res["published_hbm_gbs"] = HBM_PEAK_GBS
    del src, dst, out
    return res


def replay_ms(fn, warmup, steps):
    """Average ms of fn captured once as a hipGraph and replayed."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    for _ in range(max(warmup, 1)):
        graph.replay()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        graph.replay()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def cull_searches_groups(pl, params, n) -> bool:
    """Whether the Phase-1 cull takes its grouped search (the library's rule,
    restated on the host): at most 256 planes, one lane per Gaussian (the
    cull splits planes over lanes while n x lanes < 2^18), the per-plane flag
    unset, and at least eight valid planes sharing the bits of the normal row
    of R^-1 (computed as the library does, FP64 adjugate over determinant,
    then float, with -0 as +0) and of the origin's x and y.  Then the cull tests only the
    planes inside each Gaussian's window and its flop count is not N x P."""
    from paper_2505_05643_amd._lib import UG_FLAG_CULL_EACH_PLANE
    if pl.p > 256 or pl.p < 8 or (params.flags & UG_FLAG_CULL_EACH_PLANE):
        return False
    if pl.p > 1 and n < (1 << 18):
        return False
    groups = {}
    for q in range(pl.p):
        a, b, c, d, e, f, g_, h, i = (float(x) for x in pl.rot[q].astype(np.float64))
        det = a * (e * i - f * h) + b * (-(d * i - f * g_)) + c * (d * h - e * g_)
        if not (np.isfinite(det) and det > 0):
            continue
        r3 = np.array([(d * h - e * g_) / det, -(a * h - b * g_) / det, (a * e - b * d) / det], dtype=np.float32)
        r3 = r3 + np.float32(0.0)  # -0 as +0, as the library keys it
        key = (r3.tobytes(), pl.origin[q, 0].tobytes(), pl.origin[q, 1].tobytes())
        groups[key] = groups.get(key, 0) + 1
    return max(groups.values(), default=0) >= 8


def plan_bits(plan) -> int:
    t = max(plan.num_tiles, 2)
    return int(np.ceil(np.log2(t)))


def kernel_bytes(name, n, p, r, k, t, m, passes, w, rows, g_sort, dslots) -> int:
    """Algorithmic HBM bytes of one launch of an HBM-bound kernel: what the
    kernel must read and write once (N Gaussians, R records, K keys, T tiles,
    M pixels; W = 64-plane words per Gaussian; a sort pass reads and writes
    the key word, emission index and record id once, the first pass reading
    no emission index; the column scan reads and writes the block
    histograms of g_sort blocks x dslots digits)."""
    if name == "setup":
        return p * (56 + 160)
    if name == "cull_count":
        return 36 * n + 8 * n * w + 4 * n
    if name == "cull_write":
        return 4 * n + 8 * n * w + 8 * n + 8 * r
    if name == "record":
        return 8 * r + 44 * n + 52 * r + (16 * r if rows else 0)
    if name == "emit":
        return 4 * r + 16 * r + (48 * r if rows else 0) + 4 * r + 8 * k
    if name == "sort_hist":
        return 4 * k
    if name == "sort_scan":
        return 8 * dslots * g_sort
    if name == "sort_scatter":
        total = 20 * k + (passes - 1) * 24 * k
        return total // max(passes, 1)
    if name == "ranges":
        return 4 * k + 4 * t
    if name == "bwd_prep":
        return 20 * m
    if name == "record_adj":
        return 12 * r + 32 * k + 44 * n + 44 * n
    if name == "gauss_grad":
        return 12 * n + 44 * n
    return 0


def traffic_file(k: int) -> str:
    return os.path.join(ROOT, "profiles", f"hbm_traffic_per_kernel_c{k}.md")


def stored_traffic(kernel, k, params, plan):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a plain
    copy kernel), if they were taken on this workload and launch configuration
    with the current kernel sources; else None.  The summary file carries them
    on a line starting with "traffic-json: "."""
    try:
        with open(traffic_file(k)) as f:
            line = next((ln for ln in f if ln.startswith("traffic-json: ")), None)
        rec = json.loads(line[len("traffic-json: "):]) if line else {}
    except (OSError, ValueError):
        return None
    from paper_2505_05643_amd import _lib
    split = ":split" if params.flags & _lib.UG_FLAG_SPLIT_FORWARD else ""
    key = (f"c{k}:{kernel}:{params.tile_w}x{params.tile_h}x{plan_ppl(params)}:{params.lds_batch}:{params.box_mode}"
           f"{split}")
    if rec.get("sources") != sources_digest():
        return None
    return rec.get("bytes_per_launch", {}).get(key)


def sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_05643_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".h")):
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def plan_ppl(params) -> int:
    return params.px_per_lane or params.tile_w // 8


if __name__ == "__main__":
    main()
