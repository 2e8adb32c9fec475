"""Benchmark of the sparse-pixel training step on one MI355X.

Workload (rasterizer scaling): 300k Gaussians (means U[-1,1]^3, log-scales
N(-4, 0.5), random unit quaternions, opacity logits N(0,1), SH degree 3
N(0, 0.2)), one 1296x840 view, error-guided sampling of every tile at 25 %
(64 of 256 pixels per tile), Charbonnier + sparse NCC loss, adjoint backward
and the hybrid LM/Adam update.  A step runs every stage of the path: sample,
project, bin/sort, forward, loss, error/age update, backward, projection
backward, optimizer.  The dense GPU step (every pixel, same arithmetic) and
the 100/50/25/10 % sweep are reported beside it; the oracle is timed on the
host for a bounded sample of the same step.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N_GAUSS = 300_000
WIDTH, HEIGHT = 1296, 840
HEADLINE_RATE = 250          # per-mille of each tile's pixels
SWEEP_RATES = (1000, 500, 250, 100)
VALU_PEAK_TFLOPS = 157.3     # MI355X FP32 vector peak (packed); see DESIGN
HBM_PEAK_GBS = 8000.0

# Algorithmic FP32 operations per (Gaussian, pixel) pair of the forward
# compositing: an evaluation (offset, quadratic form, exp, alpha) and a
# blend (transmittance update and colour accumulation).
FWD_FLOP_EVAL = 14
FWD_FLOP_BLEND = 9
# Backward replay: the same evaluation, then per composited pair the
# transmittance/colour replay and the nine screen-space gradient terms.
BWD_FLOP_EVAL = 14
BWD_FLOP_BLEND = 48


# Matched-PSNR recovery task on the same scene: 100 cameras on the upper
# hemisphere (every fifth held out), targets rendered from the perturbed
# scene plus N(0, 0.01) noise, the model starting from the unperturbed one.
PSNR_CAMS = 100
PSNR_DENSE_STEPS = 500
PSNR_RATES = (500, 250, 200, 100)
PSNR_EVAL_EVERY = 25
PSNR_MAX_STEPS = 4000
TP_VIEWS = 40        # learned tile priority: training views
TP_STEPS = 600       # online steps
TP_EVAL_FROM = 400   # predictions scored from this step on
TP_LR = 3e-3
TP_SEED = 23

TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_scaling_300k_25pct.txt")
RASTER_SOURCES = ("paper_2606_15924_amd/csrc/raster.hip", "paper_2606_15924_amd/csrc/common.h")


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (already scaled by the plain-copy
    calibration), or None when there is no record for it or the kernel's
    source has changed since the counters were taken."""
    import hashlib
    try:
        rec = dict(line.split(": ", 1) for line in open(TRAFFIC_RECORD).read().splitlines()
                   if line.startswith("traffic-"))
    except OSError:
        return None
    h = hashlib.sha256()
    for f in RASTER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if rec.get("traffic-kernel") != kernel or rec.get("traffic-source-sha256") != h.hexdigest():
        return None
    return int(rec["traffic-read-bytes"]) + int(rec["traffic-write-bytes"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(dev):
    import torch

    import synth
    p = synth.gaussians(N_GAUSS, synth.SEED_SCENE)
    cam = synth.config_camera("scaling")
    gt = synth.image(HEIGHT, WIDTH, synth.SEED_NOISE)
    return p, cam, gt


def make_trainer(p, cam, gt, rate, dev, density_stats=False):
    import torch

    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    cfg = StepConfig(rate_permille=rate, density_stats=density_stats)
    E = torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev)
    A = torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev)
    tr = Trainer(torch.from_numpy(p).to(dev), [cam], [torch.from_numpy(gt).to(dev)], cfg, E=[E], A=[A])
    if rate is not None:
        tr.init_error_maps([0])
    return tr


def run(tr, steps, warmup):
    """Warmup, then an untimed pass with HIP events around every stage (the
    per-stage breakdown), then the timed steps.  Events cost the device a
    few microseconds each, so the timed steps bracket only the dominant
    raster kernel (for the roofline) and the step time is not inflated by
    the breakdown."""
    import torch
    for _ in range(warmup):
        tr.step([0])
    n_stage = max(20, steps // 2)
    tr.events = {}
    tr.timed_stages = None
    for _ in range(n_stage):
        tr.step([0])
    samples = tr.stage_samples_ms()
    stage = {k: sum(v) / n_stage for k, v in samples.items()}
    stage_spread = {k: {f"p{q}": round(float(np.percentile(v, q)), 4) for q in (10, 50, 90)}
                    for k, v in samples.items()}
    dom = max(("render_fwd", "render_bwd"), key=lambda k: stage.get(k, 0.0))
    tr.events = {}
    tr.timed_stages = {dom}
    tr.counters.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step([0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_ms = tr.stage_ms()[dom] / steps
    cnt = tr.counters.sum(dim=1).cpu().tolist()
    tr.events = None
    tr.timed_stages = None
    # spread of single steps: one event between consecutive steps (a pass of
    # its own, so the timed steps above carry no per-step events)
    n_dist = max(20, steps // 2)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_dist + 1)]
    evs[0].record()
    for k in range(n_dist):
        tr.step([0])
        evs[k + 1].record()
    torch.cuda.synchronize()
    per = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(n_dist))
    pct = {f"p{q}": round(per[min(n_dist - 1, int(q / 100 * n_dist))], 4) for q in (10, 50, 90)}
    vb = tr._bufs[0]
    pixels = (vb.width * vb.height) if vb.dense else int(vb.tile_off[-1].item())
    return dict(seconds=t1 - t0, ms_per_step=(t1 - t0) * 1000.0 / steps, evals=cnt[0], blends=cnt[1],
                stage_ms=stage, dominant=dom, dominant_ms=dom_ms, n_pairs=int(vb.n_pairs), pixels=pixels,
                step_ms_spread=pct, stage_ms_spread=stage_spread)


def matched_psnr(dev, dense_steps=PSNR_DENSE_STEPS, max_steps=PSNR_MAX_STEPS):
    """Dense training for ``dense_steps`` steps, then each sparse rate until
    its held-out PSNR reaches the dense run's final PSNR (or ``max_steps``).
    One random training view per step (seeded order, the same for every
    run); PSNR over the 20 held-out views every PSNR_EVAL_EVERY steps; only
    the training steps are clocked."""
    import torch

    import synth
    from paper_2606_15924_amd import binding as B
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer, ViewBuffers
    p0 = synth.gaussians(N_GAUSS, synth.SEED_SCENE)
    p_true = synth.perturb(p0, synth.SEED_PERTURB)
    cams = synth.hemisphere_cameras(PSNR_CAMS, width=WIDTH, height=HEIGHT, focal=300.0 * WIDTH / 256)
    held = [i for i in range(PSNR_CAMS) if i % 5 == 2]
    train = [i for i in range(PSNR_CAMS) if i % 5 != 2]
    rp = B.raster_params()
    vb = ViewBuffers(N_GAUSS, WIDTH, HEIGHT, None, -1, dev)

    def render(params, cam):
        c = B.camera(cam)
        vb.project(params, c, rp)
        vb.bin_sort(alpha_min=rp.alpha_min)
        vb.render_fwd(rp)
        return vb.out[: WIDTH * HEIGHT, :3].T.reshape(3, HEIGHT, WIDTH)

    P_true = torch.from_numpy(p_true).to(dev)
    gts = []
    for k, i in enumerate(range(PSNR_CAMS)):
        noise = torch.from_numpy(synth.pixel_noise((3, HEIGHT, WIDTH), synth.SEED_NOISE + k)).to(dev)
        gts.append((render(P_true, cams[i]) + noise).contiguous())
    del P_true

    def heldout_psnr(params):
        mse = 0.0
        for i in held:
            d = render(params, cams[i]) - gts[i]
            mse += float((d * d).mean())
        return 10.0 * np.log10(len(held) / mse)

    order = np.random.default_rng(synth.SEED_VIEWS).integers(0, len(train), size=max_steps)

    def run(rate, target_psnr, n_max, n_tiles_sel=-1, learned=False):
        cfg = StepConfig(rate_permille=rate, n_tiles_sel=n_tiles_sel, learned_tiles=learned)
        E = [torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev) for _ in train]
        A = [torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev) for _ in train]
        tr = Trainer(torch.from_numpy(p0).to(dev), [cams[i] for i in train], [gts[i] for i in train], cfg,
                     E=E, A=A)
        if rate is not None:
            tr.init_error_maps(range(len(train)))
        curve = [(0, 0.0, heldout_psnr(tr.params))]
        t_train, step = 0.0, 0
        while step < n_max:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(PSNR_EVAL_EVERY):
                tr.step([int(order[step])])
                step += 1
            torch.cuda.synchronize()
            t_train += time.perf_counter() - t0
            curve.append((step, t_train, heldout_psnr(tr.params)))
            if target_psnr is not None and curve[-1][2] >= target_psnr:
                break
        del tr
        return curve

    log(f"matched PSNR: dense {dense_steps} steps")
    dense = run(None, None, dense_steps)
    target = dense[-1][2]
    res = {"task": f"recovery of a perturbed {N_GAUSS}-Gaussian scene, {len(train)} training and "
                   f"{len(held)} held-out {WIDTH}x{HEIGHT} views, one view per step",
           "psnr_init": round(dense[0][2], 3),
           "dense": {"steps": dense[-1][0], "train_s": round(dense[-1][1], 4), "psnr": round(target, 3),
                     "ms_per_step": round(1e3 * dense[-1][1] / dense[-1][0], 4)},
           "sparse": {}}
    for r in PSNR_RATES:
        log(f"matched PSNR: sparse {r / 10:g}%")
        cv = run(r, target, max_steps)
        hit = cv[-1][2] >= target
        res["sparse"][f"{r / 10:g}%"] = {
            "steps_to_match": cv[-1][0] if hit else None, "train_s": round(cv[-1][1], 4),
            "psnr": round(cv[-1][2], 3), "ms_per_step": round(1e3 * cv[-1][1] / cv[-1][0], 4),
            "time_speedup_vs_dense": round(dense[-1][1] / cv[-1][1], 3) if hit else None}
    # a quarter of the tiles per step (64 samples each), drawn by the error-map
    # tile sums or by the learned tile priority
    n_t = ((WIDTH + 15) // 16) * ((HEIGHT + 15) // 16)
    res["quarter_tiles"] = {}
    for name, learned in (("error_map", False), ("learned", True)):
        log(f"matched PSNR: 25% of tiles, {name} tile pass")
        cv = run(250, target, max_steps, n_tiles_sel=n_t // 4, learned=learned)
        hit = cv[-1][2] >= target
        res["quarter_tiles"][name] = {
            "steps_to_match": cv[-1][0] if hit else None, "train_s": round(cv[-1][1], 4),
            "psnr": round(cv[-1][2], 3), "ms_per_step": round(1e3 * cv[-1][1] / cv[-1][0], 4),
            "time_speedup_vs_dense": round(dense[-1][1] / cv[-1][1], 3) if hit else None}
    return res


def tile_priority(dev, n_views=TP_VIEWS, steps=TP_STEPS, eval_from=TP_EVAL_FROM):
    """The learned tile-priority model trained online beside sparse training
    (25%, one view per step, seeded order) on the 300k-Gaussian recovery
    task.  Each step: the view's tile features are taken before the step
    (error and age maps as they were, pair counts of the step's binning), the
    model predicts each tile's error, the step runs, and the tile means of
    the updated error map are the targets of one training step.  Predictions
    made before training on a step are scored against that step's measured
    tile errors (Kendall tau, recall of the top quarter), next to the plain
    error-map predictor (the tile means before the step).  Kernel times from
    HIP events; the forward's FLOP count is 2 x rows x (32x64 + 64x64 + 64)."""
    import torch
    from scipy.stats import kendalltau

    import synth
    from paper_2606_15924_amd import binding as B
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer, ViewBuffers
    p0 = synth.gaussians(N_GAUSS, synth.SEED_SCENE)
    p_true = synth.perturb(p0, synth.SEED_PERTURB)
    cams = synth.hemisphere_cameras(n_views, width=WIDTH, height=HEIGHT, focal=300.0 * WIDTH / 256)
    rp = B.raster_params()
    vb = ViewBuffers(N_GAUSS, WIDTH, HEIGHT, None, -1, dev)
    P_true = torch.from_numpy(p_true).to(dev)
    gts = []
    for k, cam in enumerate(cams):
        vb.project(P_true, B.camera(cam), rp)
        vb.bin_sort(alpha_min=rp.alpha_min)
        vb.render_fwd(rp)
        noise = torch.from_numpy(synth.pixel_noise((3, HEIGHT, WIDTH), synth.SEED_NOISE + k)).to(dev)
        gts.append((vb.out[: WIDTH * HEIGHT, :3].T.reshape(3, HEIGHT, WIDTH) + noise).contiguous())
    del P_true, vb
    E = [torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev) for _ in cams]
    A = [torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev) for _ in cams]
    tr = Trainer(torch.from_numpy(p0).to(dev), cams, gts, StepConfig(rate_permille=250), E=E, A=A)
    tr.init_error_maps(range(n_views))
    bcams = [B.camera(c) for c in cams]
    n_t = ((WIDTH + 15) // 16) * ((HEIGHT + 15) // 16)
    params = torch.from_numpy(tile_init_params()).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    X = torch.empty((n_t, 32), dtype=torch.float32, device=dev)
    Xa = torch.empty_like(X)
    y = torch.empty(n_t, dtype=torch.float32, device=dev)
    act = torch.empty((n_t, 128), dtype=torch.float32, device=dev)
    ws = torch.empty(B.tgs_tile_mlp_workspace_size(n_t), dtype=torch.uint8, device=dev)
    order = np.random.default_rng(synth.SEED_VIEWS).integers(0, n_views, size=steps)
    k = n_t // 4
    scores = {"model": [], "error_map": []}
    for step in range(steps):
        vi = int(order[step])
        E0, A0 = E[vi].clone(), A[vi].clone()
        tr.step([vi])
        ranges = tr._bufs[0].ranges
        B.tgs_tile_features(ranges, E0, A0, HEIGHT, WIDTH, bcams[vi], X)
        B.tgs_tile_features(ranges, E[vi], A[vi], HEIGHT, WIDTH, bcams[vi], Xa)
        target = Xa[:, 19].contiguous()
        B.tgs_tile_mlp_fwd(params, X, n_t, y, act)
        if step >= eval_from:
            t_h, y_h, e_h = target.cpu().numpy(), y.cpu().numpy(), X[:, 19].cpu().numpy()
            top = set(np.argsort(-t_h, kind="stable")[:k].tolist())
            for name, pred in (("model", y_h), ("error_map", e_h)):
                rec = len(top & set(np.argsort(-pred, kind="stable")[:k].tolist())) / k
                scores[name].append((kendalltau(pred, t_h).statistic, rec))
        B.tgs_tile_mlp_train_step(params, m, v, X, act, y, target, n_t, step + 1, TP_LR, ws)
    torch.cuda.synchronize()
    del tr

    def timed(fn, reps=50):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    flop_row = 2 * (32 * 64 + 64 * 64 + 64)
    fwd_ms = timed(lambda: B.tgs_tile_mlp_fwd(params, X, n_t, y, act))
    nb = 1 << 20
    Xb = torch.randn((nb, 32), dtype=torch.float32, device=dev)
    yb = torch.empty(nb, dtype=torch.float32, device=dev)
    big_ms = timed(lambda: B.tgs_tile_mlp_fwd(params, Xb, nb, yb, None))
    train_ms = timed(lambda: B.tgs_tile_mlp_train_step(params, m, v, X, act, y, target, n_t, steps + 1, 0.0, ws))
    feat_ms = timed(lambda: B.tgs_tile_features(ranges, E[0], A[0], HEIGHT, WIDTH, bcams[0], X))
    res = {"task": f"online beside sparse 25% training, {n_views} views, {steps} steps; "
                   f"predictions scored before each training step from step {eval_from}",
           "kendall_tau": {kk: round(float(np.mean([s[0] for s in vv])), 4) for kk, vv in scores.items()},
           "top_quarter_recall": {kk: round(float(np.mean([s[1] for s in vv])), 4) for kk, vv in scores.items()},
           "features_ms": round(feat_ms, 4), "train_step_ms": round(train_ms, 4),
           "fwd_ms": round(fwd_ms, 4), "fwd_rows": n_t,
           "fwd_roofline": {"bound": "mfma", "rows": nb, "ms": round(big_ms, 4),
                            "achieved": round(flop_row * nb / (big_ms * 1e-3) / 1e12, 3), "peak": 2500.0,
                            "unit": "TFLOP/s",
                            "frac": round(flop_row * nb / (big_ms * 1e-3) / 1e12 / 2500.0, 5)}}
    return res


def tile_init_params():
    """Seeded initial weights of the tile-priority model: N(0, 1/fan_in)
    hidden weights, zero biases and output layer (it starts as the error-map
    predictor)."""
    import math
    rng = np.random.default_rng(TP_SEED)
    p = np.zeros(6337, dtype=np.float32)
    p[0:2048] = rng.normal(0.0, 1.0 / math.sqrt(32), 2048)
    p[2112:6208] = rng.normal(0.0, 1.0 / math.sqrt(64), 4096)
    return p


def cpu_baseline(p, cam, gt, target_s=15.0):
    """The oracle's sparse step, timed on one host thread: the parts whose
    cost scales with the sampled tiles (sampling, forward, loss, backward)
    on a random subset of tiles at the headline rate, the parts over every
    Gaussian (projection, binning of the whole view, projection backward,
    optimizer) whole.
    The subset is sized from a 32-tile probe so the tile part takes about
    ``target_s`` seconds.  The whole-view step time is extrapolated as
    fixed + per-tile x n_t / n_tiles, and so are its blends; returns
    blends/s of that step."""
    from threadpoolctl import threadpool_limits

    from oracle import binning, loss, project, project_bwd, render, sampler, optim
    from oracle.params import OptimParams, RasterParams, SampleParams
    import synth
    rp = RasterParams()
    E = synth.error_map(HEIGHT, WIDTH, 31)
    A = np.zeros((HEIGHT, WIDTH), dtype=np.uint16)
    TX, TY = (WIDTH + 15) // 16, (HEIGHT + 15) // 16
    n_t = TX * TY
    order = np.random.default_rng(0).permutation(n_t)

    def tile_part(pr, sv, ranges, tiles):
        s = sampler.sample_view(E, A, SampleParams(n_pix=64), 3, 1, 0, tiles_subset=tiles)
        xs, ys, _ = sampler.sample_coords(s, WIDTH, HEIGHT)
        out = render.render_pixels(pr, sv, ranges, xs, ys, rp)
        ls = loss.sparse_loss(out["rgb"], gt[:, ys, xs].T, s["tile_off"], xs.size, s["valid_tiles"].size)
        g2d = render.render_pixels_bwd(pr, sv, ranges, xs, ys, ls["dL"], rp)
        return xs, out, g2d

    with threadpool_limits(1):
        c0 = time.perf_counter()
        pr = project.project(p, cam, rp)
        # every tile of the view is sampled at this rate: the lists cover the view
        _, sv, ranges = binning.bin_and_sort(pr, np.arange(n_t))
        c1 = time.perf_counter()
        tile_part(pr, sv, ranges, np.sort(order[:32]))
        probe = (time.perf_counter() - c1) / 32
        n_tiles = int(min(n_t, max(32, target_s / probe)))
        tiles = np.sort(order[:n_tiles])
        c1b = time.perf_counter()
        xs, out, g2d = tile_part(pr, sv, ranges, tiles)
        c2 = time.perf_counter()
        grad = project_bwd.project_bwd(p, cam, pr, g2d, rp)
        touched = np.zeros(p.shape[1], dtype=bool)
        touched[np.unique(sv)] = True
        optim.optimizer_step(p, grad, np.zeros_like(grad), np.zeros_like(grad), touched, OptimParams(), 1)
        c3 = time.perf_counter()
    fixed = (c1 - c0) + (c3 - c2)
    per_tile = (c2 - c1b) / n_tiles
    step_s = fixed + per_tile * n_t
    blends = int(out["n_blend"].sum())
    blends_step = blends * n_t / n_tiles
    return dict(value=blends_step / step_s, unit="blends/s", cores=1, kind="oracle",
                step_s_extrapolated=round(step_s, 2),
                sample=f"{n_tiles} of {n_t} random tiles at 25% ({xs.size} pixels, {blends} blends) plus "
                       f"projection, whole-view binning, projection backward and optimizer over all "
                       f"{p.shape[1]} Gaussians; "
                       f"{fixed + (c2 - c1b):.1f} s measured ({fixed:.1f} s whole-model, "
                       f"{per_tile * 1e3:.1f} ms per tile), whole-view step extrapolated to {step_s:.1f} s")


def density_control(p, cam, gt, dev, blends_per_step):
    """The density-control statistics beside the headline step: the step
    with the back-projection fused into the backward, that backward's time,
    the standalone back-projection kernel on the same samples, and the score
    plus both percentile selections over all Gaussians."""
    import torch
    tr = make_trainer(p, cam, gt, HEADLINE_RATE, dev, density_stats=True)
    res = run(tr, 20, 3)
    vb = tr._bufs[0]

    def standalone():
        vb.density(tr.rp, tr.dstats)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    standalone()
    a.record()
    for _ in range(20):
        standalone()
    b.record()
    torch.cuda.synchronize()
    acc_ms = a.elapsed_time(b) / 20
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tr.density_select(0.5, 0.3, 0.9, 0.85)
    reps = 20
    a.record()
    for _ in range(reps):
        tr.density_select(0.5, 0.3, 0.9, 0.85)
    b.record()
    torch.cuda.synchronize()
    sel_ms = a.elapsed_time(b) / reps
    del tr
    return {"step_ms_with_accumulation": round(res["ms_per_step"], 4),
            "render_bwd_with_accumulation_ms": round(res["stage_ms"]["render_bwd"], 4),
            "standalone_accumulate_ms": round(acc_ms, 4),
            "standalone_accumulate_blends_per_s": blends_per_step / (acc_ms * 1e-3),
            "score_and_selections_ms": round(sel_ms, 4),
            "selection": "densify top 10% (eta_topk 0.9), keep top 85% (eta_final 0.85) of 300k scores"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-sweep", action="store_true", help="skip the pixel-rate sweep and dense run")
    ap.add_argument("--no-psnr", action="store_true", help="skip the matched-PSNR training comparison")
    ap.add_argument("--no-tile", action="store_true", help="skip the learned tile-priority measurement")
    ap.add_argument("--no-density", action="store_true", help="skip the density-control measurement")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU split by "
              f"views is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.calib_copy_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log("building workload")
    p, cam, gt = make_workload(dev)

    log(f"sparse {HEADLINE_RATE / 10:.0f}% run: {args.warmup} warmup + {args.steps} timed steps")
    tr = make_trainer(p, cam, gt, HEADLINE_RATE, dev)
    head = run(tr, args.steps, args.warmup)
    log(f"  {head['ms_per_step']:.3f} ms/step, stages {head['stage_ms']}")
    del tr

    sweep = {}
    dense = None
    if not args.no_sweep:
        for r in SWEEP_RATES:
            if r == HEADLINE_RATE:
                sweep[f"{r / 10:g}%"] = dict(ms_per_step=head["ms_per_step"],
                                             blends_per_s=head["blends"] / head["seconds"])
                continue
            log(f"sweep {r / 10:g}%")
            tr = make_trainer(p, cam, gt, r, dev)
            res = run(tr, max(5, args.steps // 2), 2)
            sweep[f"{r / 10:g}%"] = dict(ms_per_step=res["ms_per_step"], blends_per_s=res["blends"] / res["seconds"])
            del tr
        log("dense run")
        tr = make_trainer(p, cam, gt, None, dev)
        dres = run(tr, max(5, args.steps // 2), 2)
        dense = dict(ms_per_step=dres["ms_per_step"], blends_per_s=dres["blends"] / dres["seconds"],
                     stage_ms=dres["stage_ms"])
        del tr

    # roofline of the dominant kernel of the headline step, timed inside the timed steps
    dom = head["dominant"]
    per_launch_evals = head["evals"] / args.steps
    per_launch_blends = head["blends"] / args.steps
    if dom == "render_fwd":
        flops = FWD_FLOP_EVAL * per_launch_evals + FWD_FLOP_BLEND * per_launch_blends
    else:
        flops = BWD_FLOP_EVAL * per_launch_evals + BWD_FLOP_BLEND * per_launch_blends
    achieved = flops / (head["dominant_ms"] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(dom), "launch_ms": round(head["dominant_ms"], 4)}

    dens = None
    if not args.no_density:
        log("density-control statistics")
        dens = density_control(p, cam, gt, dev, per_launch_blends)

    tile = None
    if not args.no_tile:
        log("learned tile priority")
        tile = tile_priority(dev)
    psnr = None
    if not args.no_psnr:
        psnr = matched_psnr(dev)

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline")
        cpu = cpu_baseline(p, cam, gt)

    value = head["blends"] / head["seconds"]
    line = {
        "metric": "ms/train-step & Gaussian-pixel blends/s, sparse vs dense GPU at matched PSNR",
        "value": value,
        "unit": "blends/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rasterizer scaling: 300k Gaussians, one 1296x840 view, "
                               "25% error-guided pixels per tile, full training step",
                   "gaussians": N_GAUSS, "width": WIDTH, "height": HEIGHT, "rate": 0.25,
                   "pairs": head["n_pairs"], "parallelism": "single GPU"},
        "stage_ms": {k: round(v, 4) for k, v in head["stage_ms"].items()},
        "step_ms_spread": head["step_ms_spread"],
        "stage_ms_spread": head["stage_ms_spread"],
        # blends per second of the raster kernels alone (forward; forward + backward)
        "blends_per_s_fwd": per_launch_blends / (1e-3 * head["stage_ms"]["render_fwd"]),
        "blends_per_s_fwd_bwd": per_launch_blends / (1e-3 * (head["stage_ms"]["render_fwd"] +
                                                            head["stage_ms"]["render_bwd"])),
        "per_step": {"evaluations": per_launch_evals, "blends": per_launch_blends,
                     "sampled_pixels": head["pixels"]},
        "dense": dense,
        "sparse_vs_dense_speedup": (dense["ms_per_step"] / head["ms_per_step"]) if dense else None,
        "sweep": sweep or None,
        "roofline": roofline,
        "matched_psnr": psnr,
        "tile_priority": tile,
        "density_control": dens,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
