"""Benchmark of the sparse-pixel training step on one MI355X.

Headline workload (full training step): 1.5M Gaussians (means U[-1,1]^3,
log-scales N(-4, 0.5), random unit quaternions, opacity logits N(0,1), SH
degree 3 N(0, 0.2)), 150 cameras of 1600x1060 (f = 1875) on the upper
hemisphere of radius 3, targets rendered densely from a seed-perturbed copy
of the scene plus N(0, 0.01) noise, error maps initialised from the dense L1
error of the initial model.  Each step trains K views (K = 3 and K = 10, a
seeded random choice of distinct views per step) with error-guided sampling
of 20 % of every tile's pixels (51 of 256), Charbonnier + sparse NCC loss,
adjoint backward and the hybrid LM/Adam update.  A step runs every stage of
the path for each view: sample, project, bin/sort, forward, loss, error/age
update, backward, projection backward; then the update.  The dense GPU step
(every pixel, same arithmetic) at the same K is reported beside it.

Beside the headline: the rasterizer-scaling workload (300k Gaussians, one
1296x840 view) at 100/50/25/10 % and dense, the density-control and
learned tile-priority measurements and the matched-PSNR comparison on it;
the oracle timed on the host for a bounded sample of one view of the full
step, on one thread and on every core the process may use.

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

# full training step
FULL_N = 1_500_000
FULL_VIEWS = 150
FULL_W, FULL_H = 1600, 1060
FULL_RATE = 200              # per-mille of each tile's pixels (51 of 256)
FULL_K = (3, 10)             # views per step (the schedule's K_min and K_max)
HEADLINE_K = 3
FULL_PREFIX = 0.15           # depth-prefix lists: the nearest 15% of the Gaussians, then a continuation
PREFIX = FULL_PREFIX         # the full step's setting (--no-prefix: whole lists)
# The 300k-Gaussian workloads keep whole lists: their lists are short (2.1M
# pairs per view), where the prefix's extra launches cost more than the
# shorter lists save (binning 0.32 against 0.24 ms per view).
FULL_VIEW_STREAMS = 3        # the full step's views side by side (projection to loss), one stream each

# large scene: 5M Gaussians in a 50-unit corridor, 400 cameras 1920x1080 along it
LARGE_N = 5_000_000
LARGE_VIEWS = 400
LARGE_W, LARGE_H = 1920, 1080
LARGE_RATE = 200             # per-mille of each selected tile's pixels (51 of 256)
LARGE_TILE_FRAC = 0.75       # tiles drawn per view by the learned tile priority: 0.75 x 20% = 15% of the pixels
LARGE_K = 3
LARGE_STEPS = 3000

# rasterizer scaling
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

TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_full_step_1p5m_20pct.txt")
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
    cfg = StepConfig(rate_permille=rate, density_stats=density_stats, fuse_views=True)
    E = torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev)
    A = torch.zeros((HEIGHT, WIDTH), dtype=torch.int16, device=dev)
    tr = Trainer(torch.from_numpy(p).to(dev), [cam], [torch.from_numpy(gt).to(dev)], cfg, E=[E], A=[A])
    if rate is not None:
        tr.init_error_maps([0])
    return tr


def run(tr, steps, warmup, views_of=None):
    """Warmup, then an untimed pass with HIP events around every stage (the
    per-stage breakdown), then the timed steps.  Events cost the device a
    few microseconds each, so the timed steps bracket only the dominant
    raster kernel (for the roofline) and the step time is not inflated by
    the breakdown.  ``views_of(i)`` gives the views of the i-th step (one
    view, 0, when None); every pass draws from the same sequence."""
    import torch
    calls = [0]

    def step():
        v = [0] if views_of is None else views_of(calls[0])
        calls[0] += 1
        tr.step(v)
    for _ in range(warmup):
        step()
    n_stage = max(20, steps // 2)
    tr.events = {}
    tr.timed_stages = None
    for _ in range(n_stage):
        step()
    samples = tr.stage_samples_ms()
    stage = {k: sum(v) / n_stage for k, v in samples.items()}
    stage_spread = {k: {f"p{q}": round(float(np.percentile(v, q)), 4) for q in (10, 50, 90)}
                    for k, v in samples.items()}
    # with views side by side the forward shares the GPU with other views'
    # binning, so its event times are not kernel times; the backward runs
    # alone on the main stream
    dom = "render_bwd" if tr.cfg.view_streams > 1 else max(("render_fwd", "render_bwd"),
                                                            key=lambda k: stage.get(k, 0.0))
    tr.events = {}
    tr.timed_stages = {dom}
    tr.counters.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches = len(tr.events.get(dom, []))
    dom_ms = tr.stage_ms()[dom] / max(launches, 1)
    cnt = tr.counters.sum(dim=1).cpu().tolist()
    tr.events = None
    tr.timed_stages = None
    # spread of single steps: one event between consecutive steps (a pass of
    # its own, so the timed steps above carry no per-step events)
    n_dist = max(20, steps // 2)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_dist + 1)]
    evs[0].record()
    for k in range(n_dist):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    per = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(n_dist))
    pct = {f"p{q}": round(per[min(n_dist - 1, int(q / 100 * n_dist))], 4) for q in (10, 50, 90)}
    pixels = 0
    n_pairs = 0
    for vb in tr._bufs.values():
        pixels += (vb.width * vb.height) if vb.dense else int(vb.tile_off[-1].item())
        n_pairs += int(vb.n_pairs)
    return dict(seconds=t1 - t0, ms_per_step=(t1 - t0) * 1000.0 / steps, evals=cnt[0], blends=cnt[1],
                stage_ms=stage, dominant=dom, dominant_ms=dom_ms, launches_per_step=launches / steps,
                n_pairs=n_pairs, pixels=pixels, step_ms_spread=pct, stage_ms_spread=stage_spread)


# ------------------------------------------------------------------ full training step
def full_workload(dev):
    """The full-step scene on the device: parameters, cameras, dense
    targets of the perturbed scene plus seeded N(0, 0.01) noise."""
    import torch

    import synth
    from paper_2606_15924_amd import binding as B
    from paper_2606_15924_amd.pipeline import ViewBuffers
    p = synth.gaussians(FULL_N, synth.SEED_SCENE)
    cams = synth.hemisphere_cameras(FULL_VIEWS, width=FULL_W, height=FULL_H)
    P_true = torch.from_numpy(synth.perturb(p, synth.SEED_PERTURB)).to(dev)
    rp = B.raster_params()
    vb = ViewBuffers(FULL_N, FULL_W, FULL_H, None, -1, dev)
    gen = torch.Generator(device=dev)
    gts = []
    for k, cam in enumerate(cams):
        vb.project(P_true, B.camera(cam), rp)
        vb.bin_sort(alpha_min=rp.alpha_min)
        vb.render_fwd(rp)
        gen.manual_seed(synth.SEED_NOISE * 1000 + k)
        img = vb.out[: FULL_W * FULL_H, :3].T.reshape(3, FULL_H, FULL_W)
        gts.append((img + 0.01 * torch.randn(img.shape, generator=gen, device=dev)).contiguous())
    del P_true, vb
    torch.cuda.synchronize()
    return p, cams, gts


def full_trainer(p, cams, gts, rate, dev, prefix=FULL_PREFIX):
    import torch

    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    cfg = StepConfig(rate_permille=rate, prefix_fraction=prefix, fuse_views=True, view_streams=FULL_VIEW_STREAMS)
    E = [torch.zeros((FULL_H, FULL_W), dtype=torch.int16, device=dev) for _ in cams]
    A = [torch.zeros((FULL_H, FULL_W), dtype=torch.int16, device=dev) for _ in cams]
    tr = Trainer(torch.from_numpy(p).to(dev), cams, gts, cfg, E=E, A=A)
    if rate is not None:
        tr.init_error_maps(range(len(cams)))
    return tr


def view_order(K, n_views=FULL_VIEWS):
    """Seeded choice of K distinct views for each step (the same sequence
    for every run, sparse or dense)."""
    import synth
    rng = np.random.default_rng(synth.SEED_VIEWS)
    seq = [rng.choice(n_views, K, replace=False).tolist() for _ in range(1024)]
    return lambda i: seq[i % len(seq)]


def full_step(dev, steps, warmup, with_dense=True, prefix=FULL_PREFIX):
    """Sparse (20 %) and dense steps at K = 3 and K = 10."""
    import torch
    log("full step: building the 1.5M-Gaussian scene and 150 targets")
    p, cams, gts = full_workload(dev)
    res = {}
    for K in FULL_K:
        for name, rate in (("sparse", FULL_RATE), ("dense", None)):
            if name == "dense" and not with_dense:
                continue
            log(f"full step K={K} {name}: {warmup} warmup + {steps} timed steps")
            tr = full_trainer(p, cams, gts, rate, dev, prefix)
            r = run(tr, steps, warmup, view_order(K))
            log(f"  {r['ms_per_step']:.3f} ms/step, stages {r['stage_ms']}")
            res[(K, name)] = r
            del tr
            torch.cuda.empty_cache()
    return p, cams, res


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
        cfg = StepConfig(rate_permille=rate, n_tiles_sel=n_tiles_sel, learned_tiles=learned,
                         fuse_views=True)
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


# ------------------------------------------------------------------ large scene
def large_scene(dev, steps):
    """Sparse training on the large scene: 5M Gaussians in a corridor, 400
    cameras 1920x1080 along a 50-unit trajectory, targets rendered densely
    from a seed-perturbed copy plus N(0, 0.01) noise.  Each step trains K = 3
    views picked by the anchor and geometry-aware companion draws from the
    views' mean errors (refreshed after every step); each view samples three
    quarters of its tiles by the learned tile priority at 20% of their
    pixels (15% of the image) and the priority network trains online; the
    backward accumulates the density statistics, and density control runs
    every 100 steps from step 200 to 2500 (densify the top 2% of the scores
    that pass the gradient gates, prune the bottom 5% every 500 steps).
    Reports step time p50/p99 over the training steps (density steps
    timed apart), the Gaussian count and the peak device memory."""
    import math

    import torch

    import synth
    from paper_2606_15924_amd import binding as B
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer, ViewBuffers
    from paper_2606_15924_amd.schedule import DensityPlan, camera_pose, density_step, pick_views, scene_extent, \
        view_errors
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    p = synth.corridor_gaussians(LARGE_N, synth.SEED_SCENE)
    cams = synth.trajectory_cameras(LARGE_VIEWS, width=LARGE_W, height=LARGE_H)
    P_true = torch.from_numpy(synth.perturb(p, synth.SEED_PERTURB)).to(dev)
    rp = B.raster_params()
    vb = ViewBuffers(LARGE_N, LARGE_W, LARGE_H, None, -1, dev)
    gen = torch.Generator(device=dev)
    gts = []
    for k, cam in enumerate(cams):
        vb.project(P_true, B.camera(cam), rp)
        vb.bin_sort(alpha_min=rp.alpha_min)
        vb.render_fwd(rp)
        gen.manual_seed(synth.SEED_NOISE * 1000 + k)
        img = vb.out[: LARGE_W * LARGE_H, :3].T.reshape(3, LARGE_H, LARGE_W)
        gts.append((img + 0.01 * torch.randn(img.shape, generator=gen, device=dev)).contiguous())
    del P_true, vb
    n_t = ((LARGE_W + 15) // 16) * ((LARGE_H + 15) // 16)
    cfg = StepConfig(rate_permille=LARGE_RATE, n_tiles_sel=int(LARGE_TILE_FRAC * n_t), learned_tiles=True,
                     density_stats=True, fuse_views=True, view_streams=FULL_VIEW_STREAMS)
    E = [torch.zeros((LARGE_H, LARGE_W), dtype=torch.int16, device=dev) for _ in cams]
    A = [torch.zeros((LARGE_H, LARGE_W), dtype=torch.int16, device=dev) for _ in cams]
    tr = Trainer(torch.from_numpy(p).to(dev), cams, gts, cfg, E=E, A=A)
    tr.init_error_maps(range(len(cams)))
    plan = DensityPlan(t_from=200, t_until=2500, every=100, prune_every=500, eta_topk=0.98, eta_final=0.95)
    poses = [camera_pose(c) for c in tr.cams]
    centres, dirs = [q[0] for q in poses], [q[1] for q in poses]
    pixels = LARGE_W * LARGE_H
    means = view_errors(tr.E, pixels, dev)
    extent = scene_extent(tr.cams)
    stack = list(range(len(cams)))
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    dens = []
    n_start = tr.n
    t0 = time.perf_counter()
    ev[0].record()
    for t in range(1, steps + 1):
        views, stack = pick_views(stack, means, centres, dirs, LARGE_K, 0.05, 1.0, synth.SEED_VIEWS, t)
        tr.step(views)
        ev[t].record()
        if plan.t_from <= t <= plan.t_until and t % plan.every == 0:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            density_step(tr, t, plan.t_until, plan, extent)
            b.record()
            dens.append((a, b))
        means = view_errors(tr.E, pixels, dev, views, means)
        if t % 500 == 0:
            log(f"  large scene step {t}: {tr.n} Gaussians")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dens_ms = [a.elapsed_time(b) for a, b in dens]
    # a step's span ends at its own event; a density step in between is timed apart
    per = np.array([ev[t - 1].elapsed_time(ev[t]) for t in range(1, steps + 1)])
    dens_steps = [t for t in range(1, steps + 1) if plan.t_from <= t - 1 <= plan.t_until and (t - 1) % plan.every == 0]
    train = np.delete(per, [t - 1 for t in dens_steps])
    peak = torch.cuda.max_memory_allocated()
    res = {"workload": f"{LARGE_N} Gaussians in a 50-unit corridor, {LARGE_VIEWS} cameras {LARGE_W}x{LARGE_H} "
                       f"along it, K={LARGE_K} views per step, {int(LARGE_TILE_FRAC * 100)}% of tiles by the "
                       f"learned priority at {LARGE_RATE / 10:g}% of their pixels, density control",
           "steps": steps, "wall_s": round(wall, 2),
           "step_ms": {"p50": round(float(np.percentile(train, 50)), 4),
                       "p99": round(float(np.percentile(train, 99)), 4),
                       "mean": round(float(train.mean()), 4)},
           "density_steps": len(dens_ms), "density_ms_mean": round(float(np.mean(dens_ms)), 4) if dens_ms else None,
           "gaussians_start": n_start, "gaussians_end": tr.n,
           "peak_hbm_gb": round(peak / 2 ** 30, 2)}
    del tr, gts, E, A
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------ oracle on the host
_CPU = {}   # the oracle baseline's shared inputs (inherited by forked workers)


def _gauss_chunks(n, parts):
    edges = np.linspace(0, n, parts + 1).astype(np.int64)
    return [(int(edges[k]), int(edges[k + 1])) for k in range(parts)]


def _slice_proj(pr, lo, hi, n):
    return {k: (v[..., lo:hi] if isinstance(v, np.ndarray) and v.shape[-1] == n else v) for k, v in pr.items()}


def _w_project(lohi):
    from threadpoolctl import threadpool_limits

    from oracle import project
    lo, hi = lohi
    with threadpool_limits(1):
        return project.project(_CPU["p"][:, lo:hi], _CPU["cam"], _CPU["rp"])


def _w_tiles(tiles):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        xs, out, g2d = _cpu_tile_part(_CPU["pr"], _CPU["sv"], _CPU["ranges"], np.asarray(tiles))
    nz = np.nonzero(np.any(g2d != 0, axis=0))[0]
    return int(out["n_blend"].sum()), int(xs.size), nz, g2d[:, nz]


def _w_backward(lohi):
    from threadpoolctl import threadpool_limits

    from oracle import optim, project_bwd
    from oracle.params import OptimParams
    lo, hi = lohi
    n = _CPU["p"].shape[1]
    with threadpool_limits(1):
        p = _CPU["p"][:, lo:hi]
        grad = project_bwd.project_bwd(p, _CPU["cam"], _slice_proj(_CPU["pr"], lo, hi, n),
                                       _CPU["g2d"][:, lo:hi], _CPU["rp"])
        z = np.zeros_like(grad)
        optim.optimizer_step(p, grad, z, z, _CPU["touched"][lo:hi], OptimParams(), 1)
    return hi - lo


def _cpu_tile_part(pr, sv, ranges, tiles):
    from oracle import loss, render, sampler
    from oracle.params import SampleParams
    n_pix = (FULL_RATE * 256) // 1000
    s = sampler.sample_view(_CPU["E"], _CPU["A"], SampleParams(n_pix=n_pix), 3, 1, 0, tiles_subset=tiles)
    xs, ys, _ = sampler.sample_coords(s, FULL_W, FULL_H)
    out = render.render_pixels(pr, sv, ranges, xs, ys, _CPU["rp"])
    ls = loss.sparse_loss(out["rgb"], _CPU["gt"][:, ys, xs].T, s["tile_off"], xs.size, s["valid_tiles"].size)
    g2d = render.render_pixels_bwd(pr, sv, ranges, xs, ys, ls["dL"], _CPU["rp"])
    return xs, out, g2d


def cpu_baseline(p, cam, target_s=15.0, cores=1):
    """The oracle's sparse step for one view of the full training step, timed
    on the host: projection, binning of the whole view (the rectangle lists
    of every tile), sampling + forward + loss + backward on a random subset
    of tiles sized from a 16-tile probe so that part takes about
    ``target_s`` seconds of one thread's work, then projection backward and
    the update over every Gaussian.  The view's step time is extrapolated
    as whole-model parts + per-tile time x tiles, and so are its blends;
    the K-view step as K views plus nothing else shared.  With ``cores`` > 1
    the independent work (Gaussian ranges of the projection, backward and
    update; tiles of the tile part) is split over that many forked worker
    processes of one thread each; binning runs in one process."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    import synth
    from oracle import binning
    from oracle.params import RasterParams
    rp = RasterParams()
    n = p.shape[1]
    TX, TY = (FULL_W + 15) // 16, (FULL_H + 15) // 16
    n_t = TX * TY
    order = np.random.default_rng(0).permutation(n_t)
    _CPU.update(p=p, cam=cam, rp=rp, E=synth.error_map(FULL_H, FULL_W, 31),
                A=np.zeros((FULL_H, FULL_W), dtype=np.uint16), gt=synth.image(FULL_H, FULL_W, 32))
    ctx = mp.get_context("fork")

    def pmap(fn, items):
        # a fresh pool per phase: workers fork after that phase's inputs are in place
        with ctx.Pool(cores) as pool:
            return pool.map(fn, items)
    try:
        with threadpool_limits(1):
            c0 = time.perf_counter()
            if cores == 1:
                pr = _w_project((0, n))
            else:
                parts = pmap(_w_project, _gauss_chunks(n, cores))
                pr = {k: (np.concatenate([q[k] for q in parts], axis=-1)
                          if isinstance(parts[0][k], np.ndarray) and parts[0][k].shape[-1] == parts[0]["opacity"].size
                          else parts[0][k]) for k in parts[0]}
            c1 = time.perf_counter()
            _, sv, ranges = binning.bin_and_sort(pr, np.arange(n_t))
            c2 = time.perf_counter()
            _CPU.update(pr=pr, sv=sv, ranges=ranges)
            _cpu_tile_part(pr, sv, ranges, np.sort(order[:16]))
            probe = (time.perf_counter() - c2) / 16
            n_tiles = int(min(n_t, max(16, target_s / probe)))
            tiles = np.sort(order[:n_tiles])
            c3 = time.perf_counter()
            g2d = np.zeros((9, n))
            if cores == 1:
                res = [_w_tiles(tiles)]
            else:
                res = pmap(_w_tiles, np.array_split(tiles, cores * 4))
            blends = sum(r[0] for r in res)
            pixels = sum(r[1] for r in res)
            for r in res:
                g2d[:, r[2]] += r[3]
            c4 = time.perf_counter()
            touched = np.zeros(n, dtype=bool)
            touched[np.unique(sv)] = True
            _CPU.update(g2d=g2d, touched=touched)
            if cores == 1:
                _w_backward((0, n))
            else:
                pmap(_w_backward, _gauss_chunks(n, cores))
            c5 = time.perf_counter()
    finally:
        _CPU.clear()
    whole = (c1 - c0) + (c2 - c1) + (c5 - c4)
    per_tile = (c4 - c3) / n_tiles
    view_s = whole + per_tile * n_t
    blends_view = blends * n_t / n_tiles
    step_s = HEADLINE_K * view_s
    return dict(value=blends_view * HEADLINE_K / step_s, unit="blends/s", cores=cores, kind="oracle",
                step_s_extrapolated=round(step_s, 2), view_s_extrapolated=round(view_s, 2),
                sample=f"one 1600x1060 view of the 1.5M-Gaussian full step: {n_tiles} of {n_t} random tiles at "
                       f"20% ({pixels} pixels, {blends} blends), plus projection ({c1 - c0:.1f} s), "
                       f"whole-view binning ({c2 - c1:.1f} s, one process), projection backward and update "
                       f"({c5 - c4:.1f} s) over all {n} Gaussians; {c5 - c0:.1f} s measured, "
                       f"{per_tile * 1e3:.1f} ms per tile; the K={HEADLINE_K} step extrapolated to "
                       f"{step_s:.1f} s")


def host_cores() -> int:
    """Cores this process may use, at most 16 (one GPU's share of the host)."""
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


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


def summarize(r, steps):
    """The per-run figures reported for a step configuration."""
    out = dict(ms_per_step=round(r["ms_per_step"], 4), step_ms_spread=r["step_ms_spread"],
               blends_per_s=r["blends"] / r["seconds"], blends_per_step=r["blends"] / steps,
               evaluations_per_step=r["evals"] / steps, sampled_pixels_per_step=r["pixels"],
               pairs_per_step=r["n_pairs"], stage_ms_per_step={k: round(v, 4) for k, v in r["stage_ms"].items()})
    fwd = r["stage_ms"].get("render_fwd")
    bwd = r["stage_ms"].get("render_bwd")
    if fwd:
        out["blends_per_s_fwd"] = (r["blends"] / steps) / (1e-3 * fwd)
        if bwd:
            out["blends_per_s_fwd_bwd"] = (r["blends"] / steps) / (1e-3 * (fwd + bwd))
    return out


def roofline_of(r, steps):
    """Roofline of the dominant raster kernel of a run, from the kernel's
    average launch time measured with HIP events on its stream over the
    timed steps and the algorithmic FLOP of one launch."""
    dom = r["dominant"]
    launches = max(r["launches_per_step"] * steps, 1)
    ev, bl = r["evals"] / launches, r["blends"] / launches
    if dom == "render_fwd":
        flops = FWD_FLOP_EVAL * ev + FWD_FLOP_BLEND * bl
    else:
        flops = BWD_FLOP_EVAL * ev + BWD_FLOP_BLEND * bl
    achieved = flops / (r["dominant_ms"] * 1e-3) / 1e12
    return {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 4),
            "traffic": measured_traffic(dom), "launch_ms": round(r["dominant_ms"], 4),
            "flop_per_launch": round(flops), "evaluations_per_launch": round(ev), "blends_per_launch": round(bl)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense full steps")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 300k pixel-rate sweep and dense run")
    ap.add_argument("--no-psnr", action="store_true", help="skip the matched-PSNR training comparison")
    ap.add_argument("--no-tile", action="store_true", help="skip the learned tile-priority measurement")
    ap.add_argument("--no-density", action="store_true", help="skip the density-control measurement")
    ap.add_argument("--only-headline", action="store_true", help="the K=3 sparse full step alone (profiling)")
    ap.add_argument("--no-prefix", action="store_true", help="whole lists instead of depth-prefix lists")
    ap.add_argument("--view-streams", type=int, default=None,
                    help="streams the full step's view chains run on (default 3; 1: all on one stream)")
    ap.add_argument("--no-large", action="store_true", help="skip the large-scene run")
    ap.add_argument("--only-large", action="store_true", help="the large-scene run alone (prints its record)")
    ap.add_argument("--large-steps", type=int, default=LARGE_STEPS, help="timed steps of the large-scene run")
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

    if args.only_large:
        print(json.dumps({"large_scene": large_scene(dev, args.large_steps)}), flush=True)
        return
    if args.only_headline:
        global FULL_K
        FULL_K = (HEADLINE_K,)
    global PREFIX, FULL_VIEW_STREAMS
    PREFIX = None if args.no_prefix else FULL_PREFIX
    if args.view_streams is not None:
        FULL_VIEW_STREAMS = max(1, args.view_streams)
    p_full, cams, full = full_step(dev, args.steps, args.warmup,
                                   with_dense=not (args.no_dense or args.only_headline), prefix=PREFIX)
    head = full[(HEADLINE_K, "sparse")]
    roofline = roofline_of(head, args.steps)
    full_out = {}
    for (K, name), r in full.items():
        full_out.setdefault(f"K{K}", {})[name] = summarize(r, args.steps)
    for K in FULL_K:
        d = full_out[f"K{K}"]
        if "dense" in d:
            d["sparse_vs_dense_speedup"] = round(d["dense"]["ms_per_step"] / d["sparse"]["ms_per_step"], 3)

    scaling = None
    dens = tile = psnr = large = None
    if not args.only_headline:
        p, cam, gt = make_workload(dev)
        if not args.no_sweep:
            scaling = {}
            for r in SWEEP_RATES:
                log(f"300k sweep {r / 10:g}%")
                tr = make_trainer(p, cam, gt, r, dev)
                res = run(tr, max(10, args.steps), 2)
                scaling[f"{r / 10:g}%"] = summarize(res, max(10, args.steps))
                del tr
            log("300k dense")
            tr = make_trainer(p, cam, gt, None, dev)
            dres = run(tr, max(10, args.steps), 2)
            scaling["dense"] = summarize(dres, max(10, args.steps))
            for k in list(scaling):
                if k != "dense":
                    scaling[k]["sparse_vs_dense_speedup"] = round(
                        scaling["dense"]["ms_per_step"] / scaling[k]["ms_per_step"], 3)
            del tr
        if not args.no_density:
            log("density-control statistics")
            tr = make_trainer(p, cam, gt, HEADLINE_RATE, dev)
            res = run(tr, 10, 2)
            del tr
            dens = density_control(p, cam, gt, dev, res["blends"] / 10)
        if not args.no_tile:
            log("learned tile priority")
            tile = tile_priority(dev)
        if not args.no_psnr:
            psnr = matched_psnr(dev)
        if not args.no_large:
            log(f"large scene: {args.large_steps} steps")
            large = large_scene(dev, args.large_steps)

    cpu = None
    if not args.no_cpu:
        cores = host_cores()
        log("oracle CPU baseline, one thread")
        cpu = cpu_baseline(p_full, cams[0], target_s=5.0, cores=1)
        if cores > 1:
            log(f"oracle CPU baseline, {cores} processes")
            cpu["all_cores"] = cpu_baseline(p_full, cams[0], target_s=5.0, cores=cores)

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
        "config": {"workload": f"full training step: 1.5M Gaussians, 150 hemisphere cameras 1600x1060, "
                               f"K={HEADLINE_K} views per step, 20% error-guided pixels per tile, "
                               f"sparse NCC + Charbonnier, hybrid LM/Adam update",
                   "gaussians": FULL_N, "views": FULL_VIEWS, "width": FULL_W, "height": FULL_H,
                   "views_per_step": HEADLINE_K, "rate": FULL_RATE / 1000,
                   "depth_prefix": None if args.no_prefix else FULL_PREFIX, "view_streams": FULL_VIEW_STREAMS,
                   "parallelism": "single GPU"},
        "step_ms_spread": head["step_ms_spread"],
        "full_step": full_out,
        "roofline": roofline,
        "scaling_300k": scaling,
        "matched_psnr": psnr,
        "tile_priority": tile,
        "density_control": dens,
        "large_scene": large,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
