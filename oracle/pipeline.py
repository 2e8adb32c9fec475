"""One training step of the hot path composed from the oracle stages (Alg. 1,
steps 3-10 for the selected views): sample pixels, project, bin and sort,
render the samples, sparse loss, error/age map update, backward to the
parameters, hybrid update."""
from __future__ import annotations

import numpy as np

from . import binning, loss, maps, optim, project, project_bwd, render, sampler
from .params import LossParams, OptimParams, RasterParams, SampleParams


def gt_at(gt: np.ndarray, xs, ys) -> np.ndarray:
    """Target colours [P, 3] at pixels from a [3, H, W] image."""
    return np.asarray(gt, dtype=np.float64)[:, ys, xs].T


def forward_view(params, cam, samples, rp: RasterParams):
    proj = project.project(params, cam, rp)
    sk, sv, ranges = binning.bin_and_sort(proj, samples["valid_tiles"])
    xs, ys, slot = sampler.sample_coords(samples, cam.width, cam.height)
    out = render.render_pixels(proj, sv, ranges, xs, ys, rp)
    return dict(proj=proj, keys=sk, vals=sv, ranges=ranges, xs=xs, ys=ys, slot=slot, out=out)


def train_step(params, m, v, cams, gts, E, A, step: int, sp: SampleParams, rp: RasterParams,
               lp: LossParams, op: OptimParams, seed: int, beta: float = 0.4, views=None):
    """One step over the views ``views`` (indices into cams).  Returns the new
    state and per-view diagnostics.  E, A are lists of per-view maps.  The
    sparse update touches the Gaussians composited at a sampled pixel of one
    of the views (the support of the step's gradient)."""
    views = list(range(len(cams))) if views is None else list(views)
    samples = {vi: sampler.sample_view(E[vi], A[vi], sp, seed, step, vi) for vi in views}
    P_step = sum(int(s["tile_off"][-1]) for s in samples.values())
    tiles_step = sum(int(s["valid_tiles"].size) for s in samples.values())
    grad = np.zeros((59, params.shape[1]))
    touched = np.zeros(params.shape[1], dtype=bool)
    E, A = list(E), list(A)
    diag = {}
    total = 0.0
    for vi in views:
        fv = forward_view(params, cams[vi], samples[vi], rp)
        y = gt_at(gts[vi], fv["xs"], fv["ys"])
        ls = loss.sparse_loss(fv["out"]["rgb"], y, samples[vi]["tile_off"], P_step, tiles_step, lp)
        total += ls["loss_l1"] + ls["loss_ncc"]
        E[vi], A[vi] = maps.ema_age_update(E[vi], A[vi], fv["xs"], fv["ys"], ls["err"], beta)
        g2d = render.render_pixels_bwd(fv["proj"], fv["vals"], fv["ranges"], fv["xs"], fv["ys"],
                                       ls["dL"], rp)
        grad += project_bwd.project_bwd(params, cams[vi], fv["proj"], g2d, rp)
        touched |= fv["out"]["composited"]
        diag[vi] = dict(fwd=fv, loss=ls, g2d=g2d, samples=samples[vi])
    newp, newm, newv = optim.optimizer_step(params, grad, m, v, touched, op, step)
    return dict(params=newp, m=newm, v=newv, E=E, A=A, grad=grad, touched=touched,
                loss=total, views=diag)
