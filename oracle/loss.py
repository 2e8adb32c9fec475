"""Sparse supervision: pixel Charbonnier L1 plus tile-level sparse NCC with a
gradient-balanced weight (Sec. 3.7, Eq. ncc_weight_auto, Eq. full_loss, and
the gradient formulas of App. A).

Readings:

* per pixel and channel rho(x - y) = sqrt((x - y)^2 + eps_c^2), whose
  derivative is the App. A Charbonnier gradient (x - y)/sqrt((x - y)^2 + eps_c^2);
* NCC per channel over the tile's samples with 1/n moments,
  NCC = C_xy / sqrt(V_x V_y + eps_n); the tile loss is 1 - (mean over channels);
* the per-pixel NCC "gradient" used for the balance statistics is
  g_n = n * d(1 - NCC)/dx, i.e.
  -[(y - mu_y)/sqrt(D) - NCC V_y (x - mu_x)/D],  D = V_x V_y + eps_n,
  which is App. A's expression when eps_n -> 0;
* lambda = clip(mean_p |g1|_1 / (mean_p |g_n|_1 + eps_l), 0, 1), norms over the
  three channels, held constant (no gradient through it);
* L = mean over the step's sampled (pixel, channel) of rho
      + mean over the step's sampled tiles of lambda (1 - mean_ch NCC);
  the combined pixel gradient adds the NCC term (the sign of Eq. full_loss,
  where App. A's display subtracts: descent on 1 - NCC);
* per-pixel error e(p) = sum_ch |x - y| (Eq. l1_err).

S-SSIM variant (the ablation that replaces S-NCC by a sparse SSIM, Tab.
ablation_main): the tile term is 1 - SSIM with one window per tile and
channel over the tile's samples (the same 1/n moments as NCC),
SSIM = (2 mu_x mu_y + C1)(2 C_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(V_x + V_y + C2)),
C1 = (0.01)^2, C2 = (0.03)^2 (the SSIM constants of Wang et al. 2004 for
values in [0, 1]), averaged over channels; its per-pixel gradient for the
balance weight is g_s = n d(1 - SSIM)/dx =
-2 SSIM [mu_y/A1 + (y - mu_y)/A2 - mu_x/B1 - (x - mu_x)/B2] with A1, A2, B1,
B2 the four factors above; lambda and the combination are those of NCC.
"""
from __future__ import annotations

import numpy as np

from .params import LossParams


SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def ssim_terms(x: np.ndarray, y: np.ndarray):
    """Per-channel sparse SSIM of one tile's samples and its per-pixel
    gradient g_s = n d(1 - SSIM)/dx ([3] and [n, 3])."""
    mx, my = x.mean(axis=0), y.mean(axis=0)
    xc, yc = x - mx, y - my
    Vx = (xc * xc).mean(axis=0)
    Vy = (yc * yc).mean(axis=0)
    Cxy = (xc * yc).mean(axis=0)
    A1 = 2.0 * mx * my + SSIM_C1
    A2 = 2.0 * Cxy + SSIM_C2
    B1 = mx * mx + my * my + SSIM_C1
    B2 = Vx + Vy + SSIM_C2
    ssim = (A1 * A2) / (B1 * B2)
    gs = -2.0 * ssim * (my / A1 + yc / A2 - mx / B1 - xc / B2)
    return ssim, gs


def tile_loss(x: np.ndarray, y: np.ndarray, lp: LossParams = LossParams()) -> dict:
    """Terms of one tile: x, y are [n, 3] rendered and target colours.  With
    lp.structure == "ssim" the structure term is S-SSIM (keys ncc and gn
    then hold SSIM and its gradient)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    diff = x - y
    rho = np.sqrt(diff * diff + lp.eps_charb ** 2)
    g1 = diff / rho
    mx, my = x.mean(axis=0), y.mean(axis=0)
    xc, yc = x - mx, y - my
    Vx = (xc * xc).mean(axis=0)
    Vy = (yc * yc).mean(axis=0)
    Cxy = (xc * yc).mean(axis=0)
    D = Vx * Vy + lp.eps_ncc
    ncc = Cxy / np.sqrt(D)
    gn = -(yc / np.sqrt(D) - ncc * Vy * xc / D)
    if lp.structure == "ssim":
        ncc, gn = ssim_terms(x, y)
    gbar1 = np.abs(g1).sum(axis=1).mean()
    gbarn = np.abs(gn).sum(axis=1).mean()
    lam = min(max(gbar1 / (gbarn + lp.eps_lambda), 0.0), 1.0)
    return dict(n=n, rho=rho, g1=g1, ncc=ncc, gn=gn, lam=lam,
                err=np.abs(diff).sum(axis=1))


def sparse_loss(rgb: np.ndarray, gt_at: np.ndarray, tile_off: np.ndarray, P_step: int,
                tiles_step: int, lp: LossParams = LossParams()) -> dict:
    """Loss terms and dL/dI for one view's samples ([P, 3] each), normalised by
    the step totals (sampled pixels and tiles of all the step's views)."""
    P = rgb.shape[0]
    dL = np.zeros((P, 3))
    err = np.zeros(P)
    lam = np.zeros(tile_off.size - 1)
    ncc = np.zeros((tile_off.size - 1, 3))
    l1_sum = 0.0
    ncc_sum = 0.0
    for s in range(tile_off.size - 1):
        lo, hi = tile_off[s], tile_off[s + 1]
        if hi == lo:
            continue
        tl = tile_loss(rgb[lo:hi], gt_at[lo:hi], lp)
        n = hi - lo
        dL[lo:hi] = tl["g1"] / (3.0 * P_step) + tl["lam"] * tl["gn"] / (3.0 * n * tiles_step)
        err[lo:hi] = tl["err"]
        lam[s] = tl["lam"]
        ncc[s] = tl["ncc"]
        l1_sum += tl["rho"].sum() / (3.0 * P_step)
        ncc_sum += tl["lam"] * (1.0 - tl["ncc"].mean()) / tiles_step
    return dict(dL=dL, err=err, lam=lam, ncc=ncc, loss_l1=l1_sum, loss_ncc=ncc_sum)


def loss_value(rgb, gt_at, tile_off, P_step, tiles_step, lam, lp: LossParams = LossParams()) -> float:
    """L for fixed (detached) lambdas; used by finite-difference checks."""
    rgb = np.asarray(rgb, dtype=np.float64)
    gt_at = np.asarray(gt_at, dtype=np.float64)
    total = 0.0
    for s in range(tile_off.size - 1):
        lo, hi = tile_off[s], tile_off[s + 1]
        if hi == lo:
            continue
        x, y = rgb[lo:hi], gt_at[lo:hi]
        d = x - y
        total += np.sqrt(d * d + lp.eps_charb ** 2).sum() / (3.0 * P_step)
        if lp.structure == "ssim":
            ncc = ssim_terms(x, y)[0]
        else:
            xc, yc = x - x.mean(axis=0), y - y.mean(axis=0)
            D = (xc * xc).mean(axis=0) * (yc * yc).mean(axis=0) + lp.eps_ncc
            ncc = (xc * yc).mean(axis=0) / np.sqrt(D)
        total += lam[s] * (1.0 - ncc.mean()) / tiles_step
    return total
