"""Per-Gaussian statistics of the error-driven density control (Sec. 3.8,
Eq. gauss_err_accum and Eq. gauss_score).

A Gaussian i that is composited at pixel p with weight w_i(p) = T_i(p) alpha_i(p)
(the weight of Eq. alpha_comp) collects, summed over the views and pixels
rendered,

  E_i = sum e(p) w_i(p),   W_i = sum w_i(p),   D_i = sum D_i(p) w_i(p),

and its difficulty score is s_i = e_i + lambda_eff d_i with e_i = E_i / (W_i + eps),
d_i = D_i / (W_i + eps) and lambda_eff = lambda_base (1 - rho).

Readings (the paper leaves these open):

* e(p) is the per-pixel error of the loss stage, |I_hat(p) - I(p)|_1 over the
  three channels (the value the error-map EMA blends in, Eq. ema_err);
* D_i(p) is the Mahalanobis distance of the pixel from the splat centre under
  the conic Q (the inverse 2D covariance, dilation included):
  sqrt(d^T Q d) = sqrt(-2 power) with power as in the compositing weight, and
  it is weighted by w_i(p) as e(p) is ("replacing e by D");
* the pixels are the ones rendered (the sparse samples of the sampled tiles,
  or every pixel in dense mode); the walk, its skips and its stop are those of
  the forward render, so only composited Gaussians collect anything;
* eps = 1e-8, lambda_base and rho are inputs;
* percentile thresholds (Sec. 3.8 with the fractions eta_topk and eta_final of
  the hyper-parameter table): densify the Gaussians whose score reaches the
  eta_topk percentile, i.e. s_i >= the k-th largest score with
  k = max(1, ceil((1 - eta_topk) n)); the final pruning keeps s_i >= the
  k-th largest with k = max(1, ceil(eta_final n)).  Ties at the threshold are
  all selected.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .params import RasterParams
from .render import TILE, _tile_eval

EPS = 1e-8


def accumulate(proj: dict, sorted_vals: np.ndarray, ranges: np.ndarray, xs, ys, err,
               rp: RasterParams = RasterParams()) -> np.ndarray:
    """Eq. gauss_err_accum over the pixels (xs[i], ys[i]) with errors err[i]:
    returns [3, N] = (E, W, D) in FP64."""
    rp = rp.f64()
    TX = proj["TX"]
    N = proj["opacity"].size
    out = np.zeros((3, N))
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    e = np.asarray(err, dtype=np.float64)
    tiles = (ys // TILE) * TX + (xs // TILE)
    for t in np.unique(tiles):
        sel = np.nonzero(tiles == t)[0]
        lo, hi = ranges[t]
        gids = sorted_vals[lo:hi].astype(np.int64)
        if gids.size == 0:
            continue
        ev = _tile_eval(proj, gids, xs[sel].astype(np.float64), ys[sel].astype(np.float64), rp)
        w = np.where(ev["contrib"], ev["T_before"] * ev["alpha"], 0.0)      # [P, K]
        dist = np.sqrt(np.maximum(-2.0 * ev["power"], 0.0))                # [P, K]
        np.add.at(out[0], gids, (e[sel][:, None] * w).sum(axis=0))
        np.add.at(out[1], gids, w.sum(axis=0))
        np.add.at(out[2], gids, (dist * w).sum(axis=0))
    return out


def score(stats: np.ndarray, lambda_base: float, rho: float, eps: float = EPS) -> dict:
    """Eq. gauss_score: visibility-normalised error e_i and distance d_i, and
    s_i = e_i + lambda_base (1 - rho) d_i."""
    E, W, D = (np.asarray(stats[k], dtype=np.float64) for k in range(3))
    e = E / (W + eps)
    d = D / (W + eps)
    lam = lambda_base * (1.0 - rho)
    return dict(e=e, d=d, s=e + lam * d, lambda_eff=lam)


def kth_largest(values: np.ndarray, k: int) -> float:
    """The k-th largest entry (1 <= k <= n), by sorting."""
    v = np.sort(np.asarray(values).ravel())
    assert 1 <= k <= v.size
    return v[v.size - k]


def percentile_count(n: int, fraction: float) -> int:
    """k = max(1, ceil(fraction * n)): how many Gaussians a fraction selects."""
    return max(1, int(np.ceil(fraction * n - 1e-9)))


def select_masks(s: np.ndarray, eta_topk: float, eta_final: float, gate=None, prune: bool = True) -> dict:
    """Densification and final-pruning selections by percentile thresholds.

    ``gate`` (bool [n], optional) is the gradient condition a densified
    Gaussian must also meet (``gradient_gate``); with ``prune`` False (a
    density step that is not a final-pruning step) every Gaussian is kept.
    A Gaussian is densified only if it is kept."""
    n = s.size
    t_d = kth_largest(s, percentile_count(n, 1.0 - eta_topk))
    t_k = kth_largest(s, percentile_count(n, eta_final))
    keep = (s >= t_k) if prune else np.ones(n, dtype=bool)
    dens = (s >= t_d) & keep
    if gate is not None:
        dens &= np.asarray(gate, dtype=bool)
    return dict(densify=dens, keep=keep, thr_densify=t_d, thr_keep=t_k)


def gradient_gate(acc: np.ndarray, abs_sum: np.ndarray, tau_grad: float, tau_abs: float) -> np.ndarray:
    """The gradient condition of densification (the thresholds tau_grad and
    tau_grad^abs of the hyper-parameter table): the mean screen-space centre
    gradient norm per view in which the Gaussian was projected reaches
    tau_grad, or the mean per view of the absolute statistic (the sum over
    pixels of each pixel's own centre-gradient norm) reaches tau_grad^abs.
    Both in NDC units; a Gaussian never projected fails.  Compared in FP32,
    as the GPU compares them."""
    acc = np.asarray(acc, dtype=np.float32)
    views = acc[:, 1]
    seen = views > 0
    safe = np.where(seen, views, np.float32(1))
    g = np.where(seen, acc[:, 0] / safe, np.float32(0))
    a = np.where(seen, np.asarray(abs_sum, dtype=np.float32) / safe, np.float32(0))
    return seen & ((g >= np.float32(tau_grad)) | (a >= np.float32(tau_abs)))


def scene_extent(centres) -> float:
    """Scene size for the percent-dense split rule (the 3D Gaussian splatting
    convention): 1.1 times the largest distance of a camera centre from the
    mean camera centre."""
    c = np.asarray(centres, dtype=np.float64)
    return 1.1 * float(np.linalg.norm(c - c.mean(axis=0), axis=1).max())


def split_log_threshold(percent_dense: float, extent: float) -> float:
    """A densified Gaussian is split when its largest scale exceeds
    rho_dense times the scene extent (percent dense of the hyper-parameter
    table), i.e. its largest log-scale exceeds ln(rho_dense extent)."""
    return float(np.log(percent_dense * extent))


SPLIT_FACTOR = 1.6   # scale divisor of a split (the 3D Gaussian splatting convention)


def apply_topology(params: np.ndarray, m: np.ndarray, v: np.ndarray, keep, densify, z: np.ndarray,
                   log_split: float) -> dict:
    """Densify and prune (Alg. 1 step 11, second line) on the selections.

    Readings (the paper names the step, not its mechanics; these follow the
    3D Gaussian splatting convention it builds on):
    * a Gaussian with keep = 0 is removed; the kept ones stay in order, then
      one new Gaussian per kept Gaussian with densify = 1, in order;
    * a densified Gaussian whose largest log-scale exceeds log_split is split:
      with o = R(q / |q|) diag(exp(s)) z (z the caller's standard normal draw
      for it) the kept slot moves to mean + o and the new one to mean - o,
      both with log-scales s - ln 1.6; otherwise the new one is a clone;
    * the moments of split and new Gaussians restart at zero; the others keep
      theirs.
    Parameter rows: 0-2 mean, 3-5 log-scale, 6-9 quaternion (w, x, y, z),
    10 opacity logit, 11-58 SH."""
    from .project import quat_to_rot
    keep = np.asarray(keep).astype(bool)
    dens = np.asarray(densify).astype(bool) & keep
    P = np.asarray(params, dtype=np.float64)
    s = P[3:6]
    split = dens & (np.asarray(params[3:6]).max(axis=0) > np.float32(log_split))
    q = P[6:10] / np.linalg.norm(P[6:10], axis=0, keepdims=True)
    R = quat_to_rot(q)                                                 # [3, 3, N]
    o = np.einsum("ijn,jn->in", R, np.exp(s) * np.asarray(z, dtype=np.float64).T)
    kept = P.copy()
    kept[0:3] = np.where(split, P[0:3] + o, P[0:3])
    kept[3:6] = np.where(split, s - np.log(SPLIT_FACTOR), s)
    new = P.copy()
    new[0:3] = np.where(split, P[0:3] - o, P[0:3])
    new[3:6] = kept[3:6]
    mk = np.where(split, 0.0, np.asarray(m, dtype=np.float64))
    vk = np.where(split, 0.0, np.asarray(v, dtype=np.float64))
    out = np.concatenate([kept[:, keep], new[:, dens]], axis=1)
    zeros = np.zeros((P.shape[0], int(dens.sum())))
    return dict(params=out, m=np.concatenate([mk[:, keep], zeros], axis=1),
                v=np.concatenate([vk[:, keep], zeros], axis=1),
                n_keep=int(keep.sum()), n_new=int(dens.sum()), split=split)


def grad_screen_accumulate(acc: np.ndarray, g2d: np.ndarray, radius: np.ndarray, width: int,
                           height: int) -> np.ndarray:
    """Screen-space statistics for densification (Alg. 1 step 8, second
    line, and the gradient threshold tau_grad of the hyper-parameter table),
    per view: acc[i] = (sum of |dL/d centre_i|, views in which i was
    projected (radius > 0), largest radius, -).  Reading: the norm is taken
    of the 2D centre gradient of that view's backward in NDC units (the pixel
    gradient times (W/2, H/2)), the units of the 3D Gaussian splatting
    densification statistic that the table's thresholds are stated for."""
    acc = np.array(acc, dtype=np.float64, copy=True)
    g = np.asarray(g2d, dtype=np.float64)
    vis = np.asarray(radius) > 0
    acc[:, 0] += np.where(vis, np.hypot(0.5 * width * g[:, 0], 0.5 * height * g[:, 1]), 0.0)
    acc[:, 1] += vis
    acc[:, 2] = np.maximum(acc[:, 2], np.where(vis, np.asarray(radius, dtype=np.float64), 0.0))
    return acc


def grad_screen_mean(acc: np.ndarray) -> np.ndarray:
    """Mean gradient norm per view in which the Gaussian was projected (0 if none)."""
    acc = np.asarray(acc, dtype=np.float64)
    return np.where(acc[:, 1] > 0, acc[:, 0] / np.maximum(acc[:, 1], 1.0), 0.0)
