"""Front-to-back alpha compositing at requested pixels, and its exact adjoint.

Eq. (alpha_comp): I(p) = sum_k T_k alpha_k c_k with T_k = prod_{j<k} (1 - alpha_j)
over the depth-ordered Gaussians K(p) of p's tile (Sec. 3.6 renders only the
sampled pixels of the valid tiles, with the same per-pixel arithmetic as the
dense render).  Readings for what the paper leaves implicit (the conventions
of the 3DGS rasterizer it modifies):

* alpha_k = min(alpha_max, o_k exp(power)), power = -1/2 d^T Q d with
  d = pixel - centre and Q the conic; a Gaussian with power > 0 or
  alpha < alpha_min is skipped;
* when T (1 - alpha_k) would fall below T_min the walk stops before
  compositing Gaussian k;
* the output is C + T_final * bg; n_contrib is the range position of the last
  composited Gaussian plus one (0 if none);
* counters: an *evaluation* is a Gaussian whose alpha was computed (every
  range position up to and including the stopping one), a *blend* one that
  was composited.

The arrays are laid out per tile as [pixels, Gaussians] so each formula reads
as written; T is the running product taken left to right (cumprod), the same
sequence of multiplications as the scalar loop.

Guard band: a pixel is flagged when one of its discrete decisions (alpha vs
alpha_min or alpha_max, T (1 - alpha) vs T_min) lies within ``guard`` times
an error bound of an FP32 evaluation of that same quantity.  The bound
follows from the arithmetic of an FP32 evaluation that takes the exponent in
the conic's LDL^T form, d^T Q d = a w^2 + delta dy^2 with w = dx + beta dy,
beta = b / a, delta = c - b beta (two non-negative terms, so no
cancellation).  Per (pixel, Gaussian), with u = 2^-24:

* the terms' size S = (|a| w^2 + |delta| dy^2) / 2: the conic values, the
  scale by log2(e) and the products and sums each rounded once give an
  error of a few u S; 8 u S is taken;
* the offsets dx, dy (tile-local centre = exact integer difference plus the
  fraction, then the pixel minus it) carry absolute errors of at most
  u (2 |dx| + 18) and u (2 |dy| + 18), w in addition u (|w| + |beta dy|)
  from its own rounding and that of beta; times the exponent's slopes
  |a w| and |a beta w + delta dy| this gives the term ``slope``;

twice their sum bounds the exponent's error (about twice the largest an
FP32 emulation of that evaluation shows, on the tiny, the
rasterizer-scaling and a near-camera needle workload), so alpha carries a
relative error of at most eps_a = 2 u (8 S + slope) + 8 u (exponential,
opacity and product included).  The transmittance after position k carries
a relative error of at most the sum over the positions composited up to k
of 2 u + eps_a alpha / (1 - alpha).
FP32 and FP64 evaluations can take a decision inside its band differently;
tests exclude flagged pixels from element-wise comparison and bound how many
there are.
"""
from __future__ import annotations

import numpy as np

from .params import RasterParams

TILE = 16
U32 = 2.0 ** -24        # unit roundoff of FP32


def _tile_eval(proj, gids, xs, ys, rp):
    px, py = proj["mean2d"][0][gids], proj["mean2d"][1][gids]
    a, b, c = (proj["conic"][i][gids] for i in range(3))
    o = proj["opacity"][gids]
    dx = xs[:, None] - px[None, :]
    dy = ys[:, None] - py[None, :]
    power = -0.5 * (a[None, :] * dx * dx + c[None, :] * dy * dy) - b[None, :] * dx * dy
    G = np.exp(power)
    araw = o[None, :] * G
    alpha = np.minimum(rp.alpha_max, araw)
    ok = (power <= 0.0) & (alpha >= rp.alpha_min)
    # error bound of an FP32 exponent taken as a w^2 + delta dy^2 (the LDL^T
    # form of the conic, w = dx + beta dy): the terms' size S, and the
    # exponent's slope times the FP32 offset error of the pixel from the centre
    beta = np.where(a > 0, b / np.where(a > 0, a, 1.0), 0.0)[None, :]
    delta = np.where(a > 0, c - b * beta[0], 0.0)[None, :]
    aa = np.abs(a)[None, :]
    w = dx + beta * dy
    adx, ady = np.abs(dx), np.abs(dy)
    S = 0.5 * (aa * w * w + np.abs(delta) * dy * dy)
    slope = (aa * np.abs(w) * (np.abs(w) + np.abs(beta) * (3.0 * ady + 18.0) + 2.0 * adx + 18.0)
             + np.abs(aa * beta * w + delta * dy) * (2.0 * ady + 18.0))
    eps_a = 2.0 * U32 * (8.0 * S + slope) + 8.0 * U32
    av = np.where(ok, alpha, 0.0)
    one_m = 1.0 - av
    K = gids.size
    T_after = np.cumprod(one_m, axis=1)
    T_before = np.concatenate([np.ones((xs.size, 1)), T_after[:, :-1]], axis=1) if K else T_after
    stop = ok & (T_after < rp.T_min)
    has_stop = stop.any(axis=1)
    s = np.where(has_stop, np.argmax(stop, axis=1), K)           # first stopping position
    kidx = np.arange(K)[None, :]
    contrib = ok & (kidx < s[:, None])
    # error bound of the FP32 transmittance after each position: the sum over
    # the composited positions before it and the position itself
    step_eps = 2.0 * U32 + eps_a * av / np.maximum(1.0 - av, 1e-300)
    eps_T = np.cumsum(np.where(contrib | stop, step_eps, 0.0), axis=1)
    return dict(dx=dx, dy=dy, power=power, G=G, araw=araw, alpha=alpha, ok=ok,
                T_before=T_before, T_after=T_after, contrib=contrib, stop_at=s,
                has_stop=has_stop, a=a, b=b, c=c, o=o, eps_a=eps_a, eps_T=eps_T)


def render_pixels(proj: dict, sorted_vals: np.ndarray, ranges: np.ndarray, xs: np.ndarray,
                  ys: np.ndarray, rp: RasterParams = RasterParams(), guard: float = 2.0) -> dict:
    """Render the pixels (xs[i], ys[i]) (any order; grouped by tile internally).

    Returns rgb [P, 3], T [P], n_contrib [P], n_eval [P], n_blend [P], flag [P]
    and composited [N] (the Gaussians composited at one of the pixels at
    least: the support of the gradient, what the sparse update touches)."""
    rp = rp.f64()
    TX = proj["TX"]
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    P = xs.size
    out = np.zeros((P, 3))
    T_out = np.ones(P)
    ncon = np.zeros(P, dtype=np.int64)
    neval = np.zeros(P, dtype=np.int64)
    nblend = np.zeros(P, dtype=np.int64)
    flag = np.zeros(P, dtype=bool)
    composited = np.zeros(proj["opacity"].size, dtype=bool)
    bg = np.asarray(rp.bg, dtype=np.float64)
    tiles = (ys // TILE) * TX + (xs // TILE)
    for t in np.unique(tiles):
        sel = np.nonzero(tiles == t)[0]
        lo, hi = ranges[t]
        gids = sorted_vals[lo:hi].astype(np.int64)
        K = gids.size
        if K == 0:
            out[sel] = bg
            continue
        ev = _tile_eval(proj, gids, xs[sel].astype(np.float64), ys[sel].astype(np.float64), rp)
        composited[gids[ev["contrib"].any(axis=0)]] = True
        w = np.where(ev["contrib"], ev["T_before"] * ev["alpha"], 0.0)
        col = proj["rgb"][:, gids].T                                  # [K, 3]
        # running sums/products taken left to right, as the scalar loop does
        C = np.cumsum(w[:, :, None] * col[None, :, :], axis=1)[:, -1, :]
        last = np.where(ev["contrib"].any(axis=1),
                        K - 1 - np.argmax(ev["contrib"][:, ::-1], axis=1), -1)
        T_fin = np.cumprod(np.where(ev["contrib"], 1.0 - ev["alpha"], 1.0), axis=1)[:, -1]
        out[sel] = C + T_fin[:, None] * bg[None, :]
        T_out[sel] = T_fin
        ncon[sel] = last + 1
        neval[sel] = np.where(ev["has_stop"], ev["stop_at"] + 1, K)
        nblend[sel] = ev["contrib"].sum(axis=1)
        # guard band over the evaluated positions
        evaluated = np.arange(K)[None, :] < neval[sel][:, None]
        band_a = guard * ev["eps_a"] * ev["araw"]
        near_min = np.abs(ev["araw"] - rp.alpha_min) <= band_a
        near_max = np.abs(ev["araw"] - rp.alpha_max) <= band_a
        near_T = ev["ok"] & (np.abs(ev["T_after"] - rp.T_min) <= guard * ev["eps_T"] * ev["T_after"])
        flag[sel] = (evaluated & (near_min | near_max | near_T)).any(axis=1)
    return dict(rgb=out, T=T_out, n_contrib=ncon, n_eval=neval, n_blend=nblend, flag=flag,
                composited=composited)


def render_pixels_bwd(proj: dict, sorted_vals: np.ndarray, ranges: np.ndarray, xs, ys,
                      dL_drgb: np.ndarray, rp: RasterParams = RasterParams(),
                      with_abs: bool = False, centre_abs_scale=None):
    """Exact adjoint of ``render_pixels``: given dL/dI at the pixels, return
    dL/d(screen-space splat parameters) per Gaussian, g2d [9, N] =
    (mean2d x, y; conic a, b, c; opacity; rgb r, g, b).

    With B_k = I(p) - sum_{j<=k} T_j alpha_j c_j (what lies behind k, including
    the background term):  dI/dc_k = T_k alpha_k,
    dI/dalpha_k = T_k c_k - B_k / (1 - alpha_k).  alpha = o G is differentiated
    only where it was not clamped at alpha_max; G = exp(power).

    With ``with_abs`` it also returns, per Gaussian and field, the sum over
    pixels of an error scale for an FP32 evaluation: the absolute value of
    each term, where dL/dalpha is replaced by the magnitude of its two parts,
    sum_ch |g| (T |c| + (|I| + |C_{<=k}|) / (1 - alpha)).  A front-to-back
    evaluation obtains B_k as I - C_{<=k}, a difference of two O(|I|)
    numbers, so its rounding error scales with |I|, not with |B_k|.

    With ``centre_abs_scale = (sx, sy)`` it also returns, per Gaussian, the
    sum over pixels of the norm of that pixel's own centre gradient in scaled
    units, |(sx dL_p/dx, sy dL_p/dy)| (the absolute-gradient statistic of
    densification, Sec. 3.8; sx = W/2, sy = H/2 turn pixel units into NDC
    units): the norm is taken per pixel before summing, so pixels pulling the
    centre in opposite directions do not cancel."""
    rp = rp.f64()
    TX = proj["TX"]
    N = proj["opacity"].size
    g2d = np.zeros((9, N))
    g2d_abs = np.zeros((9, N))
    cabs = np.zeros(N)
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    g = np.asarray(dL_drgb, dtype=np.float64)
    bg = np.asarray(rp.bg, dtype=np.float64)
    tiles = (ys // TILE) * TX + (xs // TILE)
    for t in np.unique(tiles):
        sel = np.nonzero(tiles == t)[0]
        lo, hi = ranges[t]
        gids = sorted_vals[lo:hi].astype(np.int64)
        if gids.size == 0:
            continue
        ev = _tile_eval(proj, gids, xs[sel].astype(np.float64), ys[sel].astype(np.float64), rp)
        con = ev["contrib"]
        alpha = np.where(con, ev["alpha"], 0.0)
        Tb = ev["T_before"]
        col = proj["rgb"][:, gids].T                                  # [K, 3]
        w = np.where(con, Tb * alpha, 0.0)                            # [P, K]
        acc = np.cumsum(w[:, :, None] * col[None, :, :], axis=1)      # C_{<=k}
        T_fin = np.cumprod(np.where(con, 1.0 - alpha, 1.0), axis=1)[:, -1]
        Cp = acc[:, -1, :] + T_fin[:, None] * bg[None, :]
        Bk = Cp[:, None, :] - acc                                      # [P, K, 3]
        gp = g[sel]                                                    # [P, 3]
        dI_dalpha = Tb[:, :, None] * col[None, :, :] - Bk / (1.0 - alpha)[:, :, None]
        dL_dalpha = np.where(con, np.einsum("pkc,pc->pk", dI_dalpha, gp), 0.0)
        unclamped = con & (ev["araw"] < rp.alpha_max)
        G = ev["G"]
        o = ev["o"][None, :]
        dL_dpow = np.where(unclamped, o * G * dL_dalpha, 0.0)          # dL/dG * dG/dpower
        dx, dy = ev["dx"], ev["dy"]
        a, b, c = ev["a"][None, :], ev["b"][None, :], ev["c"][None, :]
        # power = -1/2 (a dx^2 + c dy^2) - b dx dy, d = pixel - centre
        terms = [(a * dx + b * dy) * dL_dpow, (b * dx + c * dy) * dL_dpow,
                 -0.5 * dx * dx * dL_dpow, -dx * dy * dL_dpow, -0.5 * dy * dy * dL_dpow,
                 np.where(unclamped, G * dL_dalpha, 0.0),
                 w * gp[:, 0:1], w * gp[:, 1:2], w * gp[:, 2:3]]
        for row, tm in enumerate(terms):
            np.add.at(g2d[row], gids, tm.sum(axis=0))
        if centre_abs_scale is not None:
            sx, sy = centre_abs_scale
            np.add.at(cabs, gids, np.hypot(sx * terms[0], sy * terms[1]).sum(axis=0))
        if with_abs:
            mag = np.einsum("pkc,pc->pk", Tb[:, :, None] * np.abs(col)[None, :, :]
                            + (np.abs(Cp)[:, None, :] + np.abs(acc)) / (1.0 - alpha)[:, :, None],
                            np.abs(gp))
            mag_pow = np.where(unclamped, o * G * mag, 0.0)
            scale = [np.abs(a * dx + b * dy) * mag_pow, np.abs(b * dx + c * dy) * mag_pow,
                     0.5 * dx * dx * mag_pow, np.abs(dx * dy) * mag_pow, 0.5 * dy * dy * mag_pow,
                     np.where(unclamped, G * mag, 0.0)] + [np.abs(tm) for tm in terms[6:]]
            for row, sc in enumerate(scale):
                np.add.at(g2d_abs[row], gids, sc.sum(axis=0))
    res = (g2d, g2d_abs) if with_abs else (g2d,)
    if centre_abs_scale is not None:
        res = res + (cabs,)
    return res if len(res) > 1 else res[0]


def dense_pixels(W: int, H: int):
    """Every in-image pixel, row-major."""
    y, x = np.mgrid[0:H, 0:W]
    return x.ravel(), y.ravel()
