"""Tile x depth keys, their sort and the per-tile ranges.

The paper renders "the standard 3DGS loop" with sampled pixels ordered by
tile index (Sec. 3.1, sparse-pixel setting; Sec. 3.6), i.e. each tile walks
its Gaussians front to back.  K(p) of Eq. (alpha_comp) is the depth-sorted
set of Gaussians that can reach p's tile.  Readings:

* a (Gaussian, tile) pair exists when the tile lies in the Gaussian's 3-sigma
  tile rectangle AND the tile can hold a composited pixel: the tile's
  pixel-centre rectangle meets the ellipse q(d) <= tau of the Gaussian's
  stored (FP32) centre and conic, q(d) = A dx^2 + 2 B dx dy + C dy^2.  Any
  composited pixel has alpha = o exp(-q/2) >= alpha_min with o <= 1, i.e.
  q <= 2 ln(1/alpha_min); tau adds a 0.1 % margin and is rounded up to a
  multiple of 1/64 (cull_threshold), so a culled pair never composites and
  the images and gradients are those of the plain rectangle lists;
* the test, row by row: the ellipse cut by the pixel-centre strip of tile
  row ty (dy in [Y0, Y1]) is convex, so the tiles of the row it meets are
  those whose pixel-centre column range [X0, X1] meets its x-extent
  [xmin, xmax].  q is convex, the right boundary x(y) of the ellipse is
  concave and the left one convex, so xmax is x(y) at the ellipse's
  rightmost point's dy clamped to the strip (and xmin likewise); with
  det = AC - B^2 the ellipse spans |dy| <= sqrt(tau A / det) and its
  rightmost point sits at dy = -B sqrt(tau / (C det)).  Exactly the tiles
  whose pixel-centre rectangle meets the ellipse (a lower bound of the
  minimum of q over the tile's pixel centres), computed in FP64 with the
  operation order of row_span, so that any implementation of the same order
  (IEEE +, -, *, /, sqrt, no fused multiply-add) reproduces the decision
  bit for bit; a conic that is not positive definite keeps its whole
  rectangle;
* one (key, value) pair per (visible Gaussian, kept tile that is valid for
  this view); emitted in Gaussian-id order, tiles row-major inside the rect;
* key = (tile_id << 32) | bits(float32(t_z)), tile_id = ty * TX + tx; t_z is
  above the near plane so the FP32 bit pattern orders like the depth;
* pairs are ordered by (key, Gaussian id), a total order (library sort);
* ranges[tile] = [first, last + 1) of that tile in the sorted list, [0, 0)
  when empty.
"""
from __future__ import annotations

import math

import numpy as np

TILE = 16


def cull_threshold(alpha_min: float) -> float:
    """tau = 2 ln(1/alpha_min) x 1.001, rounded up to a multiple of 1/64."""
    return math.ceil(128.0 * math.log(1.0 / alpha_min) * 1.001) / 64.0


def splat_fields(proj: dict) -> dict:
    """The FP32 centre (integer part, fraction) and conic of each Gaussian as
    the splat record stores them, widened to FP64."""
    px, py = proj["mean2d"]
    fx, fy = np.floor(px), np.floor(py)

    def f32(a):
        return np.asarray(a, dtype=np.float32).astype(np.float64)

    A, B, C = proj["conic"]
    return dict(xi=f32(fx), xf=f32(px - fx), yi=f32(fy), yf=f32(py - fy), A=f32(A), B=f32(B), C=f32(C))


def row_span(ty, xi, xf, yi, yf, A, B, C, tau):
    """Tile columns [lo, hi] (floats; lo > hi when none) of tile row ty
    whose pixel-centre rectangles meet q <= tau, before clamping to the
    Gaussian's rectangle (element-wise; FP64, fixed operation order).  Pixel
    centres of the row sit at y = 16 ty .. 16 ty + 15 and of column tx at
    x = 16 tx .. 16 tx + 15 relative to the image; d is measured from the
    stored centre xi + xf, yi + yf."""
    ty = np.asarray(ty, dtype=np.float64)
    A, B, C = (np.asarray(v, dtype=np.float64) for v in (A, B, C))
    with np.errstate(invalid="ignore", divide="ignore"):
        det = A * C - B * B
        pd = (A > 0.0) & (det > 0.0)
        ym = np.sqrt((tau * A) / det)                 # half-height of the ellipse
        ys = B * np.sqrt(tau / (C * det))             # -dy of its rightmost point
        Y0 = (TILE * ty - yi) - yf
        Y1 = ((TILE * ty + (TILE - 1)) - yi) - yf
        ylo = np.maximum(Y0, -ym)
        yhi = np.minimum(Y1, ym)
        yr = np.minimum(np.maximum(-ys, ylo), yhi)    # dy of the strip's rightmost point
        yl = np.minimum(np.maximum(ys, ylo), yhi)     # dy of its leftmost point
        tA = tau * A
        sr = np.sqrt(np.maximum(0.0, tA - det * (yr * yr)))
        sl = np.sqrt(np.maximum(0.0, tA - det * (yl * yl)))
        xmax = (sr - B * yr) / A
        xmin = (-sl - B * yl) / A
        PL = (xmin + xf) + xi                         # in image pixel coordinates
        PR = (xmax + xf) + xi
        lo = np.ceil((PL - (TILE - 1)) * (1.0 / TILE))
        hi = np.floor(PR * (1.0 / TILE))
    empty = pd & ~(ylo <= yhi)
    lo = np.where(pd, np.where(empty, np.inf, lo), -np.inf)
    hi = np.where(pd, np.where(empty, -np.inf, hi), np.inf)
    return lo, hi


def tile_touches(tx, ty, xi, xf, yi, yf, A, B, C, tau):
    """Whether the pixel-centre rectangle of tile (tx, ty) meets q <= tau
    (element-wise): tx inside the row's span."""
    lo, hi = row_span(ty, xi, xf, yi, yf, A, B, C, tau)
    tx = np.asarray(tx, dtype=np.float64)
    return (lo <= tx) & (tx <= hi)


def emit_pairs(rect: np.ndarray, depth32: np.ndarray, TX: int, TY: int,
               valid_tiles: np.ndarray | None = None, fields: dict | None = None, tau: float | None = None):
    """All (key, gaussian id) pairs in emission order (loops; ``fields`` and
    ``tau`` switch the ellipse test on)."""
    valid = np.ones(TX * TY, dtype=bool)
    if valid_tiles is not None:
        valid[:] = False
        valid[np.asarray(valid_tiles, dtype=np.int64)] = True
    bits = np.asarray(depth32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keys, vals = [], []
    xmin, ymin, xmax, ymax = (np.asarray(r, dtype=np.int64) for r in rect)
    for g in range(rect.shape[1]):
        for ty in range(ymin[g], ymax[g]):
            for tx in range(xmin[g], xmax[g]):
                tile = ty * TX + tx
                if not valid[tile]:
                    continue
                if fields is not None and not bool(tile_touches(
                        tx, ty, *(fields[k][g] for k in ("xi", "xf", "yi", "yf", "A", "B", "C")), tau)):
                    continue
                keys.append((np.uint64(tile) << np.uint64(32)) | bits[g])
                vals.append(g)
    return np.array(keys, dtype=np.uint64), np.array(vals, dtype=np.uint32)


def rect_tiles(rect):
    """(Gaussian id, tx, ty) of every tile of every rectangle, Gaussian-id
    order, row-major inside the rect."""
    xmin, ymin, xmax, ymax = (np.asarray(r, dtype=np.int64) for r in rect)
    w = xmax - xmin
    h = ymax - ymin
    cnt = w * h
    gid = np.repeat(np.arange(xmin.size, dtype=np.int64), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(gid.size, dtype=np.int64) - start
    wg = w[gid]
    tx = xmin[gid] + local % np.maximum(wg, 1)
    ty = ymin[gid] + local // np.maximum(wg, 1)
    return gid, tx, ty


def kept_tiles(rect, fields, tau):
    """Rect tiles that pass the ellipse test: (Gaussian id, tx, ty), in
    Gaussian-id order, row-major inside the rect (spans clamped to it)."""
    if fields is None:
        return rect_tiles(rect)
    xmin, ymin, xmax, ymax = (np.asarray(r, dtype=np.int64) for r in rect)
    h = np.maximum(ymax - ymin, 0) * (xmax > xmin)
    gr = np.repeat(np.arange(xmin.size, dtype=np.int64), h)
    ty = ymin[gr] + (np.arange(gr.size, dtype=np.int64) - np.repeat(np.cumsum(h) - h, h))
    f = {k: v[gr] for k, v in fields.items()}
    lo, hi = row_span(ty, f["xi"], f["xf"], f["yi"], f["yf"], f["A"], f["B"], f["C"], tau)
    lo = np.clip(lo, xmin[gr], xmax[gr]).astype(np.int64)
    hi = np.clip(hi, xmin[gr] - 1, xmax[gr] - 1).astype(np.int64)
    c = np.maximum(hi - lo + 1, 0)
    gid = np.repeat(gr, c)
    tx = np.repeat(lo, c) + (np.arange(gid.size, dtype=np.int64) - np.repeat(np.cumsum(c) - c, c))
    return gid, tx, np.repeat(ty, c)


def emit_pairs_fast(rect, depth32, TX, TY, valid_tiles=None, fields=None, tau=None):
    """Same pairs and order as ``emit_pairs``, built with array operations
    (the loop version pins this one on small scenes)."""
    gid, tx, ty = kept_tiles(rect, fields, tau)
    tile = ty * TX + tx
    if valid_tiles is not None:
        valid = np.zeros(TX * TY, dtype=bool)
        valid[np.asarray(valid_tiles, dtype=np.int64)] = True
        keep = valid[tile]
        tile, gid = tile[keep], gid[keep]
    bits = np.asarray(depth32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keys = (tile.astype(np.uint64) << np.uint64(32)) | bits[gid]
    return keys, gid.astype(np.uint32)


def sort_pairs(keys: np.ndarray, vals: np.ndarray):
    """Order by (key, Gaussian id) with a library sort."""
    order = np.lexsort((vals, keys))
    return keys[order], vals[order]


def tile_ranges(sorted_keys: np.ndarray, n_tiles: int) -> np.ndarray:
    """ranges[tile] = [start, end) in the sorted list; [0, 0) when empty."""
    tiles = (sorted_keys >> np.uint64(32)).astype(np.int64)
    ranges = np.zeros((n_tiles, 2), dtype=np.int64)
    t = np.arange(n_tiles)
    start = np.searchsorted(tiles, t, side="left")
    end = np.searchsorted(tiles, t, side="right")
    nonempty = end > start
    ranges[nonempty, 0] = start[nonempty]
    ranges[nonempty, 1] = end[nonempty]
    return ranges


def bin_and_sort(proj: dict, valid_tiles=None, alpha_min: float = 1.0 / 255.0):
    """Keys, values and ranges of the culled pair lists of a projection."""
    keys, vals = emit_pairs_fast(proj["rect"], proj["depth32"], proj["TX"], proj["TY"], valid_tiles,
                                 splat_fields(proj), cull_threshold(alpha_min))
    sk, sv = sort_pairs(keys, vals)
    return sk, sv, tile_ranges(sk, proj["TX"] * proj["TY"])
