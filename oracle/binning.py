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
* the test: q at the rectangle point P nearest the centre is <= tau, or the
  closed-form minimum of q along one of the (at most two) edges through P
  that face the centre is; together the continuous minimum of q over the
  tile's pixel-centre rectangle (a lower bound of the minimum over its pixel
  centres), in FP64 with the operation order of tile_touches, so that any
  implementation of the same order reproduces the decision bit for bit;
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


def _quad(A, B, C, x, y):
    return ((A * x) * x + ((2.0 * B) * x) * y) + (C * y) * y


def tile_touches(tx, ty, xi, xf, yi, yf, A, B, C, tau):
    """Whether the pixel-centre rectangle of tile (tx, ty) meets q <= tau
    (element-wise over arrays; FP64, fixed operation order).  Pixel centres
    of the tile sit at x = 16 tx .. 16 tx + 15 relative to the image; d is
    measured from the stored centre xi + xf.  With P the rectangle point
    nearest the centre, the minimum of the convex q over the rectangle lies
    on the edges through P that face the centre (x = P_x when the centre is
    left or right of the rectangle, y = P_y when above or below): kept when
    q(P) <= tau or the closed-form minimum along a facing edge is."""
    tx = np.asarray(tx, dtype=np.float64)
    ty = np.asarray(ty, dtype=np.float64)
    X0 = (TILE * tx - xi) - xf
    X1 = (TILE * tx + (TILE - 1) - xi) - xf
    Y0 = (TILE * ty - yi) - yf
    Y1 = (TILE * ty + (TILE - 1) - yi) - yf
    Px = np.minimum(np.maximum(0.0, X0), X1)
    Py = np.minimum(np.maximum(0.0, Y0), Y1)
    keep = _quad(A, B, C, Px, Py) <= tau
    det = A * C - B * B
    # vertical facing edge x = Px, y in [Y0, Y1]
    bx = B * Px
    lo = -bx < C * Y0
    hi = ~lo & (-bx > C * Y1)
    y = np.where(lo, Y0, Y1)
    edge = np.where(lo | hi, _quad(A, B, C, Px, y) <= tau, (Px * Px) * det <= tau * C)
    keep = keep | ((Px != 0.0) & edge)
    # horizontal facing edge y = Py, x in [X0, X1]
    by = B * Py
    lo = -by < A * X0
    hi = ~lo & (-by > A * X1)
    x = np.where(lo, X0, X1)
    edge = np.where(lo | hi, _quad(A, B, C, x, Py) <= tau, (Py * Py) * det <= tau * A)
    keep = keep | ((Py != 0.0) & edge)
    return keep


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
    """Rect tiles that pass the ellipse test: (Gaussian id, tx, ty)."""
    gid, tx, ty = rect_tiles(rect)
    if fields is not None:
        f = {k: v[gid] for k, v in fields.items()}
        keep = tile_touches(tx, ty, f["xi"], f["xf"], f["yi"], f["yf"], f["A"], f["B"], f["C"], tau)
        gid, tx, ty = gid[keep], tx[keep], ty[keep]
    return gid, tx, ty


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
