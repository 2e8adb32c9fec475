"""Per-tile depth-ordered Gaussian lists: keys, their sort and the ranges.

Eq. (alpha_comp) composites, at pixel p, the depth-sorted Gaussians K(p)
that can reach p's tile; the paper renders "the standard 3DGS loop" over the
sampled pixels in tile order (Sec. 3.1, sparse-pixel setting; Sec. 3.6).
Reading (the 3D Gaussian splatting convention it modifies): the list of a
tile holds every visible Gaussian whose tile rectangle (the projection's
``rect``) contains the tile, ordered front to back by its camera-space depth,
ties by Gaussian id.  As data:

* one (key, value) pair per (visible Gaussian, tile of its rectangle that is
  valid for this view); emitted in Gaussian-id order, tiles row-major inside
  the rectangle;
* key = (tile_id << 32) | bits(float32(t_z)), tile_id = ty * TX + tx; t_z is
  above the near plane, so the FP32 bit pattern orders like the depth;
* pairs are ordered by (key, Gaussian id), a total order (library sort);
* ranges[tile] = [first, last + 1) of that tile in the sorted list, [0, 0)
  when empty.

A list may leave out Gaussians that cannot composite anywhere in the tile
(alpha below alpha_min at every pixel centre of the tile): the image, the
gradients and the blend counts are unchanged.  ``max_alpha_in_tile``
evaluates that condition directly, pixel centre by pixel centre, so a
shorter list can be checked against these by an order-preserving subsequence
test plus that evaluation for every pair it drops.
"""
from __future__ import annotations

import numpy as np

TILE = 16


def emit_pairs(rect: np.ndarray, depth32: np.ndarray, TX: int, TY: int, valid_tiles: np.ndarray | None = None):
    """All (key, gaussian id) pairs in emission order, by loops over the
    rectangles (pins ``emit_pairs_fast`` on small scenes)."""
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
                keys.append((np.uint64(tile) << np.uint64(32)) | bits[g])
                vals.append(g)
    return np.array(keys, dtype=np.uint64), np.array(vals, dtype=np.uint32)


def rect_tiles(rect):
    """(Gaussian id, tx, ty) of every tile of every rectangle, Gaussian-id
    order, row-major inside the rect."""
    xmin, ymin, xmax, ymax = (np.asarray(r, dtype=np.int64) for r in rect)
    w = np.maximum(xmax - xmin, 0)
    h = np.maximum(ymax - ymin, 0)
    cnt = w * h
    gid = np.repeat(np.arange(xmin.size, dtype=np.int64), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(gid.size, dtype=np.int64) - start
    wg = w[gid]
    tx = xmin[gid] + local % np.maximum(wg, 1)
    ty = ymin[gid] + local // np.maximum(wg, 1)
    return gid, tx, ty


def emit_pairs_fast(rect, depth32, TX, TY, valid_tiles=None):
    """Same pairs and order as ``emit_pairs``, built with array operations."""
    gid, tx, ty = rect_tiles(rect)
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


def bin_and_sort(proj: dict, valid_tiles=None):
    """Keys, values and ranges of the rectangle lists of a projection."""
    keys, vals = emit_pairs_fast(proj["rect"], proj["depth32"], proj["TX"], proj["TY"], valid_tiles)
    sk, sv = sort_pairs(keys, vals)
    return sk, sv, tile_ranges(sk, proj["TX"] * proj["TY"])


def max_alpha_in_tile(proj: dict, gids, tiles, chunk: int = 4096) -> np.ndarray:
    """For each (Gaussian, tile) pair: the largest o exp(power) over the 256
    pixel centres of the tile (Eq. alpha_comp before the alpha_max clamp;
    power = -1/2 d^T Q d, d = pixel - centre), in FP64 from the
    projection's centre, conic and opacity.  A pair whose value is below
    alpha_min can composite at no pixel of the tile."""
    gids = np.asarray(gids, dtype=np.int64)
    tiles = np.asarray(tiles, dtype=np.int64)
    TX = proj["TX"]
    lx = np.tile(np.arange(TILE, dtype=np.float64), TILE)
    ly = np.repeat(np.arange(TILE, dtype=np.float64), TILE)
    out = np.empty(gids.size)
    for s in range(0, gids.size, chunk):
        g, t = gids[s:s + chunk], tiles[s:s + chunk]
        x = (TILE * (t % TX)).astype(np.float64)[:, None] + lx[None, :]
        y = (TILE * (t // TX)).astype(np.float64)[:, None] + ly[None, :]
        dx = x - proj["mean2d"][0][g][:, None]
        dy = y - proj["mean2d"][1][g][:, None]
        a, b, c = (proj["conic"][i][g][:, None] for i in range(3))
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        out[s:s + chunk] = (proj["opacity"][g][:, None] * np.exp(np.minimum(power, 0.0))).max(axis=1)
    return out
