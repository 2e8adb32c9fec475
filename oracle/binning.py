"""Tile x depth keys, their sort and the per-tile ranges.

The paper renders "the standard 3DGS loop" with sampled pixels ordered by
tile index (Sec. 3.1, sparse-pixel setting; Sec. 3.6), i.e. each tile walks
its Gaussians front to back.  K(p) of Eq. (alpha_comp) is the depth-sorted
set of Gaussians whose tile rectangle contains p's tile.  Readings:

* one (key, value) pair per (visible Gaussian, touched tile that is valid for
  this view); emitted in Gaussian-id order, tiles row-major inside the rect;
* key = (tile_id << 32) | bits(float32(t_z)), tile_id = ty * TX + tx; t_z is
  above the near plane so the FP32 bit pattern orders like the depth;
* pairs are ordered by (key, Gaussian id), a total order (library sort);
* ranges[tile] = [first, last + 1) of that tile in the sorted list, [0, 0)
  when empty.
"""
from __future__ import annotations

import numpy as np


def emit_pairs(rect: np.ndarray, depth32: np.ndarray, TX: int, TY: int,
               valid_tiles: np.ndarray | None = None):
    """All (key, gaussian id) pairs in emission order."""
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
                if valid[tile]:
                    keys.append((np.uint64(tile) << np.uint64(32)) | bits[g])
                    vals.append(g)
    return np.array(keys, dtype=np.uint64), np.array(vals, dtype=np.uint32)


def emit_pairs_fast(rect, depth32, TX, TY, valid_tiles=None):
    """Same pairs and order as ``emit_pairs``, built with array operations
    (the loop version pins this one on small scenes)."""
    xmin, ymin, xmax, ymax = (np.asarray(r, dtype=np.int64) for r in rect)
    w = xmax - xmin
    h = ymax - ymin
    cnt = w * h
    gid = np.repeat(np.arange(rect.shape[1], dtype=np.int64), cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(gid.size, dtype=np.int64) - start
    wg = w[gid]
    tx = xmin[gid] + local % np.maximum(wg, 1)
    ty = ymin[gid] + local // np.maximum(wg, 1)
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
    keys, vals = emit_pairs_fast(proj["rect"], proj["depth32"], proj["TX"], proj["TY"], valid_tiles)
    sk, sv = sort_pairs(keys, vals)
    return sk, sv, tile_ranges(sk, proj["TX"] * proj["TY"])
