"""Tile-wise error-guided sparse pixel sampling (Sec. 3.5).

Per selected tile the paper draws N_hard pixels by multinomial sampling
without replacement with probability proportional to the error map
(Eq. pix_prob_err), then the N_stable pixels of largest age among the rest
(Eq. pix_topk_age); the hyper-parameter table adds a "mixed" remainder
(0.3 of the budget).  Readings (the paper is silent on these):

* weights are the half error values scaled by 2^24, which makes every finite
  non-negative half an exact integer; negative, NaN and infinite entries weigh 0;
* sequential draws: each hard draw takes r = floor(u * W_rem / 2^64) for a
  64-bit counter draw u and the remaining weight W_rem, and picks the first
  remaining pixel (ascending local index ly*16 + lx) whose running weight
  exceeds r; the chosen pixel leaves the pool;
* when the remaining weight is zero, the unfilled hard slots join the mixed set;
* TopK age breaks ties toward the lower local index;
* mixed slots are uniform without replacement over the pixels left, the
  r = floor(u * n_left / 2^64)-th in ascending order;
* partial edge tiles sample min(N_pix, valid pixels) and recompute the split;
  pixels outside the image are never sampled;
* optional tile pass: n_tiles_sel tiles drawn without replacement with
  probability proportional to the tile's summed pixel weights, uniform over
  the remaining tiles once those weights run out; selected tiles are listed in
  ascending order.  The draw order plays no part downstream, so the pass takes
  the exponential race of Efraimidis and Spirakis ("Weighted random sampling
  with a reservoir", IPL 2006), which gives the sequential draws' distribution
  exactly: every tile gets an independent Exp(1) time divided by its weight and
  the n_tiles_sel earliest win.  Times are exact on both sides of the parity
  check: Exp(1) / ln 2 = -log2 of a uniform, taken to 47 fractional bits by the
  binary logarithm by repeated squaring, divided by the weight once in IEEE
  double; zero-weight tiles come after every weighted one, ordered by a uniform
  key; ties go to the lower tile index.
"""
from __future__ import annotations

import struct

import numpy as np

from .params import SampleParams, split_counts
from .rng import below, draw

TILE = 16


def half_weights(E_bits: np.ndarray) -> np.ndarray:
    """Integer weights w = E * 2^24 (exact), invalid or negative -> 0."""
    e = np.asarray(E_bits, dtype=np.uint16).view(np.float16).astype(np.float64)
    ok = np.isfinite(e) & (e > 0)
    w = np.where(ok, e, 0.0) * float(1 << 24)
    return w.astype(np.int64)


def tile_pixels(tile: int, TX: int, W: int, H: int):
    """Local indices of the in-image pixels of a tile, ascending."""
    tx, ty = tile % TX, tile // TX
    loc = np.arange(TILE * TILE)
    x = tx * TILE + loc % TILE
    y = ty * TILE + loc // TILE
    ok = (x < W) & (y < H)
    return loc[ok], x[ok], y[ok]


def _pick_weighted(weights, u):
    """First index whose running sum exceeds floor(u * total / 2^64)."""
    total = int(weights.sum())
    r = below(u, total)
    csum = np.cumsum(weights)
    return int(np.searchsorted(csum, r, side="right"))


PRED_MAX = 65504.0   # predictions are clamped to the largest finite half, like E


def predicted_tile_weights(pred, TX: int, TY: int, W: int, H: int) -> np.ndarray:
    """Integer tile weights from predicted mean tile errors (a reading for the
    learned tile priority): floor(clamp(p, 0, 65504) * in-image pixels * 2^24)
    with p the float32 prediction, the units of the error-map sums (mean E
    times the pixel count).  Exact in FP64: a float32 times a count up to 256
    times a power of two."""
    tw = np.zeros(TX * TY, dtype=np.int64)
    for t in range(TX * TY):
        _, x, _ = tile_pixels(t, TX, W, H)
        p = float(np.float32(pred[t]))
        p = min(p, PRED_MAX) if p > 0.0 else 0.0      # NaN and negatives give 0
        tw[t] = int(np.floor(p * x.size * float(1 << 24)))
    return tw


LOG_FRAC = 47     # fractional bits of a race time: the largest time, 64, times 2^47 is 2^53


def neg_log2_fixed(u: int) -> int:
    """2^47 * -log2(v / 2^64) for v = u | 1 (so v / 2^64 lies in (0, 1)),
    with the fraction truncated to 47 bits.  v = 2^e * m with m in [1, 2):
    -log2(v / 2^64) = 64 - e - log2(m), and the bits of log2(m) come one per
    squaring (binary logarithm by repeated squaring, e.g. Knuth, TAOCP vol. 1,
    1.2.2): m^2 >= 2 gives bit 1 and m <- m^2 / 2, else bit 0 and m <- m^2.
    m is held in Q1.63 (2^63 <= m < 2^64), each square truncated to it."""
    v = (u & ((1 << 64) - 1)) | 1
    e = v.bit_length() - 1
    m = v << (63 - e)
    frac = 0
    for _ in range(LOG_FRAC):
        sq = m * m                                # Q2.126
        if sq >> 127:
            frac = 2 * frac + 1
            m = sq >> 64
        else:
            frac = 2 * frac
            m = sq >> 63
    return ((64 - e) << LOG_FRAC) - frac


def _double_bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def tile_race_keys(tw, seed: int, step: int, view: int) -> list:
    """Race key of every tile (smaller runs first), as an unsigned 64-bit
    integer: for weight w > 0 the bit pattern of the double L / w, L the
    tile's fixed-point -log2 uniform (positive doubles order like their bit
    patterns, all below 2^63); for w = 0, 2^63 + (u >> 1), after every
    weighted tile.  u is the tile's draw in the tile pass's stream."""
    n_t = len(tw)
    keys = []
    for t in range(n_t):
        u = draw(seed, step, view, n_t, t)
        w = int(tw[t])
        if w > 0:
            keys.append(_double_bits(float(neg_log2_fixed(u)) / float(w)))
        else:
            keys.append((1 << 63) | (u >> 1))
    return keys


def race_select(tw, n_sel: int, seed: int, step: int, view: int) -> np.ndarray:
    """The n_sel tiles of smallest (race key, tile index), ascending."""
    keys = tile_race_keys(tw, seed, step, view)
    order = sorted(range(len(keys)), key=lambda t: (keys[t], t))
    return np.sort(np.array(order[:n_sel], dtype=np.int64))


def select_tiles(w: np.ndarray, TX: int, TY: int, W: int, H: int, n_sel: int,
                 seed: int, step: int, view: int, tile_pred=None) -> np.ndarray:
    """Tiles drawn without replacement with probability proportional to their
    error-map sums (or to the predicted errors when tile_pred is given)."""
    n_t = TX * TY
    if n_sel < 0 or n_sel >= n_t:
        return np.arange(n_t, dtype=np.int64)
    if tile_pred is not None:
        tw = predicted_tile_weights(tile_pred, TX, TY, W, H)
    else:
        tw = np.zeros(n_t, dtype=np.int64)
        for t in range(n_t):
            _, x, y = tile_pixels(t, TX, W, H)
            tw[t] = int(w[y, x].sum())
    return race_select(tw, n_sel, seed, step, view)


def sample_tile(w: np.ndarray, A: np.ndarray, tile: int, TX: int, W: int, H: int,
                sp: SampleParams, seed: int, step: int, view: int):
    """Hard, stable and mixed local indices of one tile (each set sorted)."""
    loc, x, y = tile_pixels(tile, TX, W, H)
    wt = w[y, x]
    at = A[y, x].astype(np.int64)
    n = min(sp.n_pix, loc.size)
    n_hard, n_stable, n_mixed = split_counts(n, sp.hard_permille, sp.stable_permille)

    free = np.ones(loc.size, dtype=bool)
    hard = []
    for j in range(n_hard):
        cand = np.nonzero(free)[0]
        wc = wt[cand]
        if int(wc.sum()) == 0:
            break
        k = cand[_pick_weighted(wc, draw(seed, step, view, tile, j))]
        free[k] = False
        hard.append(k)
    n_mixed += n_hard - len(hard)

    cand = np.nonzero(free)[0]
    order = np.lexsort((cand, -at[cand]))      # age descending, then index ascending
    stable = cand[order[:n_stable]]
    free[stable] = False

    mixed = []
    for j in range(n_mixed):
        cand = np.nonzero(free)[0]
        k = cand[below(draw(seed, step, view, tile, 256 + j), cand.size)]
        free[k] = False
        mixed.append(k)
    return (np.sort(loc[np.array(hard, dtype=np.int64)]), np.sort(loc[stable]),
            np.sort(loc[np.array(mixed, dtype=np.int64)]))


def sample_view(E_bits: np.ndarray, A: np.ndarray, sp: SampleParams, seed: int, step: int,
                view: int, tiles_subset=None, tile_pred=None) -> dict:
    """Sparse sample set of one view.

    Returns valid_tiles [n_st] (ascending tile ids), tile_off [n_st + 1],
    pix [P] (uint8 local indices, ascending within each tile) and the per-tile
    hard/stable/mixed sets.  ``tiles_subset`` restricts the per-tile pass to
    some of the selected tiles (for sampled checks at full size); offsets then
    cover only those tiles.  ``tile_pred`` (per tile, optional) replaces the
    error-map sums in the tile pass by predicted tile errors.
    """
    H, W = E_bits.shape
    TX, TY = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    w = half_weights(E_bits)
    A = np.asarray(A)
    tiles = select_tiles(w, TX, TY, W, H, sp.n_tiles_sel, seed, step, view, tile_pred)
    if tiles_subset is not None:
        keep = set(int(s) for s in tiles_subset)
        tiles = np.array([t for t in tiles if int(t) in keep], dtype=np.int64)
    pix, off, sets = [], [0], []
    for t in tiles:
        h, s, m = sample_tile(w, A, int(t), TX, W, H, sp, seed, step, view)
        allp = np.sort(np.concatenate([h, s, m]))
        pix.append(allp)
        off.append(off[-1] + allp.size)
        sets.append((h, s, m))
    return dict(valid_tiles=tiles.astype(np.int32), tile_off=np.array(off, dtype=np.int32),
                pix=(np.concatenate(pix) if pix else np.zeros(0)).astype(np.uint8),
                sets=sets, TX=TX, TY=TY)


def sample_coords(samples: dict, W: int, H: int):
    """Pixel coordinates (x, y) and owning slot of every sample."""
    TX = samples["TX"]
    off = samples["tile_off"]
    tiles = samples["valid_tiles"]
    slot = np.repeat(np.arange(tiles.size), np.diff(off))
    t = tiles[slot].astype(np.int64)
    loc = samples["pix"].astype(np.int64)
    x = (t % TX) * TILE + loc % TILE
    y = (t // TX) * TILE + loc // TILE
    return x, y, slot
