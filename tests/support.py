"""Helpers shared by the GPU parity tests: seeded scenes, conversion of oracle
stage outputs into the library's input layouts, and tolerance checks.

Every GPU stage is fed inputs that come from ``synth`` or from the oracle,
never from another GPU stage, so each comparison isolates one kernel."""
from __future__ import annotations

import numpy as np

import synth
from oracle import binning, project, render, sampler
from oracle.params import RasterParams, SampleParams

TILE = 16


def scene_c1(n=10000):
    """The tiny workload: 10k Gaussians, four 256x256 tetrahedron views."""
    return synth.gaussians(n, synth.SEED_SCENE), synth.tetra_cameras()


def scene_scaling(n=300000):
    """The rasterizer-scaling workload: 300k Gaussians, one 1296x840 view."""
    return synth.gaussians(n, synth.SEED_SCENE), synth.config_camera("scaling")


def small_scene(n=400, seed=21, W=150, H=107):
    """A few hundred Gaussians over a ragged image (partial edge tiles)."""
    p = synth.gaussians(n, seed, logscale_mean=-3.3)
    cam = synth.look_at((2.4, -1.1, 1.3), fx=W * 1.2, fy=W * 1.2, width=W, height=H)
    return p, cam


def ldl_conic(conic: np.ndarray) -> np.ndarray:
    """The record's conic form: Q = [[a, b], [b, c]] as (a, beta = b / a,
    delta = c - b beta), so that d^T Q d = a (dx + beta dy)^2 + delta dy^2
    (zero where a is not positive)."""
    a, b, c = (np.asarray(conic[i], dtype=np.float64) for i in range(3))
    ok = a > 0
    beta = np.where(ok, b / np.where(ok, a, 1.0), 0.0)
    delta = np.where(ok, c - b * beta, 0.0)
    return np.stack([a, beta, delta])


def natural_conic(rec: np.ndarray) -> np.ndarray:
    """(a, b, c) from the record's FP32 (a, beta, delta), in FP64."""
    a, beta, delta = (rec[:, 4 + i].astype(np.float64) for i in range(3))
    b = beta * a
    return np.stack([a, b, delta + beta * b])


def splat_record(pr: dict) -> np.ndarray:
    """The library's [N, 12] splat record built from an oracle projection."""
    N = pr["opacity"].size
    s = np.zeros((N, 12), dtype=np.float32)
    px, py = pr["mean2d"]
    fx, fy = np.floor(px), np.floor(py)
    s[:, 0], s[:, 1] = fx, fy
    s[:, 2], s[:, 3] = px - fx, py - fy
    s[:, 4:7] = ldl_conic(pr["conic"]).T
    s[:, 7] = pr["opacity"]
    s[:, 8:11] = pr["rgb"].T
    s[:, 11] = pr["depth32"]
    vis = pr["visible"]
    s[~vis, :11] = 0.0
    return s


def splat_as_oracle(pr: dict, rec: np.ndarray) -> dict:
    """An oracle projection dict whose 2D splat values are the FP32 record
    widened back to FP64 (so both sides composite identical splats)."""
    q = dict(pr)
    q["mean2d"] = np.stack([rec[:, 0].astype(np.float64) + rec[:, 2], rec[:, 1].astype(np.float64) + rec[:, 3]])
    q["conic"] = natural_conic(rec)
    q["opacity"] = rec[:, 7].astype(np.float64)
    q["rgb"] = rec[:, 8:11].T.astype(np.float64)
    return q


def samples_dict(s: dict):
    return s["valid_tiles"], s["tile_off"], s["pix"]


MOMENT_STRIDE = 64  # the library's Gaussian-major moment layout, [n][64]


def moments_gaussian_major(m: np.ndarray) -> np.ndarray:
    """[59][n] moments (the oracle's layout) as the library's [n][64] array
    (padding zero)."""
    out = np.zeros((m.shape[1], MOMENT_STRIDE), dtype=np.float32)
    out[:, : m.shape[0]] = m.T
    return out


def moments_rows(m: np.ndarray, rows: int = 59) -> np.ndarray:
    """The library's [n][64] moments as [59][n] (the oracle's layout)."""
    return np.ascontiguousarray(np.asarray(m)[:, :rows].T)


def close(a, b, rtol, atol=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b)
    bound = rtol * np.abs(b) + atol
    bad = err > bound
    return (~bad).all(), err, bound, bad


def assert_close(a, b, rtol, atol=0.0, what=""):
    ok, err, bound, bad = close(a, b, rtol, atol)
    if not ok:
        i = np.argmax(err - bound)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside tolerance; worst index {i}: "
                             f"got {np.asarray(a).ravel()[i]!r}, want {np.asarray(b).ravel()[i]!r}, "
                             f"max rel {np.max(err / np.maximum(np.abs(b), 1e-30)):.3g}")


def check_pair_lists(vals, ranges, n_pairs, pr: dict, valid_tiles=None, keys=None, alpha_min=1.0 / 255.0,
                     max_dropped_checked: int | None = None, seed: int = 0, tiles_subset=None) -> dict:
    """Checks a GPU pair list (vals [n_pairs] ids, ranges [n_tiles][2], keys
    optional) against the oracle's rectangle lists of the projection ``pr``:

    * ranges partition [0, n_pairs) in ascending tile order (empty: [0, 0)),
      and only valid tiles hold pairs;
    * within the whole list, (tile, depth bits, id) strictly increases, and
      every (tile, id) pair is a pair of the oracle's list, so each tile's
      GPU list is an order-preserving subsequence of the oracle's;
    * the keys, when given, are (tile << 32) | bits of the oracle's FP32 depth;
    * every pair the GPU list drops can composite nowhere in its tile: the
      oracle's o exp(power) stays below alpha_min (1 - 1e-3) at all 256 pixel
      centres (evaluated for all dropped pairs, or a seeded sample of
      ``max_dropped_checked``).

    With ``tiles_subset`` the membership and dropped-pair checks cover those
    tiles only (the order, key and range checks still cover the whole list).
    Returns counts (GPU pairs, oracle pairs, dropped, dropped checked)."""
    vals = np.asarray(vals, dtype=np.uint32)[:n_pairs].astype(np.int64)
    ranges = np.asarray(ranges, dtype=np.int64).reshape(-1, 2)
    n_t = pr["TX"] * pr["TY"]
    assert ranges.shape[0] == n_t
    listed = np.arange(n_t) if valid_tiles is None else np.asarray(valid_tiles, dtype=np.int64)
    if tiles_subset is not None:
        listed = np.intersect1d(listed, np.asarray(tiles_subset, dtype=np.int64))
    sk, sv, _ = binning.bin_and_sort(pr, listed)
    # ranges: contiguous, ascending, covering exactly n_pairs; tile of each position
    cnt = ranges[:, 1] - ranges[:, 0]
    assert (cnt >= 0).all()
    ne = np.nonzero(cnt > 0)[0]
    assert (ranges[cnt == 0] == 0).all()
    starts = np.concatenate([[0], np.cumsum(cnt[ne])[:-1]]) if ne.size else np.zeros(0, np.int64)
    assert np.array_equal(ranges[ne, 0], starts) and int(cnt.sum()) == n_pairs
    if valid_tiles is not None:
        valid = np.zeros(n_t, dtype=bool)
        valid[np.asarray(valid_tiles, dtype=np.int64)] = True
        assert valid[ne].all()
    tile = np.repeat(ne, cnt[ne])
    bits = np.asarray(pr["depth32"], dtype=np.float32).view(np.uint32).astype(np.int64)
    if keys is not None:
        k = np.asarray(keys).view(np.uint64)[:n_pairs]
        assert np.array_equal(k, (tile.astype(np.uint64) << np.uint64(32)) | bits[vals].astype(np.uint64))
    # strictly increasing (tile, depth bits, id)
    if n_pairs > 1:
        t0, t1 = tile[:-1], tile[1:]
        d0, d1 = bits[vals[:-1]], bits[vals[1:]]
        inc = (t0 < t1) | ((t0 == t1) & ((d0 < d1) | ((d0 == d1) & (vals[:-1] < vals[1:]))))
        assert inc.all()
    # membership in the oracle's (tile, id) pairs
    code_o = ((sk >> np.uint64(32)).astype(np.int64) << 32) | sv.astype(np.int64)
    code_o_sorted = np.sort(code_o)
    code_g = (tile << 32) | vals
    if tiles_subset is not None:
        code_g = code_g[np.isin(tile, listed)]
    pos = np.searchsorted(code_o_sorted, code_g)
    assert (pos < code_o_sorted.size).all() and np.array_equal(code_o_sorted[np.minimum(pos, code_o_sorted.size - 1)],
                                                               code_g)
    dropped = np.setdiff1d(code_o_sorted, code_g, assume_unique=True)
    chk = dropped
    if max_dropped_checked is not None and dropped.size > max_dropped_checked:
        chk = np.random.default_rng(seed).choice(dropped, max_dropped_checked, replace=False)
    if chk.size:
        amax = binning.max_alpha_in_tile(pr, chk & 0xFFFFFFFF, chk >> 32)
        assert (amax < alpha_min * (1.0 - 1e-3)).all(), float(amax.max() / alpha_min)
    return dict(gpu=int(code_g.size), oracle=int(sk.size), dropped=int(dropped.size), checked=int(chk.size))


def last_ids_two_part(vals, ranges, vals2, ranges2, tiles, ncontrib) -> np.ndarray:
    """last_ids over two-part lists (a tile's list is vals[ranges[t]]
    followed by vals2[ranges2[t]])."""
    vals = np.asarray(vals).astype(np.int64)
    vals2 = np.asarray(vals2).astype(np.int64)
    r1 = np.asarray(ranges, dtype=np.int64).reshape(-1, 2)[np.asarray(tiles, dtype=np.int64)]
    r2 = np.asarray(ranges2, dtype=np.int64).reshape(-1, 2)[np.asarray(tiles, dtype=np.int64)]
    pos = np.asarray(ncontrib).astype(np.int64) - 1
    n1 = r1[:, 1] - r1[:, 0]
    first = np.clip(r1[:, 0] + pos, 0, max(vals.size - 1, 0))
    second = np.clip(r2[:, 0] + pos - n1, 0, max(vals2.size - 1, 0))
    ids = np.where(pos < n1, vals[first] if vals.size else -1, vals2[second] if vals2.size else -1)
    return np.where(pos >= 0, ids, -1)


def last_ids(vals, ranges, tiles, ncontrib) -> np.ndarray:
    """The id of the last composited Gaussian of each pixel (-1 when none):
    the ncontrib-th entry of the pixel's tile list.  Unique for a pixel
    whatever Gaussians that cannot composite its list holds."""
    vals = np.asarray(vals).astype(np.int64)
    ranges = np.asarray(ranges, dtype=np.int64).reshape(-1, 2)
    nc = np.asarray(ncontrib).astype(np.int64)
    idx = ranges[np.asarray(tiles, dtype=np.int64), 0] + nc - 1
    return np.where(nc > 0, vals[np.clip(idx, 0, max(vals.size - 1, 0))], -1)
