"""Pins of the oracle's keys/sort/ranges (library sort, loops) and of its
sampler (reference RNG values, invariants, exact inclusion probabilities by
enumeration, frequency tests)."""
import itertools
import math
import os
import struct
from decimal import Decimal, getcontext

import numpy as np
import pytest

import synth
from oracle import binning, project, rng, sampler
from oracle.params import SampleParams, pixels_per_tile, split_counts

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- binning
def _scene(n=300, seed=2, size=96):
    p = synth.gaussians(n, seed, logscale_mean=-3.0)
    cam = synth.look_at((2.0, -1.5, 1.2), fx=size * 1.1, fy=size * 1.1, width=size, height=size - 20)
    return p, cam, project.project(p, cam)


def test_emit_loop_equals_vectorised():
    _, cam, pr = _scene()
    TX, TY = pr["TX"], pr["TY"]
    valid = np.array([0, 3, 5, 6, 7, 11, TX * TY - 1])
    for vt in (None, valid):
        k1, v1 = binning.emit_pairs(pr["rect"], pr["depth32"], TX, TY, vt)
        k2, v2 = binning.emit_pairs_fast(pr["rect"], pr["depth32"], TX, TY, vt)
        assert np.array_equal(k1, k2) and np.array_equal(v1, v2) and k1.size > 100


def _rect_brute(px, py, r, TX, TY):
    """The tiles whose 16-pixel span meets the closed interval [p - r, p + r - 1]
    on both axes, found by walking every tile of the grid."""
    xs = [tx for tx in range(TX) if 16 * tx <= px + r - 1 and px - r < 16 * tx + 16]
    ys = [ty for ty in range(TY) if 16 * ty <= py + r - 1 and py - r < 16 * ty + 16]
    return (xs[0], ys[0], xs[-1] + 1, ys[-1] + 1) if xs and ys else None


def test_tile_rectangle_brute_force():
    """The rectangle of the projection is exactly the set of tiles meeting
    [p - r, p + r - 1] on each axis (grid walk), and it holds every pixel
    index within that interval: pixel centres up to r - 1 from the centre on
    the right and r on the left (the 3D Gaussian splatting +15 rounding of
    the upper bound).  Checked on a projected scene and on hand-placed
    centres on and near tile boundaries, inside and outside the image."""
    TX, TY = 6, 5
    cases = []
    for px in (-20.0, -0.5, 0.0, 15.0, 15.5, 16.0, 31.999, 40.25, 95.0, 96.0, 120.0):
        for py in (-3.0, 0.0, 16.0, 47.5, 79.0, 80.0):
            for r in (1, 3, 8, 16, 17, 40):
                cases.append((px, py, r))
    _, cam, pr = _scene()
    vis = np.nonzero(pr["visible"])[0]
    assert vis.size > 200
    for g in vis:
        want = _rect_brute(pr["mean2d"][0][g], pr["mean2d"][1][g], int(pr["radius"][g]), pr["TX"], pr["TY"])
        got = tuple(int(v) for v in pr["rect"][:, g])
        assert want is not None and got == want, (g, got, want)
    n_empty = 0
    for px, py, r in cases:
        got = project.rect_of((px, py), r, TX, TY)
        want = _rect_brute(px, py, r, TX, TY)
        if want is None:
            assert got[0] >= got[2] or got[1] >= got[3], (px, py, r, got)
            n_empty += 1
            continue
        assert got == want, (px, py, r, got, want)
        for i in range(int(np.ceil(px - r)), int(np.floor(px + r - 1)) + 1):
            for j in range(int(np.ceil(py - r)), int(np.floor(py + r - 1)) + 1):
                if 0 <= i < 16 * TX and 0 <= j < 16 * TY:
                    assert got[0] <= i // 16 < got[2] and got[1] <= j // 16 < got[3]
    assert n_empty > 10 and len(cases) - n_empty > 300


def test_max_alpha_in_tile_brute_force():
    """The per-tile maximum of o exp(power) against a pixel-by-pixel loop,
    and two closed forms: a splat centred on a pixel centre of the tile
    reaches o there; one centred 40 pixels left of the tile at sigma 4
    reaches o exp(-(40 - 0)^2 / 32) at the tile's first column."""
    _, cam, pr = _scene()
    gid, tx, ty = binning.rect_tiles(pr["rect"])
    tiles = ty * pr["TX"] + tx
    pick = np.random.default_rng(3).choice(gid.size, 60, replace=False)
    got = binning.max_alpha_in_tile(pr, gid[pick], tiles[pick], chunk=7)
    for k, j in enumerate(pick):
        g, t = gid[j], tiles[j]
        best = 0.0
        for ly in range(16):
            for lx in range(16):
                dx = 16 * (t % pr["TX"]) + lx - pr["mean2d"][0][g]
                dy = 16 * (t // pr["TX"]) + ly - pr["mean2d"][1][g]
                a, b, c = pr["conic"][:, g]
                best = max(best, pr["opacity"][g] * math.exp(-0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy))
        assert abs(got[k] - best) <= 1e-15 * max(best, 1e-300), (k, got[k], best)
    iso = dict(mean2d=np.array([[21.0, 16.0 - 40.0], [9.0, 9.0]]), conic=np.array([[1 / 16, 1 / 16], [0, 0],
                                                                                      [1 / 16, 1 / 16]]),
               opacity=np.array([0.7, 0.9]), TX=3)
    m = binning.max_alpha_in_tile(iso, [0, 1], [1, 1])
    assert m[0] == 0.7 and abs(m[1] - 0.9 * math.exp(-0.5 * 40.0 ** 2 / 16)) < 1e-30


def test_sort_and_ranges_against_python():
    _, cam, pr = _scene()
    TX, TY = pr["TX"], pr["TY"]
    keys, vals = binning.emit_pairs(pr["rect"], pr["depth32"], TX, TY)
    sk, sv = binning.sort_pairs(keys, vals)
    ref = sorted(zip(keys.tolist(), vals.tolist()))
    assert [int(k) for k in sk] == [r[0] for r in ref]
    assert [int(v) for v in sv] == [r[1] for r in ref]
    ranges = binning.tile_ranges(sk, TX * TY)
    for t in range(TX * TY):
        members = [i for i, k in enumerate(sk.tolist()) if (k >> 32) == t]
        if members:
            assert (ranges[t, 0], ranges[t, 1]) == (members[0], members[-1] + 1)
        else:
            assert (ranges[t] == 0).all()
        # within a tile the order is by depth (the FP32 bits order like the depth)
        d = pr["depth"][sv[ranges[t, 0]:ranges[t, 1]]]
        assert (np.diff(d) >= 0).all()


# ---------------------------------------------------------------- rng
def test_splitmix64_reference_values():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [rng.mix64(k * rng.GAMMA) for k in (1, 2, 3)] == vals


def test_below_is_floor_of_scaled_draw():
    for u in (0, 1, (1 << 63), (1 << 64) - 1):
        for n in (1, 7, 256, (1 << 48) + 3):
            assert rng.below(u, n) == (u * n) // (1 << 64)
            assert 0 <= rng.below(u, n) < n


# ---------------------------------------------------------------- counts
def test_pixel_budget_formulas():
    assert [pixels_per_tile(r) for r in (1000, 500, 250, 200, 150, 100, 1)] == [256, 128, 64, 51, 38, 25, 1]
    assert split_counts(64, 400, 300) == (26, 19, 19)
    assert split_counts(51, 400, 300) == (20, 15, 16)
    assert split_counts(25, 400, 300) == (10, 8, 7)
    assert split_counts(128, 400, 300) == (51, 38, 39)
    assert split_counts(256, 400, 300) == (102, 77, 77)
    for n in range(1, 257):
        h, s, m = split_counts(n, 400, 300)
        assert h + s + m == n and min(h, s, m) >= 0


def test_half_weights_exact():
    vals = np.array([0.0, 2.0 ** -24, 1.0, 65504.0, -1.0, np.inf, np.nan, 0.4], dtype=np.float16)
    w = sampler.half_weights(vals.view(np.uint16))
    assert w.tolist() == [0, 1, 1 << 24, 65504 << 24, 0, 0, 0, int(float(np.float16(0.4)) * (1 << 24))]


# ---------------------------------------------------------------- sampler invariants
@pytest.mark.parametrize("W,H,n_pix,n_sel", [(80, 56, 64, -1), (64, 64, 25, 5), (70, 40, 256, -1),
                                              (48, 48, 51, 3)])
def test_sampler_invariants(W, H, n_pix, n_sel):
    E = synth.error_map(H, W, 11, zero_frac=0.3)
    A = synth.age_map(H, W, 12)
    sp = SampleParams(n_pix=n_pix, n_tiles_sel=n_sel)
    s1 = sampler.sample_view(E, A, sp, seed=3, step=7, view=1)
    s2 = sampler.sample_view(E, A, sp, seed=3, step=7, view=1)
    assert all(np.array_equal(s1[k], s2[k]) for k in ("valid_tiles", "tile_off", "pix"))
    TX, TY = s1["TX"], s1["TY"]
    vt = s1["valid_tiles"]
    assert (np.diff(vt) > 0).all()
    assert vt.size == (TX * TY if n_sel < 0 else n_sel)
    w = sampler.half_weights(E)
    for i, t in enumerate(vt):
        loc, x, y = sampler.tile_pixels(int(t), TX, W, H)
        got = s1["pix"][s1["tile_off"][i]:s1["tile_off"][i + 1]].astype(int)
        assert (np.diff(got) > 0).all()
        assert set(got) <= set(loc.tolist())
        assert got.size == min(n_pix, loc.size)
        h, st, m = s1["sets"][i]
        assert len(set(h) | set(st) | set(m)) == len(h) + len(st) + len(m) == got.size
        wl = dict(zip(loc.tolist(), w[y, x].tolist()))
        assert all(wl[int(k)] > 0 for k in h)               # zero-weight pixels are never hard
        n_h, n_s, _ = split_counts(got.size, 400, 300)
        assert len(st) == n_s and len(h) <= n_h
        # stable = TopK age among the pixels not drawn as hard (library sort)
        al = dict(zip(loc.tolist(), A[y, x].tolist()))
        rest = sorted((k for k in loc.tolist() if k not in set(h.tolist())), key=lambda k: (-al[k], k))
        assert list(st) == sorted(rest[:n_s])
    # a different seed changes the draw
    s3 = sampler.sample_view(E, A, sp, seed=4, step=7, view=1)
    assert not np.array_equal(s1["pix"], s3["pix"]) or n_pix == 256


def test_exhausted_weights_move_hard_slots_to_mixed():
    W = H = 16
    E = np.zeros((H, W), dtype=np.float16)
    E[0, :3] = 1.0                                    # only three pixels carry error
    A = np.zeros((H, W), dtype=np.uint16)
    s = sampler.sample_view(E.view(np.uint16), A, SampleParams(n_pix=64), 1, 1, 0)
    h, st, m = s["sets"][0]
    assert sorted(h.tolist()) == [0, 1, 2]
    assert len(st) == 19 and len(m) == 64 - 3 - 19


def _inclusion_exact(weights, k):
    """P(pixel in the first k sequential draws without replacement, prob. proportional
    to the weights) by enumerating every ordered draw sequence."""
    n = len(weights)
    inc = np.zeros(n)
    for seq in itertools.permutations(range(n), k):
        p, rem = 1.0, float(sum(weights))
        for i in seq:
            p *= weights[i] / rem
            rem -= weights[i]
        for i in seq:
            inc[i] += p
    return inc


def test_hard_draw_inclusion_probabilities_match_enumeration():
    """On a 5-pixel tile (a 5x1 image) with n_pix=5 -> N_hard = 2, the hard set's
    inclusion frequencies over many seeds match the exact sequential
    without-replacement probabilities (chi-square)."""
    E = np.array([[0.5, 1.0, 2.0, 0.25, 4.0]], dtype=np.float16)
    A = np.zeros((1, 5), dtype=np.uint16)
    sp = SampleParams(n_pix=5)
    wts = [float(v) for v in E[0]]
    exact = _inclusion_exact(wts, 2)
    n_seeds = 20000
    counts = np.zeros(5)
    first = np.zeros(5)
    for seed in range(n_seeds):
        h, _, _ = sampler.sample_tile(sampler.half_weights(E.view(np.uint16)), A, 0, 1, 5, 1, sp, seed, 0, 0)
        counts[h] += 1
        u = rng.draw(seed, 0, 0, 0, 0)
        first[np.searchsorted(np.cumsum(wts), rng.below(u, int(sum(wts) * 2 ** 24)) / 2 ** 24, side="right")] += 1
    expected = exact * n_seeds
    chi2 = (((counts - expected) ** 2) / expected).sum()
    assert chi2 < 20.5            # 5 cells; p ~ 0.001 threshold for 4 dof is 18.5, margin for dependence
    pf = np.array(wts) / sum(wts)
    chi2_first = (((first - pf * n_seeds) ** 2) / (pf * n_seeds)).sum()
    assert chi2_first < 18.5


def test_tile_pass_prefers_high_error_tiles():
    W = H = 64                                           # 16 tiles
    E = np.full((H, W), 0.01, dtype=np.float16)
    E[:16, :16] = 5.0                                    # tile 0 dominates
    A = np.zeros((H, W), dtype=np.uint16)
    hits = 0
    for seed in range(200):
        s = sampler.sample_view(E.view(np.uint16), A, SampleParams(n_pix=8, n_tiles_sel=2), seed, 0, 0)
        hits += 0 in s["valid_tiles"].tolist()
    assert hits > 190


def test_predicted_tile_weights_and_selection():
    """Predicted tile errors: weights floor(clamp(p, 0, 65504) * pixels * 2^24)
    (partial edge tiles count their in-image pixels); when exactly k tiles
    have a positive prediction, a pass drawing k tiles takes exactly them."""
    W, H = 40, 37
    TX, TY = 3, 3
    pred = np.array([0.5, -1.0, np.nan, 1e30, 0.25, 0.0, 2.0 ** -20, 1.0, 0.125], dtype=np.float32)
    tw = sampler.predicted_tile_weights(pred, TX, TY, W, H)
    px = [16 * 16, 16 * 16, 16 * 8, 16 * 16, 16 * 16, 16 * 8, 5 * 16, 5 * 16, 5 * 8]
    want = [int(0.5 * px[0] * 2 ** 24), 0, 0, int(65504 * px[3] * 2 ** 24), int(0.25 * px[4] * 2 ** 24), 0,
            int(2.0 ** -20 * px[6] * 2 ** 24), int(1.0 * px[7] * 2 ** 24), int(0.125 * px[8] * 2 ** 24)]
    assert tw.tolist() == want
    E = synth.error_map(H, W, 5)
    A = synth.age_map(H, W, 6)
    hot = np.zeros(TX * TY, dtype=np.float32)
    hot[[1, 4, 8]] = [0.3, 0.01, 2.0]
    for seed in range(5):
        s = sampler.sample_view(E, A, SampleParams(n_pix=16, n_tiles_sel=3), seed, 1, 0, tile_pred=hot)
        assert s["valid_tiles"].tolist() == [1, 4, 8]



# ---------------------------------------------------------------- tile pass: exponential race
def test_neg_log2_fixed_against_decimal():
    """The fixed-point -log2 of a uniform against a 50-digit decimal logarithm:
    within 2^-46 (47 fractional bits, truncated), at the extremes of v = u | 1
    and on random draws."""
    getcontext().prec = 50
    ln2 = Decimal(2).ln()
    us = [0, 1, 2, 3, (1 << 63) - 1, 1 << 63, (1 << 63) + 1, (1 << 64) - 2, (1 << 64) - 1, 1 << 32,
          0x5555555555555555, 0xAAAAAAAAAAAAAAAA] + [rng.draw(9, 1, 2, 3, k) for k in range(300)]
    for u in us:
        v = u | 1
        exact = -(Decimal(v) / Decimal(2 ** 64)).ln() / ln2
        got = Decimal(sampler.neg_log2_fixed(u)) / Decimal(2 ** sampler.LOG_FRAC)
        assert abs(got - exact) <= Decimal(2) ** -46, (u, got, exact)
    assert sampler.neg_log2_fixed(1 << 63) == 1 << sampler.LOG_FRAC        # -log2(1/2) = 1
    assert sampler.neg_log2_fixed(0) == 64 << sampler.LOG_FRAC             # v = 1: 64 exactly
    assert sampler.neg_log2_fixed((1 << 64) - 1) >= 1                      # times stay positive


def test_tile_race_inclusion_matches_sequential_enumeration():
    """The race's inclusion frequencies over many seeds match the exact
    probabilities of sequential draws without replacement proportional to
    weight (chi-square over 5 tiles); uniform (not exponential) race times or
    times multiplied by the weight fail this by orders of magnitude."""
    wts = [1, 2, 4, 8, 3]
    tw = [x << 24 for x in wts]
    exact = _inclusion_exact(wts, 2)
    n_seeds = 10000
    counts = np.zeros(5)
    for seed in range(n_seeds):
        counts[sampler.race_select(tw, 2, seed, 0, 0)] += 1
    expected = exact * n_seeds
    assert (((counts - expected) ** 2) / expected).sum() < 20.5


def test_tile_race_zero_weights_come_last_and_uniform():
    """Weighted tiles always precede zero-weight ones (the sequential draws
    take a zero-weight tile only once the weight has run out), and the
    zero-weight tiles that fill the rest are a uniform subset."""
    tw = [3 << 24, 0, 1 << 24, 0, 2 << 24, 0]
    counts = np.zeros(6)
    n_seeds = 3000
    for seed in range(n_seeds):
        got = sampler.race_select(tw, 4, seed, 1, 2)
        assert {0, 2, 4} <= set(got.tolist())
        counts[got] += 1
    # each zero-weight tile joins with probability 1/3: 3 sigma ~ 0.026
    assert np.all(np.abs(counts[[1, 3, 5]] / n_seeds - 1 / 3) < 0.03)
    assert sampler.race_select([0] * 5, 0, 1, 1, 1).size == 0
    # all weights zero: uniform over every 2-subset of 4 tiles (6 subsets)
    pairs = {}
    for seed in range(3000):
        key = tuple(sampler.race_select([0, 0, 0, 0], 2, seed, 0, 0).tolist())
        pairs[key] = pairs.get(key, 0) + 1
    assert len(pairs) == 6 and all(abs(c / 3000 - 1 / 6) < 0.025 for c in pairs.values())


def test_tile_race_keys_order_and_ties(monkeypatch):
    """Key layout: a weighted tile's key is the bit pattern of L / w (larger
    weight, earlier run for the same L), every zero-weight key is >= 2^63;
    equal keys fall back to the tile index."""
    tw = [5, 0, 1 << 40, 7]
    keys = sampler.tile_race_keys(tw, 4, 5, 6)
    for t in (0, 2, 3):
        u = rng.draw(4, 5, 6, 4, t)
        want = float(sampler.neg_log2_fixed(u)) / float(tw[t])
        assert keys[t] == struct.unpack("<Q", struct.pack("<d", want))[0] < (1 << 63)
    assert keys[1] >= 1 << 63
    # identical keys (forced) keep index order
    monkeypatch.setattr(sampler, "tile_race_keys", lambda tw, *a: [7, 7, 3, 7])
    assert sampler.race_select([1, 1, 1, 1], 2, 0, 0, 0).tolist() == [0, 2]
