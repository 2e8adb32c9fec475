"""Pins of the oracle's keys/sort/ranges (library sort, loops) and of its
sampler (reference RNG values, invariants, exact inclusion probabilities by
enumeration, frequency tests)."""
import itertools
import math
import os

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
    fields, tau = binning.splat_fields(pr), binning.cull_threshold(1.0 / 255.0)
    for vt in (None, valid):
        for f, t in ((None, None), (fields, tau)):
            k1, v1 = binning.emit_pairs(pr["rect"], pr["depth32"], TX, TY, vt, f, t)
            k2, v2 = binning.emit_pairs_fast(pr["rect"], pr["depth32"], TX, TY, vt, f, t)
            assert np.array_equal(k1, k2) and np.array_equal(v1, v2)


def test_cull_threshold():
    # 2 ln(255) = 11.0825..., plus 0.1 %, rounded up to 1/64
    assert binning.cull_threshold(1.0 / 255.0) == 710 / 64
    for a in (1e-3, 1.0 / 255.0, 0.01, 0.1):
        t = binning.cull_threshold(a)
        assert 2 * math.log(1 / a) * 1.001 <= t < 2 * math.log(1 / a) * 1.001 + 1 / 64
        assert (t * 64) == int(t * 64)


def test_cull_never_drops_a_compositing_pixel():
    """Brute force over every pixel centre of every culled rect tile: with
    the largest opacity (1) the Gaussian's alpha stays below alpha_min."""
    amin = 1.0 / 255.0
    tau = binning.cull_threshold(amin)
    culled_total = 0
    for seed, lm in ((2, -3.0), (4, -2.5), (6, -3.5)):
        p = synth.gaussians(400, seed, logscale_mean=lm)
        cam = synth.look_at((2.0, -1.5, 1.2), fx=105.6, fy=105.6, width=96, height=76)
        pr = project.project(p, cam)
        f = binning.splat_fields(pr)
        gid, tx, ty = binning.rect_tiles(pr["rect"])
        g = {k: v[gid] for k, v in f.items()}
        keep = binning.tile_touches(tx, ty, g["xi"], g["xf"], g["yi"], g["yf"], g["A"], g["B"], g["C"], tau)
        lx, ly = np.meshgrid(np.arange(16.0), np.arange(16.0))
        for j in np.nonzero(~keep)[0]:
            dx = (16 * tx[j] + lx) - (g["xi"][j] + g["xf"][j])
            dy = (16 * ty[j] + ly) - (g["yi"][j] + g["yf"][j])
            q = g["A"][j] * dx * dx + 2 * g["B"][j] * dx * dy + g["C"][j] * dy * dy
            assert (np.exp(-0.5 * q) < amin).all()
        culled_total += int((~keep).sum())
        assert (~keep).mean() > 0.15          # the test does remove pairs
    assert culled_total > 100


def test_cull_matches_dense_rectangle_minimum():
    """Random SPD conics and rectangles: the decision agrees with the minimum
    of q over a dense grid of the rectangle wherever that minimum is clearly
    below or above tau (a dropped factor, sign or swapped axis fails)."""
    rng = np.random.default_rng(11)
    tau = 11.0
    n_in = n_out = 0
    for _ in range(400):
        th = rng.uniform(0, np.pi)
        s1, s2 = np.exp(rng.uniform(-1, 3, size=2))
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        Sig = R @ np.diag([s1 * s1, s2 * s2]) @ R.T
        Q = np.linalg.inv(Sig)
        A, B, C = Q[0, 0], Q[0, 1], Q[1, 1]
        cx, cy = rng.uniform(-60, 60, size=2)
        xi, xf = np.floor(cx), cx - np.floor(cx)
        yi, yf = np.floor(cy), cy - np.floor(cy)
        tx, ty = rng.integers(-3, 3, size=2)
        keep = bool(binning.tile_touches(tx, ty, xi, xf, yi, yf, A, B, C, tau))
        gx = np.linspace(16 * tx, 16 * tx + 15, 301) - cx
        gy = np.linspace(16 * ty, 16 * ty + 15, 301) - cy
        X, Y = np.meshgrid(gx, gy)
        qmin = (A * X * X + 2 * B * X * Y + C * Y * Y).min()
        if qmin < 0.98 * tau:
            assert keep
            n_in += 1
        elif qmin > 1.05 * tau + 0.5:
            assert not keep
            n_out += 1
    assert n_in > 30 and n_out > 30


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

