"""Pins of the density-control oracle (Sec. 3.8, Eq. gauss_err_accum and
Eq. gauss_score) against closed forms and invariants of compositing (CPU only)."""
import math

import numpy as np

import synth
from oracle import binning, density, project, render, sampler
from oracle.params import RasterParams, SampleParams

from support import small_scene


def _proj(centres, sigma, opacity, TX=1):
    """A hand-built projection: isotropic splats with conic I / sigma^2."""
    n = len(opacity)
    c = np.asarray(centres, dtype=np.float64).T
    return dict(mean2d=c, conic=np.stack([np.full(n, 1 / sigma ** 2), np.zeros(n), np.full(n, 1 / sigma ** 2)]),
                opacity=np.asarray(opacity, dtype=np.float64), rgb=np.zeros((3, n)), TX=TX)


def test_two_splats_at_one_pixel_closed_form():
    # pixel (3, 4); splat 0 at (3, 2), splat 1 at (6, 8): |d| = 2 and 5
    sigma = 2.5
    pr = _proj([(3.0, 2.0), (6.0, 8.0)], sigma, [0.8, 0.6])
    vals = np.array([0, 1], dtype=np.uint32)
    ranges = np.array([[0, 2]])
    st = density.accumulate(pr, vals, ranges, [3], [4], [0.7], RasterParams())
    a0 = 0.8 * math.exp(-0.5 * 4 / sigma ** 2)
    a1 = 0.6 * math.exp(-0.5 * 25 / sigma ** 2)
    w = [a0, (1 - a0) * a1]
    dist = [2 / sigma, 5 / sigma]
    for i in range(2):
        assert abs(st[1, i] - w[i]) < 1e-15
        assert abs(st[0, i] - 0.7 * w[i]) < 1e-15
        assert abs(st[2, i] - dist[i] * w[i]) < 1e-15


def test_walk_stops_where_the_forward_stops():
    # alpha = 0.9 at the centre: T after k splats is 0.1^k; the fifth would
    # take T below T_min = 1e-4, so it and everything behind collect nothing
    pr = _proj([(5.0, 5.0)] * 7, 1.0, [0.9] * 7)
    vals = np.arange(7, dtype=np.uint32)
    st = density.accumulate(pr, vals, np.array([[0, 7]]), [5], [5], [1.0], RasterParams())
    want = [0.9 * 0.1 ** k for k in range(4)] + [0.0] * 3
    assert np.allclose(st[1], want, rtol=1e-12, atol=0)
    assert not st[2].any()          # every composited splat sits at the pixel itself: D = 0


def _scene_case(seed):
    p, cam = small_scene(n=2500, seed=seed)
    rp = RasterParams()
    pr = project.project(p, cam, rp)
    E = synth.error_map(cam.height, cam.width, 50 + seed)
    A = synth.age_map(cam.height, cam.width, 60 + seed)
    s = sampler.sample_view(E, A, SampleParams(n_pix=64), 3, 1, 0)
    _, sv, ranges = binning.bin_and_sort(pr, s["valid_tiles"])
    xs, ys, _ = sampler.sample_coords(s, cam.width, cam.height)
    err = np.random.default_rng(seed).uniform(0.0, 2.0, xs.size)
    return pr, sv, ranges, xs, ys, err, rp


def test_weights_telescope_to_one_minus_final_transmittance():
    """sum_k T_k alpha_k = 1 - T_final at every pixel, so summed over the
    Gaussians W and E equal the pixel sums of (1 - T) and e (1 - T) taken
    from the forward render."""
    pr, sv, ranges, xs, ys, err, rp = _scene_case(3)
    st = density.accumulate(pr, sv, ranges, xs, ys, err, rp)
    T = render.render_pixels(pr, sv, ranges, xs, ys, rp)["T"]
    assert abs(st[1].sum() - (1 - T).sum()) <= 1e-10 * (1 - T).sum()
    assert abs(st[0].sum() - (err * (1 - T)).sum()) <= 1e-10 * (err * (1 - T)).sum()
    assert (1 - T).sum() > 10.0     # the case composites a lot


def test_constant_error_and_distance_bound():
    pr, sv, ranges, xs, ys, _, rp = _scene_case(4)
    st = density.accumulate(pr, sv, ranges, xs, ys, np.full(xs.size, 0.25), rp)
    assert np.allclose(st[0], 0.25 * st[1], rtol=1e-13, atol=0)
    seen = st[1] > 0
    assert seen.sum() > 100
    sc = density.score(st, 0.5, 0.2)
    # composited means o exp(-D^2 / 2) >= alpha_min, so D <= sqrt(2 ln(1 / alpha_min))
    dmax = math.sqrt(2 * math.log(255.0))
    assert (sc["d"][seen] <= dmax * (1 + 1e-9)).all()
    assert np.allclose(sc["e"][seen], 0.25 * st[1][seen] / (st[1][seen] + density.EPS), rtol=1e-14)
    assert not sc["s"][~seen].any()


def test_score_is_a_weighted_mean_and_linear_in_lambda():
    pr, sv, ranges, xs, ys, err, rp = _scene_case(5)
    st = density.accumulate(pr, sv, ranges, xs, ys, err, rp)
    seen = st[1] > 1e-3
    sc = density.score(st, 0.0, 0.0)
    # e_i is a w-weighted mean of the pixel errors (up to eps)
    assert (sc["e"][seen] >= err.min() * (1 - 1e-6)).all() and (sc["e"][seen] <= err.max()).all()
    s1 = density.score(st, 2.0, 0.25)
    assert s1["lambda_eff"] == 1.5
    assert np.allclose(s1["s"], sc["e"] + 1.5 * sc["d"], rtol=1e-15, atol=0)
    # the sums are additive over views: two calls on halves equal one call on all
    h = xs.size // 2
    st2 = (density.accumulate(pr, sv, ranges, xs[:h], ys[:h], err[:h], rp)
           + density.accumulate(pr, sv, ranges, xs[h:], ys[h:], err[h:], rp))
    assert np.allclose(st2, st, rtol=1e-12, atol=1e-15)


def test_kth_largest_by_counting_and_library_extremes():
    rng = np.random.default_rng(12)
    v = np.concatenate([rng.exponential(1.0, 5000), np.full(300, 0.5), np.zeros(700)]).astype(np.float32)
    rng.shuffle(v)
    assert density.kth_largest(v, 1) == v.max()
    assert density.kth_largest(v, v.size) == v.min()
    for k in (1, 2, 17, 1000, 2500, 4700, 4999, 5000, 5001, 5299, 5300, 5301, 5999, 6000):
        t = density.kth_largest(v, k)
        assert (v > t).sum() < k <= (v >= t).sum(), k
        assert t in v


def test_select_masks_counts():
    rng = np.random.default_rng(13)
    s = rng.exponential(1.0, 1003)
    s[:200] = 0.0                                   # never composited
    m = density.select_masks(s, eta_topk=0.9, eta_final=0.75)
    k_d, k_k = density.percentile_count(1003, 0.1), density.percentile_count(1003, 0.75)
    assert (k_d, k_k) == (101, 753)
    assert m["densify"].sum() == 101 and m["keep"].sum() == 753     # no ties among the positive scores
    assert (s[m["densify"]].min() >= s[~m["densify"]].max())
    # keeping more than the 803 positive scores reaches the zeros, which all tie
    assert density.select_masks(s, 0.9, 0.85)["keep"].all()
    assert density.percentile_count(10, 0.3) == 3 and density.percentile_count(7, 0.0) == 1


def test_topology_split_clone_prune_closed_forms():
    n = 5
    P = np.zeros((59, n))
    P[0:3] = np.arange(15, dtype=np.float64).reshape(3, n)
    P[3:6] = np.log(2.0)                                   # scale 2 on every axis
    P[3:6, 1] = np.log(0.01)                               # Gaussian 1: small (clone)
    P[6] = 1.0                                             # identity rotation
    P[6:10, 3] = [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)]   # Gaussian 3: 90 degrees about z
    P[10] = np.arange(n)
    P[11:] = np.random.default_rng(1).normal(size=(48, n))
    m = np.full((59, n), 0.5)
    v = np.full((59, n), 0.25)
    keep = np.array([1, 1, 0, 1, 1], np.uint8)
    dens = np.array([1, 1, 1, 1, 0], np.uint8)             # Gaussian 2 is pruned, so not densified
    z = np.array([[1.0, -2.0, 0.5]] * n)
    r = density.apply_topology(P, m, v, keep, dens, z, log_split=np.log(0.1))
    assert (r["n_keep"], r["n_new"]) == (4, 3) and r["params"].shape == (59, 7)
    out = r["params"]
    # order: kept 0, 1, 3, 4, then new copies of 0, 1, 3
    assert np.array_equal(out[10], [0, 1, 3, 4, 0, 1, 3])
    assert np.array_equal(out[11:], P[11:][:, [0, 1, 3, 4, 0, 1, 3]])
    # Gaussian 0, identity rotation: o = S z = (2, -4, 1)
    assert np.allclose(out[0:3, 0], P[0:3, 0] + [2, -4, 1], atol=1e-14)
    assert np.allclose(out[0:3, 4], P[0:3, 0] - [2, -4, 1], atol=1e-14)
    assert np.allclose(out[3:6, [0, 4]], np.log(2.0 / 1.6), atol=1e-15)
    # Gaussian 3, 90 degrees about z maps x to y: o = (4, 2, 1)
    assert np.allclose(out[0:3, 2], P[0:3, 3] + [4, 2, 1], atol=1e-12)
    assert np.allclose((out[0:3, 2] + out[0:3, 6]) / 2, P[0:3, 3], atol=1e-12)   # centroid kept
    # Gaussian 1 is small: an exact clone that keeps its scale
    assert np.array_equal(out[:, 1], P[:, 1]) and np.array_equal(out[:, 5], P[:, 1])
    # Gaussian 4: kept, untouched
    assert np.array_equal(out[:, 3], P[:, 4])
    # moments: split slots and new ones restart at zero
    assert np.array_equal(r["m"][0], [0, 0.5, 0, 0.5, 0, 0, 0])
    assert np.array_equal(r["v"][5], [0, 0.25, 0, 0.25, 0, 0, 0])


def test_grad_screen_statistics():
    acc = np.zeros((4, 4))
    g = np.zeros((4, 9))
    g[:, 0:2] = [[3, 4], [-5, 12], [1, 1], [0, 0]]
    g[:, 2:] = 7.0                                    # other gradient fields do not enter
    # W = H = 2: NDC units equal pixel units
    acc = density.grad_screen_accumulate(acc, g, np.array([2, 9, 0, 4]), 2, 2)
    acc = density.grad_screen_accumulate(acc, g * 2, np.array([5, 0, 0, 1]), 2, 2)
    assert np.allclose(acc[:, 0], [5 + 10, 13, 0, 0])
    assert np.array_equal(acc[:, 1], [2, 1, 0, 2]) and np.array_equal(acc[:, 2], [5, 9, 0, 4])
    assert np.allclose(density.grad_screen_mean(acc), [7.5, 13, 0, 0])
    # NDC units: x scaled by W/2, y by H/2 (a 6 x 8 image: (3, 4) -> (9, 16))
    one = density.grad_screen_accumulate(np.zeros((1, 4)), g[:1], np.array([1]), 6, 8)
    assert one[0, 0] == math.hypot(9.0, 16.0)


def test_gradient_gate_and_selection_with_gate_and_prune_cadence():
    acc = np.array([[6.0, 2.0, 0, 0],      # mean 3
                    [1.0, 1.0, 0, 0],      # mean 1
                    [9.0, 0.0, 0, 0],      # never projected
                    [0.5, 1.0, 0, 0]])     # mean 0.5
    absum = np.array([0.0, 0.0, 100.0, 8.0])  # abs means 0, 0, -, 8
    gate = density.gradient_gate(acc, absum, tau_grad=2.0, tau_abs=5.0)
    assert gate.tolist() == [True, False, False, True]
    assert density.gradient_gate(acc, absum, 3.0, 8.0).tolist() == [True, False, False, True]
    assert density.gradient_gate(acc, absum, 3.001, 8.001).tolist() == [False] * 4
    s = np.array([4.0, 3.0, 2.0, 1.0])
    m = density.select_masks(s, eta_topk=0.5, eta_final=0.5, gate=gate)
    # top half densified by score (0 and 1), gated: only 0; keep the top half
    assert m["densify"].tolist() == [True, False, False, False]
    assert m["keep"].tolist() == [True, True, False, False]
    m2 = density.select_masks(s, eta_topk=0.5, eta_final=0.5, gate=gate, prune=False)
    assert m2["keep"].all() and m2["densify"].tolist() == [True, False, False, False]
    # a pruned Gaussian is never densified
    m3 = density.select_masks(s, eta_topk=1.0, eta_final=0.25, gate=np.ones(4, bool))
    assert m3["densify"].tolist() == [True, False, False, False]


def test_scene_extent_and_split_threshold():
    # cameras on a sphere of radius 3 around the origin, symmetric: extent 1.1 * 3
    c = 3.0 * np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=float)
    assert abs(density.scene_extent(c) - 3.3) < 1e-12
    assert abs(density.scene_extent(c + 5.0) - 3.3) < 1e-12        # translation does not change it
    assert abs(np.exp(density.split_log_threshold(0.01, 3.3)) - 0.033) < 1e-15


def test_absolute_centre_gradient_statistic():
    """The absolute statistic is the sum over pixels of each pixel's own
    centre-gradient norm: for one pixel it equals the norm of the summed
    gradient; for two pixels placed symmetrically about an isotropic splat the
    centre gradients cancel in the sum but not in the absolute statistic;
    in general it bounds the norm of the sum (triangle inequality)."""
    pr = _proj([(5.0, 5.0)], 2.0, [0.5])
    pr["rgb"] = np.array([[0.8], [0.3], [0.1]])
    vals = np.array([0], dtype=np.uint32)
    ranges = np.array([[0, 1]])
    rp = RasterParams()
    g1, a1 = render.render_pixels_bwd(pr, vals, ranges, [7], [5], np.array([[1.0, 0.5, -0.2]]), rp,
                                      centre_abs_scale=(3.0, 2.0))
    assert abs(a1[0] - math.hypot(3.0 * g1[0, 0], 2.0 * g1[1, 0])) < 1e-15 and a1[0] > 0
    g2, a2 = render.render_pixels_bwd(pr, vals, ranges, [7, 3], [5, 5], np.array([[1.0, 0.5, -0.2]] * 2), rp,
                                      centre_abs_scale=(3.0, 2.0))
    assert abs(g2[0, 0]) < 1e-15 and abs(g2[1, 0]) < 1e-15       # the two pulls cancel
    assert abs(a2[0] - 2.0 * a1[0]) < 1e-14                       # the absolute sums do not
    p, cam = small_scene(n=600, seed=4)
    prs = project.project(p, cam, rp)
    _, sv, rg = binning.bin_and_sort(prs)
    rng = np.random.default_rng(2)
    xs, ys = rng.integers(0, cam.width, 300), rng.integers(0, cam.height, 300)
    g, a = render.render_pixels_bwd(prs, sv, rg, xs, ys, rng.normal(size=(300, 3)), rp,
                                    centre_abs_scale=(cam.width / 2, cam.height / 2))
    norm = np.hypot(cam.width / 2 * g[0], cam.height / 2 * g[1])
    assert (a >= norm * (1 - 1e-12)).all() and (a > 0).sum() > 50
