"""Pins of the oracle's compositing and its adjoint: brute-force per-pixel
compositing over all Gaussians, weight partition of unity, closed forms,
finite differences in smooth mode."""
import math

import numpy as np
import pytest

import synth
from oracle import binning, project, project_bwd, render
from oracle.params import RasterParams


def _scene(n=120, seed=7, W=72, H=56, logscale=-2.6):
    p = synth.gaussians(n, seed, logscale_mean=logscale)
    cam = synth.look_at((2.2, 1.4, 1.0), fx=W * 1.0, fy=W * 1.0, width=W, height=H)
    return p, cam


def _brute_pixel(pr, x, y, rp):
    """Eq. (alpha_comp) for one pixel by a plain loop: every visible Gaussian
    whose tile rectangle holds the pixel's tile, sorted by (FP32 depth, id)."""
    rp = rp.f64()
    tx, ty = x // 16, y // 16
    members = [g for g in range(pr["opacity"].size) if pr["visible"][g]
               and pr["rect"][0, g] <= tx < pr["rect"][2, g] and pr["rect"][1, g] <= ty < pr["rect"][3, g]]
    members.sort(key=lambda g: (float(pr["depth32"][g]), g))
    T, C, ncon, nblend = 1.0, np.zeros(3), 0, 0
    for pos, g in enumerate(members):
        dx = x - pr["mean2d"][0, g]
        dy = y - pr["mean2d"][1, g]
        a, b, c = pr["conic"][:, g]
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        if power > 0:
            continue
        alpha = min(rp.alpha_max, pr["opacity"][g] * math.exp(power))
        if alpha < rp.alpha_min:
            continue
        test = T * (1 - alpha)
        if test < rp.T_min:
            break
        C += T * alpha * pr["rgb"][:, g]
        T = test
        ncon = pos + 1
        nblend += 1
    return C + T * np.asarray(rp.bg), T, ncon, nblend


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.2, 0.5, 1.0)])
def test_tiled_render_equals_brute_force(bg):
    p, cam = _scene()
    rp = RasterParams(bg=bg)
    pr = project.project(p, cam, rp)
    _, sv, ranges = binning.bin_and_sort(pr)
    rng = np.random.default_rng(0)
    xs = rng.integers(0, cam.width, 150)
    ys = rng.integers(0, cam.height, 150)
    out = render.render_pixels(pr, sv, ranges, xs, ys, rp)
    for i in range(xs.size):
        C, T, ncon, nb = _brute_pixel(pr, int(xs[i]), int(ys[i]), rp)
        assert np.allclose(out["rgb"][i], C, rtol=1e-13, atol=1e-15)
        assert abs(out["T"][i] - T) <= 1e-14
        assert out["n_contrib"][i] == ncon and out["n_blend"][i] == nb


def test_weights_plus_transmittance_is_one_and_sparse_equals_dense():
    p, cam = _scene(seed=8)
    rp = RasterParams()
    pr = project.project(p, cam, rp)
    pr1 = dict(pr)
    pr1["rgb"] = np.ones_like(pr["rgb"])           # white splats: C = sum of weights
    _, sv, ranges = binning.bin_and_sort(pr)
    xs, ys = render.dense_pixels(cam.width, cam.height)
    dense = render.render_pixels(pr1, sv, ranges, xs, ys, rp)
    assert np.allclose(dense["rgb"][:, 0] + dense["T"], 1.0, atol=1e-12)
    sel = np.random.default_rng(1).choice(xs.size, 500, replace=False)
    sparse = render.render_pixels(pr1, sv, ranges, xs[sel], ys[sel], rp)
    for k in ("rgb", "T", "n_contrib", "n_eval", "n_blend"):
        assert np.array_equal(sparse[k], dense[k][sel])


def test_single_gaussian_closed_form():
    cam = synth.Camera(R=np.eye(3), t=np.zeros(3), fx=100.0, fy=100.0, cx=24.0, cy=16.0, width=48, height=32)
    p = np.zeros((59, 1), dtype=np.float32)
    p[0:3, 0] = [0.05, -0.02, 2.0]
    p[3:6, 0] = [-2.5, -3.0, -2.8]
    p[6:10, 0] = [0.9, 0.1, -0.2, 0.3]
    p[10, 0] = 0.4
    p[11:14, 0] = [0.3, -0.1, 0.2]
    rp = RasterParams(sh_degree=0)
    pr = project.project(p, cam, rp)
    _, sv, ranges = binning.bin_and_sort(pr)
    xs, ys = render.dense_pixels(cam.width, cam.height)
    out = render.render_pixels(pr, sv, ranges, xs, ys, rp)
    dx = xs - pr["mean2d"][0, 0]
    dy = ys - pr["mean2d"][1, 0]
    a, b, c = pr["conic"][:, 0]
    alpha = np.minimum(0.99, pr["opacity"][0] * np.exp(-0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy))
    tx, ty = xs // 16, ys // 16
    inside = (pr["rect"][0, 0] <= tx) & (tx < pr["rect"][2, 0]) & (pr["rect"][1, 0] <= ty) & (ty < pr["rect"][3, 0])
    alpha = np.where(inside & (alpha >= float(np.float32(1 / 255))), alpha, 0.0)
    assert np.allclose(out["rgb"], alpha[:, None] * pr["rgb"][:, 0][None, :], atol=1e-15)


def test_zero_opacity_gaussians_change_nothing():
    p, cam = _scene(seed=9)
    rp = RasterParams()
    q = np.concatenate([p, synth.gaussians(40, 99, logscale_mean=-2.6)], axis=1)
    q[10, p.shape[1]:] = -200.0                      # opacity 0 (sigmoid of -200)
    pr_a = project.project(p, cam, rp)
    pr_b = project.project(q, cam, rp)
    xs, ys = render.dense_pixels(cam.width, cam.height)
    _, sva, ra = binning.bin_and_sort(pr_a)
    _, svb, rb = binning.bin_and_sort(pr_b)
    oa = render.render_pixels(pr_a, sva, ra, xs, ys, rp)
    ob = render.render_pixels(pr_b, svb, rb, xs, ys, rp)
    assert np.array_equal(oa["rgb"], ob["rgb"]) and np.array_equal(oa["T"], ob["T"])
    g = np.random.default_rng(2).normal(size=(xs.size, 3))
    g2d = render.render_pixels_bwd(pr_b, svb, rb, xs, ys, g, rp)
    assert (g2d[:, p.shape[1]:] == 0).all()
    grad = project_bwd.project_bwd(q, cam, pr_b, g2d, rp)
    assert (grad[:, p.shape[1]:] == 0).all()


# ---------------------------------------------------------------- finite differences
SMOOTH = RasterParams(alpha_min=0.0, alpha_max=1.0, T_min=0.0, clamp_color=False, bg=(0.1, 0.2, 0.3))


def _render_from_splats(pr, sv, ranges, xs, ys, rp):
    return render.render_pixels(pr, sv, ranges, xs, ys, rp)["rgb"]


def test_render_adjoint_matches_finite_differences_smooth_mode():
    p, cam = _scene(n=40, seed=10, W=48, H=40)
    pr = project.project(p, cam, SMOOTH)
    _, sv, ranges = binning.bin_and_sort(pr)
    xs, ys = render.dense_pixels(cam.width, cam.height)
    wgt = np.random.default_rng(3).normal(size=(xs.size, 3))
    g2d = render.render_pixels_bwd(pr, sv, ranges, xs, ys, wgt, SMOOTH)
    fields = [("mean2d", 0), ("mean2d", 1), ("conic", 0), ("conic", 1), ("conic", 2),
              ("opacity", None), ("rgb", 0), ("rgb", 1), ("rgb", 2)]
    vis = np.nonzero(pr["visible"])[0]
    rng = np.random.default_rng(4)
    for row, (name, comp) in enumerate(fields):
        u = np.zeros(pr["opacity"].size)
        u[vis] = rng.normal(size=vis.size)
        h = 1e-6 if name != "conic" else 1e-8
        vals = []
        for sgn in (1, -1):
            q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in pr.items()}
            if comp is None:
                q[name] = q[name] + sgn * h * u
            else:
                q[name][comp] = q[name][comp] + sgn * h * u
            vals.append((wgt * _render_from_splats(q, sv, ranges, xs, ys, SMOOTH)).sum())
        fd = (vals[0] - vals[1]) / (2 * h)
        an = (g2d[row] * u).sum()
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, comp, fd, an)


def test_full_chain_matches_finite_differences_smooth_mode():
    p, cam = _scene(n=30, seed=11, W=40, H=40, logscale=-2.3)
    p = p.astype(np.float64)
    xs, ys = render.dense_pixels(cam.width, cam.height)
    wgt = np.random.default_rng(5).normal(size=(xs.size, 3))

    def value(params):
        pr = project.project(params, cam, SMOOTH)
        _, sv, ranges = binning.bin_and_sort(pr)
        return (wgt * render.render_pixels(pr, sv, ranges, xs, ys, SMOOTH)["rgb"]).sum(), pr["rect"]

    pr = project.project(p, cam, SMOOTH)
    _, sv, ranges = binning.bin_and_sort(pr)
    g2d = render.render_pixels_bwd(pr, sv, ranges, xs, ys, wgt, SMOOTH)
    grad = project_bwd.project_bwd(p, cam, pr, g2d, SMOOTH)
    groups = {"mean": range(0, 3), "logscale": range(3, 6), "quat": range(6, 10),
              "opacity": [10], "sh_dc": range(11, 14), "sh_rest": range(14, 59)}
    rng = np.random.default_rng(6)
    for name, rows in groups.items():
        u = np.zeros_like(p)
        u[list(rows)] = rng.normal(size=(len(rows), p.shape[1]))
        h = 1e-6
        vp, rect_p = value(p + h * u)
        vm, rect_m = value(p - h * u)
        assert np.array_equal(rect_p, pr["rect"]) and np.array_equal(rect_m, pr["rect"])
        fd = (vp - vm) / (2 * h)
        an = (grad * u).sum()
        assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (name, fd, an)


def test_dropping_non_compositing_pairs_leaves_images_and_gradients_unchanged():
    """A list without the pairs that stay below alpha_min at every pixel
    centre of their tile (max_alpha_in_tile) renders the same colour,
    transmittance and blend counts, and has the same adjoint, as the
    rectangle list: the argument that lets a GPU list be any order-preserving
    subsequence that keeps every pair able to composite."""
    for seed, ls in ((21, -2.6), (22, -2.2)):
        p, cam = _scene(n=150, seed=seed, logscale=ls)
        rp = RasterParams()
        pr = project.project(p, cam, rp)
        TX, TY = pr["TX"], pr["TY"]
        sk0, sv0, rg0 = binning.bin_and_sort(pr)
        tiles = (sk0 >> np.uint64(32)).astype(np.int64)
        keep = binning.max_alpha_in_tile(pr, sv0, tiles) >= rp.f64().alpha_min
        assert 0.1 < 1 - keep.mean() < 0.9
        sk1, sv1 = sk0[keep], sv0[keep]
        rg1 = binning.tile_ranges(sk1, TX * TY)
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        xs, ys = xs.ravel(), ys.ravel()
        a = render.render_pixels(pr, sv0, rg0, xs, ys, rp)
        b = render.render_pixels(pr, sv1, rg1, xs, ys, rp)
        assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["T"], b["T"])
        assert np.array_equal(a["n_blend"], b["n_blend"]) and np.array_equal(a["composited"], b["composited"])
        assert (b["n_eval"] <= a["n_eval"]).all() and b["n_eval"].sum() < a["n_eval"].sum()
        dL = np.random.default_rng(seed).normal(size=(xs.size, 3))
        ga = render.render_pixels_bwd(pr, sv0, rg0, xs, ys, dL, rp)
        gb = render.render_pixels_bwd(pr, sv1, rg1, xs, ys, dL, rp)
        # equal up to the summation order numpy picks for the longer lists
        assert np.allclose(ga, gb, rtol=1e-12, atol=1e-14 * np.abs(ga).max())


# ---------------------------------------------------------------- threshold branches
def _splats(centres, conics, opacities, colours, TX=1, TY=1):
    """A projection record built by hand: splats at the given tile-space
    centres, all listed in tile 0 in the given order."""
    n = len(opacities)
    pr = dict(mean2d=np.array(centres, dtype=np.float64).T.copy(),
              conic=np.array(conics, dtype=np.float64).T.copy(),
              opacity=np.array(opacities, dtype=np.float64),
              rgb=np.array(colours, dtype=np.float64).T.copy(), TX=TX, TY=TY)
    sv = np.arange(n, dtype=np.uint32)
    ranges = np.zeros((TX * TY, 2), dtype=np.int64)
    ranges[0] = (0, n)
    return pr, sv, ranges


def test_alpha_max_clamp_zeroes_opacity_and_geometry_gradient():
    """One Gaussian whose o G exceeds alpha_max at a pixel composites exactly
    alpha_max there: the colour is alpha_max c + (1 - alpha_max) bg, its
    gradient wrt the colour is alpha_max dL, and the opacity, centre and
    conic gradients of that pixel are exactly zero (the clamp is flat).  At
    a pixel where o G is below alpha_max the same Gaussian gets the
    unclamped derivatives, which finite differences confirm."""
    rp = RasterParams(bg=(0.1, 0.2, 0.3))
    amax = rp.f64().alpha_max
    pr, sv, rg = _splats([(7.3, 8.1)], [(0.02, 0.004, 0.03)], [0.999], [(0.6, 0.3, 0.9)])
    xs, ys = np.array([7, 15]), np.array([8, 1])
    ev = render.render_pixels(pr, sv, rg, xs, ys, rp)
    G = np.exp(-0.5 * (0.02 * 0.3 ** 2 + 0.03 * 0.1 ** 2) - 0.004 * (-0.3) * (-0.1))
    assert 0.999 * G > amax                                      # the clamped pixel
    bg = np.asarray(rp.f64().bg)
    assert np.allclose(ev["rgb"][0], amax * pr["rgb"][:, 0] + (1 - amax) * bg, rtol=0, atol=1e-15)
    dL = np.array([[0.7, -1.1, 0.4], [0.0, 0.0, 0.0]])
    g = render.render_pixels_bwd(pr, sv, rg, xs, ys, dL, rp)
    assert (g[0:6, 0] == 0).all()
    assert np.allclose(g[6:9, 0], amax * dL[0], rtol=1e-15, atol=0)
    # the unclamped pixel: non-zero derivatives that match finite differences
    dL2 = np.array([[0.0, 0.0, 0.0], [0.7, -1.1, 0.4]])
    g2 = render.render_pixels_bwd(pr, sv, rg, xs, ys, dL2, rp)
    assert (g2[0:6, 0] != 0).all()
    for name, comp, row in (("mean2d", 0, 0), ("conic", 1, 3), ("opacity", None, 5)):
        h = 1e-7
        vals = []
        for sgn in (1, -1):
            q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in pr.items()}
            if comp is None:
                q[name] = q[name] + sgn * h
            else:
                q[name][comp] += sgn * h
            vals.append((dL2 * render.render_pixels(q, sv, rg, xs, ys, rp)["rgb"]).sum())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g2[row, 0]) <= 1e-6 * abs(fd), (name, fd, g2[row, 0])


def test_transmittance_stop_fixed_position_matches_finite_differences():
    """Four broad Gaussians stacked on one pixel, each with alpha near 0.95:
    T after them is 0.05, 2.5e-3, 1.25e-4, 6.25e-6, so the walk stops before
    the fourth (T would fall below T_min = 1e-4) with a wide margin on both
    sides.  The fourth Gaussian gets exactly zero gradient; the three in
    front match finite differences of the rendered colour in every splat
    field, and the colour is the closed form over the first three."""
    rp = RasterParams(bg=(0.25, 0.5, 0.75))
    c = 2.0e-3
    cols = [(0.9, 0.1, 0.2), (0.3, 0.8, 0.4), (0.5, 0.5, 0.9), (0.1, 0.9, 0.6)]
    pr, sv, rg = _splats([(6.2, 7.4), (5.1, 9.3), (8.8, 6.6), (7.0, 7.0)],
                         [(c, 0.0002, c * 1.3), (c * 0.8, -0.0003, c), (c * 1.1, 0.0001, c * 0.9), (c, 0.0, c)],
                         [0.955, 0.952, 0.957, 0.95], cols)
    xs, ys = np.array([7]), np.array([7])
    out = render.render_pixels(pr, sv, rg, xs, ys, rp)
    assert out["n_contrib"][0] == 3 and out["n_blend"][0] == 3 and out["n_eval"][0] == 4
    # closed form over the first three
    d = np.array([7.0, 7.0])[:, None] - pr["mean2d"]
    a_, b_, c_ = pr["conic"]
    alpha = pr["opacity"] * np.exp(-0.5 * (a_ * d[0] ** 2 + c_ * d[1] ** 2) - b_ * d[0] * d[1])
    T = np.concatenate([[1.0], np.cumprod(1 - alpha)])
    assert T[3] > 1.2 * rp.T_min and T[4] < 0.2 * rp.T_min
    want = (T[:3, None] * alpha[:3, None] * pr["rgb"][:, :3].T).sum(0) + T[3] * np.asarray(rp.f64().bg)
    assert np.allclose(out["rgb"][0], want, rtol=1e-14, atol=0)
    dL = np.array([[0.6, -0.9, 1.3]])
    g = render.render_pixels_bwd(pr, sv, rg, xs, ys, dL, rp)
    assert (g[:, 3] == 0).all() and (g[:, :3] != 0).all()
    fields = [("mean2d", 0), ("mean2d", 1), ("conic", 0), ("conic", 1), ("conic", 2),
              ("opacity", None), ("rgb", 0), ("rgb", 1), ("rgb", 2)]
    for row, (name, comp) in enumerate(fields):
        for k in range(3):
            h = 1e-6
            vals = []
            for sgn in (1, -1):
                q = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in pr.items()}
                if comp is None:
                    q[name][k] += sgn * h
                else:
                    q[name][comp, k] += sgn * h
                r = render.render_pixels(q, sv, rg, xs, ys, rp)
                assert r["n_contrib"][0] == 3
                vals.append((dL * r["rgb"]).sum())
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g[row, k]) <= 1e-6 * max(abs(fd), 1e-2), (name, comp, k, fd, g[row, k])


def _fp32_band_ratios(pr, tiles, n_loc, seed, TX):
    """Worst ratios of an FP32 evaluation's alpha and transmittance errors to
    eps_a and eps_T over sampled pixels of ``tiles``, and the flag count.
    The FP32 side: the splat record rounded to FP32 (conic in its LDL^T form
    a, beta, delta), the tile-local centre as the exact integer difference
    plus the fraction, w = fma(beta, dy, dx), p2 = fma(A, w^2, D dy^2) with
    A, D the conic values times -log2(e)/2, each operation rounded once, and
    a rounded exponential."""
    from support import splat_record
    f32 = np.float32
    l2e = f32(1.4426950408889634)
    rp = RasterParams()
    r64 = rp.f64()
    rec = splat_record(pr)
    _, sv, rg = binning.bin_and_sort(pr, tiles)
    rng = np.random.default_rng(seed)
    worst_a = worst_T = amp = 0.0
    flagged = total = 0
    for t in tiles:
        lo, hi = rg[t]
        gids = sv[lo:hi].astype(np.int64)
        if gids.size == 0:
            continue
        loc = rng.choice(256, n_loc, replace=False)
        xs = (t % TX) * 16 + loc % 16
        ys = (t // TX) * 16 + loc // 16
        ev = render._tile_eval(pr, gids, xs.astype(float), ys.astype(float), r64)
        r = rec[gids]
        x0, y0 = f32((t % TX) * 16), f32((t // TX) * 16)
        gx = (r[:, 0] - x0) + r[:, 2]
        gy = (r[:, 1] - y0) + r[:, 3]
        A = r[:, 4] * f32(-0.5 * l2e)
        D = r[:, 6] * f32(-0.5 * l2e)
        dx = (loc % 16).astype(f32)[:, None] - gx[None]
        dy = (loc // 16).astype(f32)[:, None] - gy[None]
        w = (r[None, :, 5].astype(np.float64) * dy + dx).astype(f32)     # fma: one rounding
        p2 = (A[None].astype(np.float64) * (w * w) + D[None] * (dy * dy)).astype(f32)
        a32 = r[None, :, 7] * np.exp2(p2.astype(np.float64)).astype(f32)
        neval = np.where(ev["has_stop"], ev["stop_at"] + 1, gids.size)
        m = (np.arange(gids.size)[None] < neval[:, None]) & (ev["araw"] > 1e-30)
        rel = np.abs(a32 - ev["araw"]) / np.where(m, ev["araw"], 1.0)
        if m.any():
            worst_a = max(worst_a, float((rel / ev["eps_a"])[m].max()))
            # size of the terms a dx^2 / 2, b dx dy, c dy^2 / 2 against the exponent
            terms = (0.5 * np.abs(ev["a"])[None] * ev["dx"] ** 2 + 0.5 * np.abs(ev["c"])[None] * ev["dy"] ** 2
                     + np.abs(ev["b"][None] * ev["dx"] * ev["dy"]))
            amp = max(amp, float((terms / np.maximum(np.abs(ev["power"]), 0.5))[m & ev["ok"]].max(initial=0.0)))
        al = np.minimum(f32(r64.alpha_max), a32)
        T = np.ones(xs.size, f32)
        for k in range(gids.size):
            Tn = T * (f32(1) - al[:, k])
            mk = ev["contrib"][:, k] | (ev["ok"][:, k] & (ev["stop_at"] == k))
            if mk.any():
                relT = np.abs(Tn - ev["T_after"][:, k])[mk] / ev["T_after"][mk, k]
                worst_T = max(worst_T, float((relT / ev["eps_T"][mk, k]).max()))
            T = np.where(ev["contrib"][:, k], Tn, T)
        out = render.render_pixels(pr, sv, rg, xs, ys, rp)
        flagged += int(out["flag"].sum())
        total += xs.size
    return worst_a, worst_T, flagged, total, amp


def test_guard_band_bounds_an_fp32_evaluation():
    """The guard band is wide enough and not too wide: the FP32 evaluation's
    alpha and running transmittance stay within the oracle's error bounds
    eps_a and eps_T (half the band at the default guard of two) at every
    evaluated position of two tiny-workload views' sampled tiles, and the
    largest ratio is above 1/20 (the bound is not vacuous); few pixels are
    flagged."""
    rp = RasterParams()
    p = synth.gaussians(10000, synth.SEED_SCENE)
    cams = synth.tetra_cameras()
    worst_a = worst_T = 0.0
    flagged = total = 0
    for vi in (0, 3):
        pr = project.project(p, cams[vi], rp)
        tiles = np.random.default_rng(vi).choice(256, 24, replace=False)
        wa, wt, f, n, _ = _fp32_band_ratios(pr, tiles, 48, 10 + vi, 16)
        worst_a, worst_T = max(worst_a, wa), max(worst_T, wt)
        flagged, total = flagged + f, total + n
    assert 0.05 < worst_a < 0.8 and worst_T < 0.8, (worst_a, worst_T)
    assert flagged <= 1e-3 * total, (flagged, total)


def test_guard_band_bounds_an_fp32_evaluation_of_needle_splats():
    """The same on a near-camera corridor view (1920x1080) where one Gaussian
    in fifty is a needle (scales 150:1): two units from the camera these
    project to splats hundreds of pixels long, where
    the exponent's terms a dx^2, 2 b dx dy, c dy^2 reach a thousand times
    the exponent itself at composited positions; the LDL^T evaluation keeps the band narrow (no
    pixel flagged more often than on the tiny workload)."""
    rp = RasterParams()
    p = synth.corridor_gaussians(150_000, 11, length=6.0)
    p[3:6, ::50] = np.array([-1.5, -6.5, -6.5], dtype=np.float32)[:, None]   # 2%: one long axis (150:1)
    cam = synth.trajectory_cameras(4, length=6.0)[1]
    pr = project.project(p, cam, rp)
    TX, TY = pr["TX"], pr["TY"]
    tiles = np.sort(np.random.default_rng(6).choice(TX * TY, 40, replace=False))
    worst_a, worst_T, flagged, total, amp = _fp32_band_ratios(pr, tiles, 32, 12, TX)
    assert total > 1000
    assert amp > 1000, amp          # the view does hold such needles
    assert 0.05 < worst_a < 0.8 and worst_T < 0.8, (worst_a, worst_T)
    assert flagged <= 3e-3 * total, (flagged, total)
