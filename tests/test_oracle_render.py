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
