"""Degenerate inputs through the C-ABI: no Gaussians at all, every Gaussian
behind the camera (no pairs), a single Gaussian, and one Gaussian whose
footprint covers every tile of the image on top of a small scene.

What fixes the expected values: the oracle for the single and covering
cases; for the empty cases the definition of front-to-back compositing
(an empty list leaves T = 1 and the pixel shows the background, Sec. 3.1)
and of the sparse optimizer (a Gaussian that no pair references keeps its
parameters and moments)."""
import numpy as np
import pytest
import torch

import synth
from oracle import binning, project, render, sampler
from oracle.params import RasterParams, SampleParams

from support import moments_gaussian_major, moments_rows, assert_close, check_pair_lists, small_scene, splat_as_oracle, splat_record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15924_amd import binding
    binding.lib()
    return binding


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _project(B, p, cam, brp):
    n = p.shape[1]
    k = max(n, 1)
    out = dict(splat=torch.zeros((k, 12), dtype=torch.float32, device="cuda"),
               depth=torch.zeros(k, dtype=torch.float32, device="cuda"),
               radius=torch.zeros(k, dtype=torch.int32, device="cuda"),
               rect=torch.zeros((k, 4), dtype=torch.int32, device="cuda"),
               clamp=torch.zeros(k, dtype=torch.uint8, device="cuda"))
    B.tgs_project(dev(p) if n else torch.zeros(1, device="cuda"), n, B.camera(cam), brp, out["splat"],
                  out["depth"], out["radius"], out["rect"], out["clamp"])
    return out


def _bin(B, pj, n, TX, TY, tile_slot=None, cap=1 << 16):
    K = torch.empty(cap, dtype=torch.int64, device="cuda")
    V = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    R = torch.full((TX * TY, 2), -5, dtype=torch.int32, device="cuda")
    # entries of Gaussians without a pair are left as they are: 2 marks them
    touched = torch.full((max(n, 1),), 2, dtype=torch.uint8, device="cuda")
    ws = torch.empty(B.tgs_bin_sort_workspace_size(n, cap, TX * TY), dtype=torch.uint8, device="cuda")
    npairs = B.tgs_bin_sort(pj["rect"], pj["splat"], pj["depth"], n, tile_slot, TX, TY, 1.0 / 255.0, K, V, cap, R,
                            touched if n else None, ws)
    return npairs, K, V, R, touched


def _state(B, n_slots, max_per_tile):
    """The forward's state record, as the training step passes it (the
    backward then runs split into (tile, chunk) workgroups)."""
    return torch.empty(B.tgs_render_state_size(n_slots, max_per_tile) // 4 + 4, dtype=torch.float32, device="cuda")


def _render_dense(B, splat, V, R, cam, brp, dl=None):
    TX, TY = (cam.width + 15) // 16, (cam.height + 15) // 16
    P = cam.width * cam.height
    out = torch.full((P, 4), -1.0, dtype=torch.float32, device="cuda")
    nc = torch.full((P,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros((2, B.COUNTER_SLOTS), dtype=torch.int64, device="cuda")
    st = _state(B, TX * TY, 256)
    B.tgs_render_fwd(splat, V, R, TX, TY, cam.width, cam.height, None, None, None, TX * TY, 256, brp, out, nc, cnt,
                     st)
    G = None
    if dl is not None:
        G = torch.zeros((splat.shape[0], 9), dtype=torch.float32, device="cuda")
        B.tgs_render_bwd(splat, V, R, TX, TY, cam.width, cam.height, None, None, None, TX * TY, 256, brp, out, nc,
                         dev(dl), G, st)
    return out, nc, cnt, G


def _behind_camera(n, seed, cam_eye):
    """Gaussians placed behind a camera at cam_eye looking at the origin."""
    p = synth.gaussians(n, seed, logscale_mean=-3.3)
    eye = np.asarray(cam_eye, dtype=np.float32)
    p[0:3] = eye[:, None] * 1.5 + p[0:3] * 0.2
    return p


def test_empty_scene(B):
    """n = 0: no pairs, every range empty, every pixel the background with
    T = 1 and no contributors; the backward writes nothing."""
    _, cam = small_scene(n=1)
    bg = (0.25, 0.5, 0.75)
    brp = B.raster_params(bg=bg)
    TX, TY = (cam.width + 15) // 16, (cam.height + 15) // 16
    pj = _project(B, np.zeros((59, 0), dtype=np.float32), cam, brp)
    npairs, K, V, R, _ = _bin(B, pj, 0, TX, TY)
    assert npairs == 0
    assert (host(R) == 0).all()
    out, nc, cnt, G = _render_dense(B, pj["splat"], V, R, cam, brp,
                                    dl=np.ones((cam.width * cam.height, 4), np.float32))
    o = host(out)
    assert np.array_equal(o[:, :3], np.tile(np.float32(bg), (o.shape[0], 1)))
    assert (o[:, 3] == 1.0).all() and (host(nc) == 0).all()
    assert (host(cnt) == 0).all()
    assert (host(G) == 0).all()


def test_all_gaussians_behind_camera(B):
    """Every Gaussian culled at projection: radius 0, no pairs, nothing
    touched, background everywhere, zero screen-space gradient, and the
    fused backward + optimizer leaves parameters and moments unchanged."""
    _, cam = small_scene(n=1)
    eye = np.asarray(project.camera_center(cam))
    p = _behind_camera(500, 3, eye)
    rp = RasterParams(bg=(0.1, 0.2, 0.3))
    pr = project.project(p, cam, rp)
    assert not pr["visible"].any()
    brp = B.raster_params(bg=rp.bg)
    n = p.shape[1]
    TX, TY = pr["TX"], pr["TY"]
    pj = _project(B, p, cam, brp)
    assert (host(pj["radius"]) == 0).all()
    assert np.array_equal(host(pj["depth"]).view(np.uint32), pr["depth32"].view(np.uint32))
    npairs, K, V, R, touched = _bin(B, pj, n, TX, TY)
    assert npairs == 0
    assert (host(R) == 0).all()
    assert (host(touched) == 2).all()
    touched.zero_()
    xs, ys = render.dense_pixels(cam.width, cam.height)
    ref = render.render_pixels(pr, np.zeros(0, np.uint32), np.zeros((TX * TY, 2), np.int64), xs, ys, rp)
    dl = np.random.default_rng(2).normal(size=(xs.size, 4)).astype(np.float32)
    out, nc, _, G = _render_dense(B, pj["splat"], V, R, cam, brp, dl=dl)
    o = host(out)
    assert np.array_equal(o[:, :3], ref["rgb"].astype(np.float32))
    assert (o[:, 3] == 1.0).all() and (host(nc) == 0).all()
    assert (host(G) == 0).all()
    m0 = np.full((59, n), 1e-3, np.float32)
    v0 = np.full((59, n), 1e-5, np.float32)
    P, M, Vv = dev(p), dev(moments_gaussian_major(m0)), dev(moments_gaussian_major(v0))
    B.tgs_project_bwd_optimizer_step(P, n, B.camera(cam), brp, pj["radius"], pj["clamp"], G, None, M, Vv,
                                     touched, B.optim_params(lm_mode=0), 3,
                                     torch.empty(B.tgs_project_bwd_optimizer_workspace_size(n),
                                                 dtype=torch.uint8, device="cuda"))
    assert np.array_equal(host(P), p) and np.array_equal(moments_rows(host(M)), m0)
    assert np.array_equal(moments_rows(host(Vv)), v0)


def _full_chain_parity(B, p, cam, rp, sample=None):
    """Projection, binning, forward and backward of one view against the
    oracle, at the bars of the per-stage tests."""
    pr = project.project(p, cam, rp)
    brp = B.raster_params(bg=rp.bg)
    n = p.shape[1]
    TX, TY = pr["TX"], pr["TY"]
    pj = _project(B, p, cam, brp)
    vis = pr["visible"]
    safe = vis & (pr["radius_margin"] > 1e-9)      # radius not on a rounding boundary
    assert safe.sum() >= vis.sum() - 2
    assert np.array_equal(host(pj["radius"])[safe], pr["radius"][safe])
    valid = None if sample is None else sample["valid_tiles"]
    tile_slot = None
    if valid is not None:
        ts = -np.ones(TX * TY, dtype=np.int32)
        ts[valid] = np.arange(valid.size)
        tile_slot = dev(ts)
    rec = splat_record(pr)
    assert np.array_equal(host(pj["splat"])[vis][:, :2], rec[vis][:, :2])
    # binning and rendering take the oracle's record (FP32) as input, as the
    # per-stage tests do: a last-bit difference in a conic must not move a
    # culling decision
    sk, sv, ranges = binning.bin_and_sort(pr, valid)
    q = splat_as_oracle(pr, rec)
    ob = dict(rect=dev(pr["rect"].T.astype(np.int32)), splat=dev(rec), depth=dev(pr["depth32"]))
    npairs, K, V, R, touched = _bin(B, ob, n, TX, TY, tile_slot)
    gv = host(V)[:npairs].view(np.uint32)
    check_pair_lists(gv, host(R), npairs, q, valid, keys=host(K))
    t_ref = np.full(n, 2, dtype=np.uint8)
    t_ref[np.unique(gv)] = 1
    assert np.array_equal(host(touched)[:n], t_ref)
    if sample is None:
        xs, ys = render.dense_pixels(cam.width, cam.height)
    else:
        xs, ys, _ = sampler.sample_coords(sample, cam.width, cam.height)
    ref = render.render_pixels(q, sv, ranges, xs, ys, rp)
    g = np.random.default_rng(5).normal(size=(xs.size, 3)) * 1e-3
    g[ref["flag"]] = 0.0
    g2d, g2d_abs = render.render_pixels_bwd(q, sv, ranges, xs, ys, g, rp, with_abs=True)
    splat = dev(rec)
    V = dev(sv.view(np.int32)) if sv.size else torch.zeros(1, dtype=torch.int32, device="cuda")
    R = dev(ranges.astype(np.int32))
    if sample is None:
        dl = np.zeros((cam.width * cam.height, 4), np.float32)
        dl[ys * cam.width + xs, :3] = g
        out, nc, _, G = _render_dense(B, splat, V, R, cam, brp, dl=dl)
        o, c = host(out)[ys * cam.width + xs], host(nc)[ys * cam.width + xs]
    else:
        P = xs.size
        n_pix = max(int(np.diff(sample["tile_off"]).max()), 1)
        vt, off, pix = dev(sample["valid_tiles"]), dev(sample["tile_off"]), dev(sample["pix"])
        n_st = sample["valid_tiles"].size
        out = torch.empty((P, 4), dtype=torch.float32, device="cuda")
        nc = torch.empty(P, dtype=torch.int32, device="cuda")
        st = _state(B, n_st, n_pix)
        B.tgs_render_fwd(splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, n_pix, brp, out, nc,
                         None, st)
        dl = np.zeros((P, 4), np.float32)
        dl[:, :3] = g
        G = torch.zeros((n, 9), dtype=torch.float32, device="cuda")
        B.tgs_render_bwd(splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, n_pix, brp, out, nc,
                         dev(dl), G, st)
        o, c = host(out), host(nc)
    ok = ~ref["flag"]
    assert ok.mean() > 0.99, ok.mean()
    assert_close(o[ok, :3], ref["rgb"][ok], 1e-5, 1e-7, "rgb")
    assert_close(o[ok, 3], ref["T"][ok], 1e-5, 1e-7, "T")
    assert np.array_equal(c[ok], ref["n_contrib"][ok])
    got = host(G).T
    for f in range(9):
        assert_close(got[f], g2d[f], 1e-4, 2e-6 * g2d_abs[f] + 1e-12, f"g2d[{f}]")
    return pr, sv


def test_single_gaussian(B):
    """One Gaussian in front of the camera: the whole chain against the
    oracle, dense and on a sampled view."""
    p = synth.gaussians(1, 17, logscale_mean=-2.0)
    p[0:3, 0] = (0.05, -0.02, 0.03)
    p[10, 0] = 2.0
    _, cam = small_scene(n=1)
    rp = RasterParams(bg=(0.3, 0.3, 0.3))
    pr, sv = _full_chain_parity(B, p, cam, rp)
    assert pr["visible"][0] and sv.size > 1
    E = synth.error_map(cam.height, cam.width, 51)
    A = synth.age_map(cam.height, cam.width, 52)
    s = sampler.sample_view(E, A, SampleParams(n_pix=51), 3, 1, 0)
    _full_chain_parity(B, p, cam, rp, sample=s)


def test_gaussian_covering_every_tile(B):
    """A small scene plus one wide, opaque Gaussian at the look-at point
    whose rectangle spans the whole tile grid: its pair lands in every tile
    (the largest per-Gaussian pair count the image allows)."""
    p, cam = small_scene(n=1500, seed=23)
    big = synth.gaussians(1, 29, logscale_mean=0.3, logscale_std=0.0)
    big[0:3, 0] = 0.0
    big[10, 0] = 4.0
    p = np.concatenate([p, big], axis=1)
    rp = RasterParams()
    pr, sv = _full_chain_parity(B, p, cam, rp)
    TX, TY = pr["TX"], pr["TY"]
    assert np.count_nonzero(sv == p.shape[1] - 1) == TX * TY


@pytest.mark.parametrize("n", [0, 1, 5, 1023, 1_000_003])
def test_check_finite_counts_nan_and_inf(B, n):
    """tgs_check_finite against numpy's isfinite: NaNs of several payloads,
    both infinities, the largest finite float and subnormals (finite), at
    lengths that are not multiples of four."""
    rng = np.random.default_rng(n)
    x = rng.normal(size=n).astype(np.float32)
    if n:
        bad = rng.choice(n, max(1, n // 97), replace=False)
        vals = np.array([np.nan, np.inf, -np.inf, np.float32(np.nan) * -1], dtype=np.float32)
        x[bad] = vals[rng.integers(0, 4, bad.size)]
        x.view(np.uint32)[bad[: bad.size // 2]] |= 0x7fc00123         # quiet NaNs with payloads
        ok = np.setdiff1d(np.arange(n), bad)[:8]
        x[ok[:4]] = np.float32(3.4e38)
        x[ok[4:]] = np.float32(1e-42)
    assert B.check_finite(dev(x)) == int((~np.isfinite(x)).sum())
