"""GPU parity of each stage against the oracle, stage by stage, on identical
seeded inputs (each GPU stage gets its inputs from synth or the oracle).

Bars: bit-exact for keys, values, ranges, sample indices, tile maps, age
maps and half error maps; FP32 values against the FP64 oracle within the
stated relative tolerances (images 1e-5, gradients 1e-4, plus an FP32
summation bound where terms cancel); pixels whose discrete decisions lie in
the oracle's guard band are excluded and counted."""
import numpy as np
import pytest
import torch

import synth
from oracle import binning, loss, maps, optim, project, project_bwd, render, sampler
from oracle.params import LossParams, OptimParams, RasterParams, SampleParams

from support import (moments_gaussian_major, moments_rows, assert_close, check_pair_lists, last_ids, ldl_conic, scene_c1, scene_scaling, small_scene,
                     splat_as_oracle, splat_record)

pytestmark = pytest.mark.gpu

RP = RasterParams()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15924_amd import binding
    binding.lib()
    return binding


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ------------------------------------------------------------------ projection
@pytest.mark.parametrize("case", ["c1", "ragged", "deg0"])
def test_project_parity(B, case):
    if case == "c1":
        p, cams = scene_c1()
        cam = cams[2]
        rp = RP
    else:
        p, cam = small_scene(n=3000, seed=5)
        rp = RasterParams(sh_degree=0) if case == "deg0" else RP
    pr = project.project(p, cam, rp)
    n = p.shape[1]
    P = dev(p)
    splat = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    depth = torch.empty(n, dtype=torch.float32, device="cuda")
    radius = torch.empty(n, dtype=torch.int32, device="cuda")
    rect = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    clamp = torch.empty(n, dtype=torch.uint8, device="cuda")
    brp = B.raster_params(sh_degree=rp.sh_degree)
    B.tgs_project(P, n, B.camera(cam), brp, splat, depth, radius, rect, clamp)
    s, d, r, rc, cm = host(splat), host(depth), host(radius), host(rect), host(clamp)
    # depth key bits: exact for every Gaussian
    assert np.array_equal(d.view(np.uint32), pr["depth32"].view(np.uint32))
    vis = pr["visible"]
    safe = vis & (pr["radius_margin"] > 1e-9)
    assert safe.sum() >= vis.sum() - 2
    assert np.array_equal(r[safe], pr["radius"][safe])
    assert np.array_equal(rc[safe], pr["rect"].T[safe])
    assert np.array_equal(r[~vis], np.zeros((~vis).sum()))
    rec = splat_record(pr)
    assert np.array_equal(s[vis][:, :2], rec[vis][:, :2])               # integer parts of the centre
    px = s[:, 0].astype(np.float64) + s[:, 2]
    py = s[:, 1].astype(np.float64) + s[:, 3]
    assert_close(px[vis], pr["mean2d"][0][vis], 0, 2e-7 * 2 ** 0, "centre x")
    assert_close(py[vis], pr["mean2d"][1][vis], 0, 2e-7, "centre y")
    # the conic in its LDL^T form (a, beta, delta); beta against the scale
    # sqrt(c / a) it can reach (|beta| <= sqrt(c / a) for a positive definite Q)
    ldl = ldl_conic(pr["conic"]).T[vis]
    assert_close(s[vis][:, 4], ldl[:, 0], 2e-7, 0, "conic a")
    scale_b = np.sqrt(pr["conic"][2][vis] / pr["conic"][0][vis])
    assert np.all(np.abs(s[vis][:, 5] - ldl[:, 1]) <= 2e-7 * (np.abs(ldl[:, 1]) + 1e-3 * scale_b)), "conic beta"
    assert_close(s[vis][:, 6], ldl[:, 2], 2e-7, 0, "conic delta")
    assert_close(s[vis][:, 7], pr["opacity"][vis], 2e-7, 0, "opacity")
    assert_close(s[vis][:, 8:11], pr["rgb"].T[vis], 2e-7, 1e-12, "rgb")
    clamp_bits = (pr["clamp"][0] * 1 + pr["clamp"][1] * 2 + pr["clamp"][2] * 4).astype(np.uint8)
    assert np.array_equal(cm[vis], clamp_bits[vis])


# ------------------------------------------------------------------ binning + sort
@pytest.mark.parametrize("case", ["c1_sampled", "scaling"])
def test_bin_sort_async_equals_the_blocking_call(B, case):
    """tgs_bin_sort_async queues the same lists without a host wait: keys,
    ids and ranges bit for bit equal to tgs_bin_sort's, counts = (list
    length, capacity needed); with a short capacity the lists come out
    empty and counts[1] still reports the capacity needed."""
    if case == "c1_sampled":
        p, cams = scene_c1()
        cam = cams[2]
    else:
        p, cam = scene_scaling()
    pr = project.project(p, cam, RP)
    TX, TY = pr["TX"], pr["TY"]
    n = p.shape[1]
    ts = None
    if case == "c1_sampled":
        valid = np.sort(np.random.default_rng(3).choice(TX * TY, 64, replace=False))
        t = -np.ones(TX * TY, dtype=np.int32)
        t[valid] = np.arange(valid.size)
        ts = dev(t)
    rec = splat_record(pr)
    rect, splat, depth = dev(pr["rect"].T.astype(np.int32)), dev(rec), dev(pr["depth32"])
    rect_area = (pr["rect"][2] - pr["rect"][0]) * (pr["rect"][3] - pr["rect"][1])
    cap = int(rect_area[pr["visible"]].sum()) + 5
    ws = torch.empty(B.tgs_bin_sort_workspace_size(n, cap, TX * TY), dtype=torch.uint8, device="cuda")
    out = []
    for sync in (True, False):
        K = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
        V = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        R = torch.full((TX * TY, 2), -1, dtype=torch.int32, device="cuda")
        c = torch.full((2,), -1, dtype=torch.int64, device="cuda")
        if sync:
            npairs = B.tgs_bin_sort(rect, splat, depth, n, ts, TX, TY, 1.0 / 255.0, K, V, cap, R, None, ws)
        else:
            B.tgs_bin_sort_async(rect, splat, depth, n, ts, TX, TY, 1.0 / 255.0, K, V, cap, R, None, c, ws)
        out.append((host(K), host(V), host(R), host(c)))
    (k1, v1, r1, _), (k2, v2, r2, c2) = out
    assert c2[0] == npairs > 0 and npairs <= c2[1] <= cap
    assert np.array_equal(k1[:npairs], k2[:npairs]) and np.array_equal(v1[:npairs], v2[:npairs])
    assert np.array_equal(r1, r2)
    short = int(c2[1]) - 1
    R = torch.full((TX * TY, 2), -1, dtype=torch.int32, device="cuda")
    c = torch.zeros(2, dtype=torch.int64, device="cuda")
    V = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    B.tgs_bin_sort_async(rect, splat, depth, n, ts, TX, TY, 1.0 / 255.0, None, V, short, R, None, c, ws)
    assert np.array_equal(host(c), c2) and not host(R).any() and (host(V) == -7).all()


def test_bin_sort_wide_tile_ids_with_id_payload(B):
    """A 4100x4100 view (66,049 tiles: 17 tile bits) of 50k Gaussians (16 id
    bits): tile and id no longer fit one 32-bit key, so the pair sort keys on
    the tile and carries the id as a payload.  Keys, ids and ranges against
    the oracle's rectangle lists as in the other binning tests."""
    p = synth.gaussians(50000, 41, logscale_mean=-5.0)
    W = H = 4100
    cam = synth.look_at((1.9, -1.6, 1.5), fx=300.0 * W / 256, fy=300.0 * W / 256, width=W, height=H)
    pr = project.project(p, cam, RP)
    TX, TY = pr["TX"], pr["TY"]
    assert TX * TY == 66049
    rec = splat_record(pr)
    q = splat_as_oracle(pr, rec)
    rect_area = (pr["rect"][2] - pr["rect"][0]) * (pr["rect"][3] - pr["rect"][1])
    cap = int(rect_area[pr["visible"]].sum()) + 17
    n = p.shape[1]
    K = torch.empty(cap, dtype=torch.int64, device="cuda")
    V = torch.empty(cap, dtype=torch.int32, device="cuda")
    R = torch.empty((TX * TY, 2), dtype=torch.int32, device="cuda")
    ws = torch.empty(B.tgs_bin_sort_workspace_size(n, cap, TX * TY), dtype=torch.uint8, device="cuda")
    npairs = B.tgs_bin_sort(dev(pr["rect"].T.astype(np.int32)), dev(rec), dev(pr["depth32"]), n, None, TX, TY,
                            1.0 / 255.0, K, V, cap, R, None, ws)
    info = check_pair_lists(host(V)[:npairs].view(np.uint32), host(R), npairs, q, keys=host(K),
                            max_dropped_checked=100000)
    assert npairs > 100000 and info["dropped"] > 0


@pytest.mark.parametrize("case", ["c1_all", "c1_sampled", "ragged"])
def test_bin_sort_lists_against_rectangle_lists(B, case):
    """The GPU's per-tile lists against the oracle's rectangle lists: an
    order-preserving subsequence with consistent keys and ranges, every
    dropped pair unable to composite anywhere in its tile (checked at all
    256 pixel centres), only valid tiles listed, touched = the Gaussians
    listed; and the capacity contract (a short capacity reports a count that
    then suffices)."""
    if case.startswith("c1"):
        p, cams = scene_c1()
        cam = cams[0]
    else:
        p, cam = small_scene(n=3000, seed=6)
    pr = project.project(p, cam, RP)
    TX, TY = pr["TX"], pr["TY"]
    n = p.shape[1]
    valid = None
    tile_slot = None
    if case == "c1_sampled":
        valid = np.sort(np.random.default_rng(1).choice(TX * TY, 64, replace=False))
        ts = -np.ones(TX * TY, dtype=np.int32)
        ts[valid] = np.arange(valid.size)
        tile_slot = dev(ts)
    rec = splat_record(pr)
    q = splat_as_oracle(pr, rec)
    rect = dev(pr["rect"].T.astype(np.int32))
    splat = dev(rec)
    depth = dev(pr["depth32"])
    rect_area = (pr["rect"][2] - pr["rect"][0]) * (pr["rect"][3] - pr["rect"][1])
    cap = int(rect_area[pr["visible"]].sum()) + 17              # the rectangle lists bound any list
    K = torch.empty(cap, dtype=torch.int64, device="cuda")
    V = torch.empty(cap, dtype=torch.int32, device="cuda")
    R = torch.empty((TX * TY, 2), dtype=torch.int32, device="cuda")
    touched = torch.zeros(n, dtype=torch.uint8, device="cuda")
    ws = torch.empty(B.tgs_bin_sort_workspace_size(n, cap, TX * TY), dtype=torch.uint8, device="cuda")
    npairs = B.tgs_bin_sort(rect, splat, depth, n, tile_slot, TX, TY, 1.0 / 255.0, K, V, cap, R, touched, ws)
    vals = host(V)[:npairs].view(np.uint32)
    info = check_pair_lists(vals, host(R), npairs, q, valid, keys=host(K))
    assert info["dropped"] > 0.15 * info["oracle"] and info["checked"] == info["dropped"]
    t_ref = np.zeros(n, dtype=np.uint8)
    t_ref[np.unique(vals)] = 1
    assert np.array_equal(host(touched), t_ref)
    # too-small capacity reports the required count, which then suffices (the
    # failed call clears its ranges, so it gets arrays of its own)
    R_first = R.clone()
    with pytest.raises(B.CapacityError) as ei:
        B.tgs_bin_sort(rect, splat, depth, n, tile_slot, TX, TY, 1.0 / 255.0, K.clone(), V.clone(), 10,
                       torch.empty_like(R), None, ws)
    req = ei.value.required
    assert npairs <= req <= int(rect_area[np.unique(vals)].sum())
    ws2 = torch.empty(B.tgs_bin_sort_workspace_size(n, req, TX * TY), dtype=torch.uint8, device="cuda")
    K2 = torch.empty(req, dtype=torch.int64, device="cuda")
    V2 = torch.empty(req, dtype=torch.int32, device="cuda")
    R2 = torch.empty((TX * TY, 2), dtype=torch.int32, device="cuda")
    assert B.tgs_bin_sort(rect, splat, depth, n, tile_slot, TX, TY, 1.0 / 255.0, K2, V2, req, R2, None, ws2) == npairs
    assert torch.equal(K2[:npairs], K[:npairs]) and torch.equal(V2[:npairs], V[:npairs]) and torch.equal(R2, R_first)


# ------------------------------------------------------------------ sampler
@pytest.mark.parametrize("W,H,n_pix,n_sel,zero,pred", [(256, 256, 64, 64, 0.1, False), (150, 107, 25, -1, 0.3, False),
                                                        (150, 107, 256, -1, 0.0, False), (96, 80, 51, 7, 1.0, False),
                                                        (1296, 840, 64, -1, 0.1, False), (256, 256, 64, 64, 0.1, True),
                                                        (150, 107, 25, 20, 0.3, True), (1296, 840, 64, 1073, 0.1, False),
                                                        (1296, 840, 64, 1073, 0.1, True),
                                                        (1296, 840, 16, 3000, 0.1, "sparse"),
                                                        (2560, 1440, 8, 10800, 0.1, "sparse"),
                                                        (1920, 1600, 8, 9000, 0.1, False),
                                                        (2560, 1900, 8, 5000, 0.1, "sparse"),
                                                        (3840, 2160, 8, 100, 0.1, False),
                                                        (150, 107, 25, 1, 0.3, False), (96, 80, 51, 29, 0.0, False)])
def test_sampler_bit_exact(B, W, H, n_pix, n_sel, zero, pred):
    """pred: the tile pass draws by predicted tile errors (negative, NaN and
    out-of-range predictions included); "sparse": seven tiles in ten predict
    no error, so the weighted race runs out and the rest are uniform.  The
    select stages the keys in LDS up to 19,040 tiles and reads them from
    global memory at 32,400; one tile drawn, and all but one of 30."""
    E = synth.error_map(H, W, 31, zero_frac=zero)
    A = synth.age_map(H, W, 32)
    seed, step, view = 3, 5, 2
    sp = SampleParams(n_pix=n_pix, n_tiles_sel=n_sel)
    tile_pred = None
    if pred:
        nt = ((W + 15) // 16) * ((H + 15) // 16)
        tile_pred = np.random.default_rng(33).normal(0.2, 0.2, nt).astype(np.float32)
        tile_pred[:3] = [np.nan, 1e30, -1.0]
        if pred == "sparse":
            tile_pred[np.random.default_rng(34).random(nt) < 0.7] = 0.0
    bsp = B.sample_params(n_pix, n_tiles_sel=n_sel, seed=seed, step=step, view=view)
    n_st = B.tgs_sample_tile_count(H, W, bsp)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    vt = torch.empty(n_st, dtype=torch.int32, device="cuda")
    off = torch.empty(n_st + 1, dtype=torch.int32, device="cuda")
    pix = torch.empty(n_st * n_pix, dtype=torch.uint8, device="cuda")
    slot = torch.empty(TX * TY, dtype=torch.int32, device="cuda")
    totals = torch.zeros(2, dtype=torch.int64, device="cuda")
    ws = torch.empty(B.tgs_sample_workspace_size(H, W), dtype=torch.uint8, device="cuda")
    B.tgs_sample(dev(E), dev(A), H, W, bsp, vt, off, pix, slot, totals, ws,
                 tile_pred=None if tile_pred is None else dev(tile_pred))
    g_vt, g_off, g_pix, g_slot, g_tot = host(vt), host(off), host(pix), host(slot), host(totals)
    subset = None
    if W * H > 200000 and n_sel < 0:   # full-size view, every tile: the oracle checks a subset of them
        rng = np.random.default_rng(0)
        subset = np.unique(np.concatenate([rng.choice(TX * TY, 120, replace=False),
                                           np.arange(TX * TY - TX, TX * TY), np.arange(TX - 1, TX * TY, TX)]))
    ref = sampler.sample_view(E, A, sp, seed, step, view, tiles_subset=subset, tile_pred=tile_pred)
    if subset is None:
        assert np.array_equal(g_vt, ref["valid_tiles"])
        assert np.array_equal(g_off, ref["tile_off"])
        assert np.array_equal(g_pix[: g_off[-1]], ref["pix"])
        ts = -np.ones(TX * TY, dtype=np.int32)
        ts[ref["valid_tiles"]] = np.arange(ref["valid_tiles"].size)
        assert np.array_equal(g_slot, ts)
        assert g_tot.tolist() == [int(ref["tile_off"][-1]), n_st]
    else:
        assert np.array_equal(g_vt, np.arange(TX * TY))
        for i, t in enumerate(ref["valid_tiles"]):
            got = g_pix[g_off[t]:g_off[t + 1]]
            want = ref["pix"][ref["tile_off"][i]:ref["tile_off"][i + 1]]
            assert np.array_equal(got, want), t


@pytest.mark.parametrize("hard,stable", [(0, 0), (1000, 0), (0, 1000)])
def test_sampler_split_extremes_bit_exact(B, hard, stable):
    """The sampler with the whole budget in one class: all mixed (uniform
    random pixels per tile, the random-pixel-sampling baseline), all error
    draws, all largest-age."""
    W, H, n_pix = 150, 107, 64
    E = synth.error_map(H, W, 34, zero_frac=0.2)
    A = synth.age_map(H, W, 35)
    sp = SampleParams(n_pix=n_pix, hard_permille=hard, stable_permille=stable)
    bsp = B.sample_params(n_pix, hard, stable, seed=3, step=6, view=1)
    n_st = B.tgs_sample_tile_count(H, W, bsp)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    vt = torch.empty(n_st, dtype=torch.int32, device="cuda")
    off = torch.empty(n_st + 1, dtype=torch.int32, device="cuda")
    pix = torch.empty(n_st * n_pix, dtype=torch.uint8, device="cuda")
    slot = torch.empty(TX * TY, dtype=torch.int32, device="cuda")
    totals = torch.zeros(2, dtype=torch.int64, device="cuda")
    ws = torch.empty(B.tgs_sample_workspace_size(H, W), dtype=torch.uint8, device="cuda")
    B.tgs_sample(dev(E), dev(A), H, W, bsp, vt, off, pix, slot, totals, ws)
    ref = sampler.sample_view(E, A, sp, 3, 6, 1)
    g_off = host(off)
    assert np.array_equal(host(vt), ref["valid_tiles"])
    assert np.array_equal(g_off, ref["tile_off"])
    assert np.array_equal(host(pix)[: g_off[-1]], ref["pix"])


# ------------------------------------------------------------------ forward render
def _render_case(case):
    if case == "c1_sparse":
        p, cams = scene_c1()
        cam = cams[1]
        E = synth.error_map(cam.height, cam.width, 41)
        A = synth.age_map(cam.height, cam.width, 42)
        s = sampler.sample_view(E, A, SampleParams(n_pix=64, n_tiles_sel=64), 3, 1, 1)
    elif case == "ragged_sparse25":
        p, cam = small_scene(n=2500, seed=7)
        E = synth.error_map(cam.height, cam.width, 43)
        A = synth.age_map(cam.height, cam.width, 44)
        s = sampler.sample_view(E, A, SampleParams(n_pix=25), 3, 1, 0)
    elif case == "ragged_sparse128":
        p, cam = small_scene(n=2500, seed=8)
        E = synth.error_map(cam.height, cam.width, 45)
        A = synth.age_map(cam.height, cam.width, 46)
        s = sampler.sample_view(E, A, SampleParams(n_pix=128), 3, 1, 0)
    else:
        p, cam = small_scene(n=2500, seed=9)
        s = None
    return p, cam, s


def _gpu_render(B, rec, sv, ranges, cam, s, rp, n_pix):
    TX, TY = (cam.width + 15) // 16, (cam.height + 15) // 16
    splat = dev(rec)
    V = dev(sv.view(np.int32))
    R = dev(ranges.astype(np.int32))
    if s is None:
        P = cam.width * cam.height
        vt = off = pix = None
        n_st, mpt = TX * TY, 256
    else:
        P = int(s["tile_off"][-1])
        vt, off, pix = dev(s["valid_tiles"]), dev(s["tile_off"]), dev(s["pix"])
        n_st, mpt = s["valid_tiles"].size, n_pix
    out = torch.empty((max(P, 1), 4), dtype=torch.float32, device="cuda")
    nc = torch.empty(max(P, 1), dtype=torch.int32, device="cuda")
    cnt = torch.zeros((2, B.COUNTER_SLOTS), dtype=torch.int64, device="cuda")
    B.tgs_render_fwd(splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, mpt, rp, out, nc, cnt)
    return out, nc, cnt, (splat, V, R, vt, off, pix, n_st, mpt, TX, TY)


@pytest.mark.parametrize("case,bg", [("c1_sparse", (0, 0, 0)), ("ragged_sparse25", (0, 0, 0)),
                                     ("ragged_sparse128", (0.3, 0.6, 0.9)), ("dense", (0, 0, 0))])
def test_render_fwd_parity(B, case, bg):
    p, cam, s = _render_case(case)
    rp = RasterParams(bg=bg)
    pr = project.project(p, cam, rp)
    rec = splat_record(pr)
    q = splat_as_oracle(pr, rec)
    valid = None if s is None else s["valid_tiles"]
    _, sv, ranges = binning.bin_and_sort(pr, valid)
    if s is None:
        xs, ys = render.dense_pixels(cam.width, cam.height)
    else:
        xs, ys, _ = sampler.sample_coords(s, cam.width, cam.height)
    ref = render.render_pixels(q, sv, ranges, xs, ys, rp)
    n_pix = 256 if s is None else max(int(np.diff(s["tile_off"]).max()), 1)
    out, nc, cnt, _ = _gpu_render(B, rec, sv, ranges, cam, s, B.raster_params(bg=bg), n_pix)
    o, c, k = host(out)[: xs.size], host(nc)[: xs.size], host(cnt).sum(axis=1)
    ok = ~ref["flag"]
    assert ok.mean() > 0.995, ok.mean()
    assert_close(o[ok, :3], ref["rgb"][ok], 1e-5, 1e-7, "rgb")
    assert_close(o[ok, 3], ref["T"][ok], 1e-5, 1e-7, "T_final")
    assert np.array_equal(c[ok], ref["n_contrib"][ok])
    # counters: exact when no pixel sits in the guard band
    if ok.all():
        assert k.tolist() == [int(ref["n_eval"].sum()), int(ref["n_blend"].sum())]
    else:
        assert abs(int(k[1]) - int(ref["n_blend"].sum())) <= 64 * (~ok).sum()


def test_sparse_full_rate_equals_dense_bitwise(B):
    p, cam = small_scene(n=2500, seed=10)
    pr = project.project(p, cam, RP)
    rec = splat_record(pr)
    _, sv, ranges = binning.bin_and_sort(pr)
    TX, TY = pr["TX"], pr["TY"]
    E = synth.error_map(cam.height, cam.width, 47)
    A = synth.age_map(cam.height, cam.width, 48)
    s = sampler.sample_view(E, A, SampleParams(n_pix=256), 3, 1, 0)
    out_s, nc_s, _, _ = _gpu_render(B, rec, sv, ranges, cam, s, B.raster_params(), 256)
    out_d, nc_d, _, _ = _gpu_render(B, rec, sv, ranges, cam, None, B.raster_params(), 256)
    xs, ys, _ = sampler.sample_coords(s, cam.width, cam.height)
    od = host(out_d)[ys * cam.width + xs]
    assert np.array_equal(host(out_s)[: xs.size].view(np.uint32), od.view(np.uint32))
    assert np.array_equal(host(nc_s)[: xs.size], host(nc_d)[ys * cam.width + xs])


# ------------------------------------------------------------------ backward render
@pytest.mark.parametrize("case", ["c1_sparse", "ragged_sparse25", "ragged_sparse128", "dense"])
def test_render_bwd_parity(B, case):
    p, cam, s = _render_case(case)
    rp = RasterParams(bg=(0.2, 0.1, 0.4))
    pr = project.project(p, cam, rp)
    rec = splat_record(pr)
    q = splat_as_oracle(pr, rec)
    valid = None if s is None else s["valid_tiles"]
    _, sv, ranges = binning.bin_and_sort(pr, valid)
    if s is None:
        xs, ys = render.dense_pixels(cam.width, cam.height)
    else:
        xs, ys, _ = sampler.sample_coords(s, cam.width, cam.height)
    ref = render.render_pixels(q, sv, ranges, xs, ys, rp)
    g = np.random.default_rng(3).normal(size=(xs.size, 3)) * 1e-3
    g[ref["flag"]] = 0.0                     # guard-band pixels carry no gradient
    g2d, g2d_abs = render.render_pixels_bwd(q, sv, ranges, xs, ys, g, rp, with_abs=True)
    n_pix = 256 if s is None else max(int(np.diff(s["tile_off"]).max()), 1)
    brp = B.raster_params(bg=rp.bg)
    # forward outputs from the oracle (FP32), ncontrib exact
    out = np.zeros((xs.size, 4), dtype=np.float32)
    out[:, :3] = ref["rgb"]
    out[:, 3] = ref["T"]
    dl = np.zeros((xs.size, 4), dtype=np.float32)
    dl[:, :3] = g
    if s is None:
        o_full = np.zeros((cam.width * cam.height, 4), dtype=np.float32)
        d_full = np.zeros_like(o_full)
        nc_full = np.zeros(cam.width * cam.height, dtype=np.int32)
        idx = ys * cam.width + xs
        o_full[idx], d_full[idx], nc_full[idx] = out, dl, ref["n_contrib"]
        out, dl, ncv = o_full, d_full, nc_full
    else:
        ncv = ref["n_contrib"].astype(np.int32)
    TX, TY = pr["TX"], pr["TY"]
    G = torch.zeros((p.shape[1], 9), dtype=torch.float32, device="cuda")
    vt = off = pix = None
    n_st = TX * TY
    if s is not None:
        vt, off, pix = dev(s["valid_tiles"]), dev(s["tile_off"]), dev(s["pix"])
        n_st = s["valid_tiles"].size
    touched = torch.full((p.shape[1],), 2, dtype=torch.uint8, device="cuda")
    B.tgs_render_bwd(dev(rec), dev(sv.view(np.int32)), dev(ranges.astype(np.int32)), TX, TY, cam.width,
                     cam.height, vt, off, pix, n_st, n_pix, brp, dev(out), dev(ncv), dev(dl), G, touched=touched)
    got = host(G).T
    # touched: the Gaussians composited at a sample (1), the rest untouched (2)
    t_got = host(touched)
    assert set(np.unique(t_got).tolist()) <= {1, 2}
    on = t_got == 1
    ok = ~ref["flag"]
    sure = render.render_pixels(q, sv, ranges, xs[ok], ys[ok], rp)["composited"]
    near = np.zeros_like(on)
    for t in np.unique(((ys // 16) * pr["TX"] + xs // 16)[~ok]):
        near[sv[ranges[t, 0]:ranges[t, 1]].astype(np.int64)] = True
    assert not (sure & ~on).any() and not (on & ~(ref["composited"] | near)).any() and sure.sum() > 100
    names = ["dx", "dy", "ca", "cb", "cc", "opacity", "r", "g", "b"]
    for f in range(9):
        # 1e-4 relative, plus 16 FP32 ulps of the error scale of each sum (see
        # render_pixels_bwd: B_k = I - C_{<=k} cancels in a front-to-back replay)
        assert_close(got[f], g2d[f], 1e-4, 2e-6 * g2d_abs[f] + 1e-12, names[f])


@pytest.mark.parametrize("mode", ["sparse64", "sparse128", "dense"])
def test_render_bwd_chunked_equals_single(B, mode):
    """Deep lists (half the pixels composite more than 192 Gaussians): the
    forward's state record does not change its outputs, and the backward
    split into (tile, chunk) workgroups starting from that record gives the
    gradients of the single-workgroup replay (same per-pixel arithmetic;
    only the order of the float atomics differs)."""
    p, cam = small_scene(n=4000, seed=12)
    p = np.array(p)
    p[10] = -3.5                              # opacity logit: ~3% per Gaussian
    pr = project.project(p, cam, RP)
    rec = splat_record(pr)
    _, sv, ranges = binning.bin_and_sort(pr)
    if mode == "dense":
        s, n_pix = None, 256
    else:
        n_pix = 64 if mode == "sparse64" else 128
        E = synth.error_map(cam.height, cam.width, 61)
        A = synth.age_map(cam.height, cam.width, 62)
        s = sampler.sample_view(E, A, SampleParams(n_pix=n_pix), 3, 1, 0)
    out, nc, _, (splat, V, R, vt, off, pix, n_st, mpt, TX, TY) = _gpu_render(
        B, rec, sv, ranges, cam, s, B.raster_params(), n_pix)
    state = torch.zeros(B.tgs_render_state_size(n_st, mpt) // 4, dtype=torch.float32, device="cuda")
    out2 = torch.empty_like(out)
    nc2 = torch.empty_like(nc)
    B.tgs_render_fwd(splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, mpt, B.raster_params(),
                     out2, nc2, None, state)
    assert np.array_equal(host(out).view(np.uint32), host(out2).view(np.uint32))
    assert np.array_equal(host(nc), host(nc2))
    assert (host(nc) > (B.RENDER_CHUNKS - 1) * B.RENDER_CHUNK_LEN).mean() > 0.1   # the last chunk has work
    dl = torch.from_numpy(np.random.default_rng(5).normal(size=out.shape).astype(np.float32) * 1e-3).cuda()
    G1 = torch.zeros((p.shape[1], 9), dtype=torch.float32, device="cuda")
    G2 = torch.zeros_like(G1)
    args = (splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, mpt, B.raster_params(), out, nc, dl)
    B.tgs_render_bwd(*args, G1)
    B.tgs_render_bwd(*args, G2, state)
    g1, g2 = host(G1), host(G2)
    scale = np.abs(g1).max(axis=0) + 1e-12
    assert_close(g2, g1, 1e-5, 1e-6 * scale, "chunked vs single")


# ------------------------------------------------------------------ loss, maps
@pytest.mark.parametrize("structure", ["ncc", "ssim"])
@pytest.mark.parametrize("case", ["c1", "ragged25", "dense"])
def test_loss_parity(B, case, structure):
    """The sparse loss (Charbonnier plus the tile S-NCC, or the S-SSIM of the
    ablation) against the oracle: per-pixel error, balance weights, dL/dI
    and the loss value."""
    lp = LossParams(structure=structure)
    rng = np.random.default_rng(4)
    if case == "dense":
        W, H = 70, 45
        TX, TY = 5, 3
        x = rng.uniform(size=(W * H, 3)).astype(np.float32)
        gt = synth.image(H, W, 50)
        xs, ys = render.dense_pixels(W, H)
        tiles = (ys // 16) * TX + xs // 16
        order = np.argsort(tiles, kind="stable")
        off = np.concatenate([[0], np.cumsum(np.bincount(tiles, minlength=TX * TY))])
        P_step, T_step = W * H + 100, TX * TY + 3
        ref = loss.sparse_loss(x[order], gt[:, ys[order], xs[order]].T, off, P_step, T_step, lp)
        dL_ref = np.zeros((W * H, 3))
        dL_ref[order] = ref["dL"]
        err_ref = np.zeros(W * H)
        err_ref[order] = ref["err"]
        out = np.zeros((W * H, 4), dtype=np.float32)
        out[:, :3] = x
        vt = offt = pix = None
        n_st = TX * TY
        lam_ref = ref["lam"]
    else:
        W, H, n_pix, n_sel = (256, 256, 64, 64) if case == "c1" else (150, 107, 25, -1)
        E = synth.error_map(H, W, 51)
        A = synth.age_map(H, W, 52)
        s = sampler.sample_view(E, A, SampleParams(n_pix=n_pix, n_tiles_sel=n_sel), 3, 1, 0)
        xs, ys, _ = sampler.sample_coords(s, W, H)
        gt = synth.image(H, W, 53)
        x = np.clip(gt[:, ys, xs].T + rng.normal(0, 0.05, size=(xs.size, 3)), 0, 1).astype(np.float32)
        P_step, T_step = xs.size * 3, s["valid_tiles"].size * 3
        ref = loss.sparse_loss(x, gt[:, ys, xs].T, s["tile_off"], P_step, T_step, lp)
        dL_ref, err_ref, lam_ref = ref["dL"], ref["err"], ref["lam"]
        out = np.zeros((xs.size, 4), dtype=np.float32)
        out[:, :3] = x
        vt, offt, pix = dev(s["valid_tiles"]), dev(s["tile_off"]), dev(s["pix"])
        n_st = s["valid_tiles"].size
    Pn = out.shape[0]
    dL = torch.empty((Pn, 4), dtype=torch.float32, device="cuda")
    err = torch.empty(Pn, dtype=torch.float32, device="cuda")
    lam = torch.empty(n_st, dtype=torch.float32, device="cuda")
    tl = torch.empty((n_st, 2), dtype=torch.float32, device="cuda")
    totals = dev(np.array([P_step, T_step], dtype=np.int64))
    B.tgs_loss(dev(out), dev(gt), H, W, vt, offt, pix, n_st, totals, B.loss_params(structure=structure), dL, err,
               lam, tl)
    gd, ge, gl, gt_l = host(dL), host(err), host(lam), host(tl)
    assert_close(ge, err_ref, 1e-6, 1e-7, "err")
    assert_close(gl, lam_ref, 1e-4, 1e-6, "lambda")
    scale = np.abs(dL_ref).max()
    assert_close(gd[:, :3], dL_ref, 1e-4, 1e-5 * scale, "dL/dI")
    assert (gd[:, 3] == 0).all()
    assert_close(gt_l.sum(), ref["loss_l1"] + ref["loss_ncc"], 1e-5, 0, "loss")


def test_ema_age_and_error_init_bit_exact(B):
    W, H = 150, 107
    E = synth.error_map(H, W, 61)
    A = synth.age_map(H, W, 62, max_age=65535)
    A[0, :5] = 65535
    s = sampler.sample_view(E, A, SampleParams(n_pix=51, n_tiles_sel=9), 3, 1, 0)
    xs, ys, _ = sampler.sample_coords(s, W, H)
    err = np.random.default_rng(5).uniform(0, 2, size=xs.size).astype(np.float32)
    E_ref, A_ref = maps.ema_age_update(E, A, xs, ys, err, 0.4)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    ts = -np.ones(TX * TY, dtype=np.int32)
    ts[s["valid_tiles"]] = np.arange(s["valid_tiles"].size)
    Eg, Ag = dev(E.view(np.int16)), dev(A.view(np.int16))
    B.tgs_ema_age_update(Eg, Ag, H, W, dev(ts), dev(s["tile_off"]), dev(s["pix"]), dev(err), 0.4)
    assert np.array_equal(host(Eg).view(np.uint16), E_ref)
    assert np.array_equal(host(Ag).view(np.uint16), A_ref)
    # dense error initialisation
    x = np.random.default_rng(6).uniform(size=(H, W, 3)).astype(np.float32)
    gt = synth.image(H, W, 63)
    out = np.zeros((H * W, 4), dtype=np.float32)
    out[:, :3] = x.reshape(-1, 3)
    Eo = torch.empty(H * W, dtype=torch.int16, device="cuda")
    B.tgs_error_init(dev(out), dev(gt), H, W, Eo)
    assert np.array_equal(host(Eo).view(np.uint16), maps.dense_error_init(x, gt).ravel())


# ------------------------------------------------------------------ projection backward
@pytest.mark.parametrize("case", ["c1", "deg1_bg"])
def test_project_bwd_parity(B, case):
    if case == "c1":
        p, cams = scene_c1(4000)
        cam, rp = cams[3], RP
    else:
        p, cam = small_scene(n=3000, seed=12)
        rp = RasterParams(sh_degree=1)
    pr = project.project(p, cam, rp)
    n = p.shape[1]
    g2d = np.random.default_rng(7).normal(size=(9, n))
    g2d[2:5] *= 1e2                                      # conic gradients are large per unit
    ref = project_bwd.project_bwd(p, cam, pr, g2d, rp)
    P = dev(p)
    brp = B.raster_params(sh_degree=rp.sh_degree)
    splat = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    depth = torch.empty(n, dtype=torch.float32, device="cuda")
    radius = torch.empty(n, dtype=torch.int32, device="cuda")
    rect = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    clamp = torch.empty(n, dtype=torch.uint8, device="cuda")
    c = B.camera(cam)
    B.tgs_project(P, n, c, brp, splat, depth, radius, rect, clamp)
    grad0 = np.random.default_rng(8).normal(size=(59, n)).astype(np.float32)   # accumulation target
    G = dev(grad0)
    B.tgs_project_bwd(P, n, c, brp, radius, clamp, dev(g2d.T.astype(np.float32)), G)
    got = host(G).astype(np.float64) - grad0
    g32 = g2d.astype(np.float32).astype(np.float64)
    ref = project_bwd.project_bwd(p, cam, pr, g32, rp)
    groups = {"mean": slice(0, 3), "logscale": slice(3, 6), "quat": slice(6, 10), "opacity": slice(10, 11),
              "sh": slice(11, 59)}
    for name, sl in groups.items():
        scale = np.abs(ref[sl]).max()
        assert_close(got[sl], ref[sl], 1e-5, 1e-6 * scale + 4e-7 * np.abs(grad0[sl]), name)
    # overwrite mode: every entry written, culled Gaussians get zeros
    G2 = torch.full((59, n), float("nan"), dtype=torch.float32, device="cuda")
    B.tgs_project_bwd(P, n, c, brp, radius, clamp, dev(g2d.T.astype(np.float32)), G2, accumulate=False)
    got2 = host(G2).astype(np.float64)
    assert np.isfinite(got2).all()
    culled = host(radius) == 0
    assert (got2[:, culled] == 0).all()
    for name, sl in groups.items():
        scale = np.abs(ref[sl]).max()
        assert_close(got2[sl], ref[sl], 1e-5, 1e-6 * scale, name)


# ------------------------------------------------------------------ fused backward + optimizer
@pytest.mark.parametrize("mode,prev,deg,n", [(0, False, 3, 4000), (1, True, 3, 4000), (2, False, 3, 4000),
                                            (0, True, 1, 4000), (0, False, 3, 20011), (1, True, 3, 20011)])
def test_project_bwd_optimizer_fused(B, mode, prev, deg, n):
    """The fused entry point equals tgs_project_bwd then tgs_optimizer_step
    bit for bit (culled, untouched and touched-but-culled Gaussians included;
    at 20011 Gaussians the update runs as two halves on two streams)."""
    p, cams = scene_c1(n)
    cam = cams[2]
    n = p.shape[1]
    rng = np.random.default_rng(31 + mode)
    brp = B.raster_params(sh_degree=deg)
    c = B.camera(cam)
    P0 = dev(p)
    splat = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    depth = torch.empty(n, dtype=torch.float32, device="cuda")
    radius = torch.empty(n, dtype=torch.int32, device="cuda")
    rect = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    clamp = torch.empty(n, dtype=torch.uint8, device="cuda")
    B.tgs_project(P0, n, c, brp, splat, depth, radius, rect, clamp)
    g2d = rng.normal(size=(n, 9)).astype(np.float32)
    g2d[:, 2:5] *= 100.0
    m0 = (rng.normal(size=(59, n)) * 1e-3).astype(np.float32)
    v0 = rng.uniform(0, 1e-4, size=(59, n)).astype(np.float32)
    touched = (rng.uniform(size=n) < 0.8).astype(np.uint8)
    grad_prev = rng.normal(size=(59, n)).astype(np.float32) if prev else None
    op = B.optim_params(lm_mode=mode)
    step = 5
    # unfused: gradient (accumulated onto the earlier views' one), then the update
    Pa, Ma, Va = dev(p), dev(moments_gaussian_major(m0)), dev(moments_gaussian_major(v0))
    G = dev(grad_prev) if prev else torch.empty((59, n), dtype=torch.float32, device="cuda")
    B.tgs_project_bwd(Pa, n, c, brp, radius, clamp, dev(g2d), G, accumulate=prev)
    B.tgs_optimizer_step(Pa, G, Ma, Va, n, dev(touched), op, step)
    # fused
    Pb, Mb, Vb = dev(p), dev(moments_gaussian_major(m0)), dev(moments_gaussian_major(v0))
    B.tgs_project_bwd_optimizer_step(Pb, n, c, brp, radius, clamp, dev(g2d), dev(grad_prev) if prev else None,
                                     Mb, Vb, dev(touched), op, step,
                                     torch.empty(B.tgs_project_bwd_optimizer_workspace_size(n), dtype=torch.uint8,
                                                 device="cuda"))
    assert (host(radius) == 0).any() and (touched == 0).any()
    for name, a, b in (("params", Pa, Pb), ("m", Ma, Mb), ("v", Va, Vb)):
        assert torch.equal(a, b), name
    assert np.array_equal(host(Pb)[:, touched == 0], p[:, touched == 0])


# ------------------------------------------------------------------ optimizer
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_optimizer_parity(B, mode):
    rng = np.random.default_rng(9 + mode)
    N = 5000
    p = rng.normal(size=(59, N)).astype(np.float32)
    g = (rng.normal(size=(59, N)) * 10.0 ** rng.uniform(-5, 0, size=(59, N))).astype(np.float32)
    m = (rng.normal(size=(59, N)) * 1e-3).astype(np.float32)
    v = (rng.uniform(0, 1e-4, size=(59, N))).astype(np.float32)
    touched = (rng.uniform(size=N) < 0.7).astype(np.uint8)
    op = OptimParams(lm_mode=mode)
    step = 7
    rp_, rm, rv = optim.optimizer_step(p, g, m, v, touched, op, step)
    P, M, V = dev(p), dev(moments_gaussian_major(m)), dev(moments_gaussian_major(v))
    B.tgs_optimizer_step(P, dev(g), M, V, N, dev(touched), B.optim_params(lm_mode=mode), step)
    gp, gm, gv = host(P), moments_rows(host(M)), moments_rows(host(V))
    # FP64 inside: results equal the FP32 rounding of the FP64 oracle to 1 ulp
    for name, a, b in (("params", gp, rp_), ("m", gm, rm), ("v", gv, rv)):
        b32 = b.astype(np.float32)
        ulp = np.abs(np.spacing(b32))
        assert (np.abs(a.astype(np.float64) - b32) <= ulp).all(), name
    assert np.array_equal(gp[:, touched == 0], p[:, touched == 0])
