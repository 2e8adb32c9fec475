"""GPU parity of the density-control statistics (Sec. 3.8): the
back-projection of per-pixel errors, weights and distances onto the
Gaussians (Eq. gauss_err_accum) and the difficulty score (Eq. gauss_score),
the percentile thresholds (an exact k-th largest, bit for bit), densify and
prune, and the screen-space statistics against the oracle, plus the
telescoping property, the selection counts and training on after a
topology change at the full training size.

Tolerances: every summed term is non-negative, so a per-Gaussian sum carries
the relative error of its terms; a term's weight T alpha is a product of up
to a few hundred FP32 factors (1e-4 relative).  The distance sqrt(d^T Q d)
near a splat centre is the square root of a small FP32 difference, so D
also gets an absolute 1e-3 per unit of weight."""
import numpy as np
import pytest
import torch

import synth
from oracle import binning, density, project, render, sampler
from oracle.params import RasterParams, SampleParams

from support import moments_gaussian_major, moments_rows, assert_close, scene_c1, small_scene, splat_as_oracle, splat_record

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


def _case(case):
    if case == "c1_sparse64":
        p, cams = scene_c1()
        cam = cams[2]
        E = synth.error_map(cam.height, cam.width, 141)
        A = synth.age_map(cam.height, cam.width, 142)
        s = sampler.sample_view(E, A, SampleParams(n_pix=64, n_tiles_sel=64), 3, 1, 2)
    elif case in ("ragged_sparse25", "ragged_sparse128"):
        n_pix = 25 if case.endswith("25") else 128
        p, cam = small_scene(n=2500, seed=17)
        E = synth.error_map(cam.height, cam.width, 143)
        A = synth.age_map(cam.height, cam.width, 144)
        s = sampler.sample_view(E, A, SampleParams(n_pix=n_pix), 3, 1, 0)
    else:
        p, cam = small_scene(n=2500, seed=18)
        s = None
    return p, cam, s


@pytest.mark.parametrize("case", ["c1_sparse64", "ragged_sparse25", "ragged_sparse128", "dense"])
def test_density_accumulate_parity(B, case):
    p, cam, s = _case(case)
    rp = RasterParams(bg=(0.1, 0.2, 0.3))
    pr = project.project(p, cam, rp)
    rec = splat_record(pr)
    q = splat_as_oracle(pr, rec)
    _, sv, ranges = binning.bin_and_sort(pr, None if s is None else s["valid_tiles"])
    if s is None:
        xs, ys = render.dense_pixels(cam.width, cam.height)
    else:
        xs, ys, _ = sampler.sample_coords(s, cam.width, cam.height)
    ref = render.render_pixels(q, sv, ranges, xs, ys, rp)
    err = np.random.default_rng(5).uniform(0.0, 2.0, xs.size).astype(np.float32)
    ok = ~ref["flag"]
    assert ok.mean() > 0.99
    # guard-band pixels: no contributors on the GPU side, left out of the oracle's sums
    nc = np.where(ok, ref["n_contrib"], 0).astype(np.int32)
    want = density.accumulate(q, sv, ranges, xs[ok], ys[ok], err[ok], rp)
    n = p.shape[1]
    TX, TY = pr["TX"], pr["TY"]
    if s is None:
        idx = ys * cam.width + xs
        nc_full = np.zeros(cam.width * cam.height, np.int32)
        e_full = np.zeros(cam.width * cam.height, np.float32)
        nc_full[idx], e_full[idx] = nc, err
        nc, err = nc_full, e_full
        vt = off = pix = None
        n_st, mpt = TX * TY, 256
    else:
        vt, off, pix = dev(s["valid_tiles"]), dev(s["tile_off"]), dev(s["pix"])
        n_st, mpt = s["valid_tiles"].size, max(int(np.diff(s["tile_off"]).max()), 1)
    stats = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    args = (dev(rec), dev(sv.view(np.int32)), dev(ranges.astype(np.int32)), TX, TY, cam.width, cam.height,
            vt, off, pix, n_st, mpt, B.raster_params(bg=rp.bg), dev(nc), dev(err), n, stats)
    B.tgs_density_accumulate(*args)
    got = host(stats)[:, :3].T.astype(np.float64)
    assert (want[1] > 0).sum() > 200
    assert_close(got[0], want[0], 1e-4, 1e-9, "E")
    assert_close(got[1], want[1], 1e-4, 1e-9, "W")
    assert_close(got[2], want[2], 1e-4, 1e-3 * want[1] + 1e-9, "D")
    # a second call adds the same sums again
    B.tgs_density_accumulate(*args)
    assert_close(host(stats)[:, :3].T.astype(np.float64), 2 * want, 1e-4, 2e-3 * want[1] + 2e-9, "twice")


def test_density_score_parity_and_errors(B):
    rng = np.random.default_rng(9)
    n = 100003
    W = rng.uniform(0, 3, n) * (rng.uniform(0, 1, n) < 0.8)      # a fifth never composited
    st = np.stack([W * rng.uniform(0, 2, n), W, W * rng.uniform(0, 3.3, n)]).astype(np.float32)
    want = density.score(st.astype(np.float64), 0.7, 0.35, eps=float(np.float32(1e-8)))
    st = np.ascontiguousarray(np.concatenate([st.T, np.full((n, 1), np.nan, np.float32)], axis=1))  # [n][4]
    e, d, sc = (torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))
    B.tgs_density_score(dev(st), n, 0.7, 0.35, 1e-8, e, d, sc)
    for name, g in (("e", e), ("d", d), ("s", sc)):
        assert_close(host(g), want[name], 1e-6, 0.0, name)
    assert not host(sc)[W == 0].any()
    # without the optional outputs
    s2 = torch.empty(n, dtype=torch.float32, device="cuda")
    B.tgs_density_score(dev(st), n, 0.7, 0.35, 1e-8, None, None, s2)
    assert torch.equal(s2, sc)
    with pytest.raises(RuntimeError, match="rho"):
        B.tgs_density_score(dev(st), n, 0.7, 1.5, 1e-8, None, None, s2)
    with pytest.raises(RuntimeError, match="eps"):
        B.tgs_density_score(dev(st), n, 0.7, 0.5, 0.0, None, None, s2)
    B.tgs_density_score(dev(st), 0, 0.7, 0.5, 1e-8, None, None, s2)   # empty: nothing to do


def test_density_accumulate_without_tiles_leaves_stats(B):
    p, cam = small_scene(n=300, seed=4)
    pr = project.project(p, cam, RasterParams())
    rec = splat_record(pr)
    _, sv, ranges = binning.bin_and_sort(pr)
    stats = torch.full((300, 4), 0.5, dtype=torch.float32, device="cuda")
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.tgs_density_accumulate(dev(rec), dev(sv.view(np.int32)), dev(ranges.astype(np.int32)), pr["TX"], pr["TY"],
                             cam.width, cam.height, z, z, z.to(torch.uint8), 0, 64, B.raster_params(),
                             z, z.float(), 300, stats)
    assert (host(stats) == 0.5).all()


def test_trainer_density_sums_telescope_at_full_size(B):
    """300k Gaussians, one 1296x840 view at 25%: summed over the Gaussians,
    W equals the sum over the samples of 1 - T_final and E the sum of
    e (1 - T_final), both read from the step's own forward outputs."""
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    from support import scene_scaling
    p, cam = scene_scaling()
    H, W = cam.height, cam.width
    gt = dev(synth.image(H, W, 171))
    E = [dev(synth.error_map(H, W, 172).view(np.int16))]
    A = [dev(synth.age_map(H, W, 173).view(np.int16))]
    tr = Trainer(dev(p), [cam], [gt], StepConfig(rate_permille=250, density_stats=True), E=E, A=A)
    used = tr.step([0])
    vb = used[0]
    P = int(host(vb.tile_off)[-1])
    T = host(vb.out)[:P, 3].astype(np.float64)
    err = host(vb.err)[:P].astype(np.float64)
    st = host(tr.dstats)[:, :3].T.astype(np.float64)
    assert P > 200000
    assert abs(st[1].sum() - (1 - T).sum()) <= 1e-4 * (1 - T).sum()
    assert abs(st[0].sum() - (err * (1 - T)).sum()) <= 1e-4 * (err * (1 - T)).sum()
    assert (st >= 0).all() and (st[2][st[1] == 0] == 0).all()
    e, d, sc = tr.density_scores(0.5, 0.25)
    seen = st[1] > 1e-3
    dg = host(d).astype(np.float64)
    assert (dg[seen] <= np.sqrt(2 * np.log(255.0)) * (1 + 1e-4)).all()
    assert np.allclose(host(sc), host(e) + 0.375 * dg, rtol=1e-6, atol=0)
    tr.reset_density()
    assert not tr.dstats.any()


@pytest.mark.parametrize("n", [1, 1000, 300000, (1 << 20) + 7])
def test_select_kth_largest_bit_exact(B, n):
    rng = np.random.default_rng(n)
    v = rng.exponential(1.0, n).astype(np.float32)
    if n > 10:
        v[rng.integers(0, n, n // 5)] = 0.0                       # ties at zero
        v[rng.integers(0, n, n // 10)] = np.float32(0.75)        # ties inside
        v[rng.integers(0, n, n // 20)] = -rng.exponential(1.0, n // 20).astype(np.float32)
        v[:2] = [np.inf, -np.inf]
    V = dev(v)
    ws = torch.empty(B.tgs_select_workspace_size(), dtype=torch.uint8, device="cuda")
    out = torch.empty(1, dtype=torch.float32, device="cuda")
    mask = torch.empty(n, dtype=torch.uint8, device="cuda")
    ks = sorted(k for k in {1, 2, n // 3 + 1, n // 2, n - 1, n} if 1 <= k <= n)
    for k in ks:
        B.tgs_select_kth_largest(V, n, k, out, ws)
        t = density.kth_largest(v, k)
        got = host(out)[0]
        assert np.float32(got).view(np.uint32) == np.float32(t).view(np.uint32), (k, got, t)
        B.tgs_threshold_mask(V, n, out, mask)
        assert np.array_equal(host(mask).astype(bool), v >= t), k
    with pytest.raises(RuntimeError, match="k"):
        B.tgs_select_kth_largest(V, n, n + 1, out, ws)
    with pytest.raises(RuntimeError, match="k"):
        B.tgs_select_kth_largest(V, n, 0, out, ws)


def test_trainer_density_selection_at_full_size(B):
    """Two steps of sparse training at 300k Gaussians, then the percentile
    selections: each mask holds at least k Gaussians and everything above its
    threshold, and fewer than k lie strictly above it."""
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    from support import scene_scaling
    p, cam = scene_scaling()
    H, W = cam.height, cam.width
    gt = dev(synth.image(H, W, 181))
    E = [dev(synth.error_map(H, W, 182).view(np.int16))]
    A = [dev(synth.age_map(H, W, 183).view(np.int16))]
    tr = Trainer(dev(p), [cam], [gt], StepConfig(rate_permille=250, density_stats=True), E=E, A=A)
    tr.step([0])
    tr.step([0])
    dm, km, thr, (_, _, sc) = tr.density_select(0.5, 0.3, eta_topk=0.95, eta_final=0.85)
    s = host(sc)
    t = host(thr)
    for mask, k, th in ((host(dm), 15000, t[0]), (host(km), 255000, t[1])):
        m = mask.astype(bool)
        assert np.array_equal(m, s >= th)
        assert (s > th).sum() < k <= m.sum()
    # about 24k Gaussians are composited in two steps of one view: the
    # densification threshold lies among them, the keep threshold at the
    # zero scores of the rest (all kept)
    assert (s > 0).sum() > 15000 and t[0] > 0
    assert t[1] == 0 and host(km).all()


@pytest.mark.parametrize("mode", ["sparse64", "sparse128", "dense"])
def test_density_accumulate_chunked_equals_single(B, mode):
    """Deep lists (faint Gaussians, so most pixels reach the last chunk): the
    walk split into (tile, chunk) workgroups from the forward's state record
    gives the sums of the single-workgroup walk (same per-pixel arithmetic,
    another order of the float atomics)."""
    p, cam = small_scene(n=4000, seed=12)
    p = np.array(p)
    p[10] = -3.5                              # opacity logit: ~3% per Gaussian
    rp = RasterParams()
    pr = project.project(p, cam, rp)
    rec = splat_record(pr)
    _, sv, ranges = binning.bin_and_sort(pr)
    TX, TY = pr["TX"], pr["TY"]
    if mode == "dense":
        vt = off = pix = None
        n_st, mpt, P = TX * TY, 256, cam.width * cam.height
    else:
        mpt = 64 if mode == "sparse64" else 128
        E = synth.error_map(cam.height, cam.width, 61)
        A = synth.age_map(cam.height, cam.width, 62)
        s = sampler.sample_view(E, A, SampleParams(n_pix=mpt), 3, 1, 0)
        vt, off, pix = dev(s["valid_tiles"]), dev(s["tile_off"]), dev(s["pix"])
        n_st, P = s["valid_tiles"].size, int(s["tile_off"][-1])
    splat, V, R = dev(rec), dev(sv.view(np.int32)), dev(ranges.astype(np.int32))
    brp = B.raster_params()
    out = torch.empty((P, 4), dtype=torch.float32, device="cuda")
    nc = torch.empty(P, dtype=torch.int32, device="cuda")
    state = torch.zeros(B.tgs_render_state_size(n_st, mpt) // 4, dtype=torch.float32, device="cuda")
    B.tgs_render_fwd(splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, mpt, brp, out, nc, None, state)
    assert (host(nc) > (B.RENDER_CHUNKS - 1) * B.RENDER_CHUNK_LEN).mean() > 0.1   # the last chunk has work
    err = dev(np.random.default_rng(6).uniform(0, 2, P).astype(np.float32))
    n = p.shape[1]
    S1 = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    S2 = torch.zeros_like(S1)
    args = (splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, mpt, brp, nc, err, n)
    B.tgs_density_accumulate(*args, S1)
    B.tgs_density_accumulate(*args, S2, state=state)
    s1, s2 = host(S1)[:, :3].T.astype(np.float64), host(S2)[:, :3].T.astype(np.float64)
    assert (s1[1] > 0).sum() > 1000
    assert_close(s2, s1, 1e-5, 1e-6 * s1.max(axis=1, keepdims=True), "chunked vs single")
    assert not host(S2)[:, 3].any()                  # the fourth entry of a slot is untouched


@pytest.mark.parametrize("case,chunked", [("c1_sparse64", True), ("ragged_sparse25", False),
                                          ("ragged_sparse128", True), ("dense", True)])
def test_render_bwd_density_parity(B, case, chunked):
    """The backward with the density sums fused in: its sums match the oracle
    as the standalone kernel's do, and its gradient matches tgs_render_bwd."""
    p, cam, s = _case(case)
    rp = RasterParams(bg=(0.1, 0.2, 0.3))
    pr = project.project(p, cam, rp)
    rec = splat_record(pr)
    q = splat_as_oracle(pr, rec)
    _, sv, ranges = binning.bin_and_sort(pr, None if s is None else s["valid_tiles"])
    if s is None:
        xs, ys = render.dense_pixels(cam.width, cam.height)
    else:
        xs, ys, _ = sampler.sample_coords(s, cam.width, cam.height)
    ref = render.render_pixels(q, sv, ranges, xs, ys, rp)
    ok = ~ref["flag"]
    err = np.random.default_rng(7).uniform(0.0, 2.0, xs.size).astype(np.float32)
    want = density.accumulate(q, sv, ranges, xs[ok], ys[ok], err[ok], rp)
    n = p.shape[1]
    TX, TY = pr["TX"], pr["TY"]
    P = xs.size
    brp = B.raster_params(bg=rp.bg)
    splat, V, R = dev(rec), dev(sv.view(np.int32)), dev(ranges.astype(np.int32))
    if s is None:
        vt = off = pix = None
        n_st, mpt, Pbuf = TX * TY, 256, cam.width * cam.height
        idx = ys * cam.width + xs
    else:
        vt, off, pix = dev(s["valid_tiles"]), dev(s["tile_off"]), dev(s["pix"])
        n_st, mpt, Pbuf = s["valid_tiles"].size, max(int(np.diff(s["tile_off"]).max()), 1), P
        idx = np.arange(P)
    # forward outputs from the GPU forward (its state record for the chunked walk);
    # guard-band pixels get no contributors and drop out of the oracle's sums
    out = torch.empty((Pbuf, 4), dtype=torch.float32, device="cuda")
    nc = torch.empty(Pbuf, dtype=torch.int32, device="cuda")
    state = None
    if chunked:
        state = torch.zeros(B.tgs_render_state_size(n_st, mpt) // 4, dtype=torch.float32, device="cuda")
    B.tgs_render_fwd(splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, mpt, brp, out, nc, None, state)
    nch = host(nc)
    assert np.array_equal(nch[idx][ok], ref["n_contrib"][ok])
    nch[idx[~ok]] = 0
    e_full = np.zeros(Pbuf, np.float32)
    e_full[idx] = err
    dl = torch.from_numpy(np.random.default_rng(8).normal(size=(Pbuf, 4)).astype(np.float32) * 1e-3).cuda()
    G1 = torch.zeros((n, 9), dtype=torch.float32, device="cuda")
    G2 = torch.zeros_like(G1)
    S = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    args = (splat, V, R, TX, TY, cam.width, cam.height, vt, off, pix, n_st, mpt, brp, out, dev(nch), dl)
    B.tgs_render_bwd(*args, G1, state)
    B.tgs_render_bwd_density(*args, G2, dev(e_full), n, S, state=state)
    got = host(S)[:, :3].T.astype(np.float64)
    assert (want[1] > 0).sum() > 200
    assert_close(got[0], want[0], 1e-4, 1e-9, "E")
    assert_close(got[1], want[1], 1e-4, 1e-9, "W")
    assert_close(got[2], want[2], 1e-4, 1e-3 * want[1] + 1e-9, "D")
    g1, g2 = host(G1), host(G2)
    assert_close(g2, g1, 1e-5, 1e-6 * (np.abs(g1).max(axis=0) + 1e-12), "g2d fused vs plain")
    # the absolute statistic: per-pixel centre-gradient norms in NDC units;
    # each term carries the error of its pixel's gradient (1e-4 relative plus
    # 16 FP32 ulps of the oracle's error scale of the two centre fields)
    sx, sy = cam.width / 2, cam.height / 2
    _, gabs, cabs = render.render_pixels_bwd(q, sv, ranges, xs[ok], ys[ok], host(dl)[idx[ok], :3], rp,
                                             with_abs=True, centre_abs_scale=(sx, sy))
    scale = np.hypot(sx * gabs[0], sy * gabs[1])
    assert (cabs > 0).sum() > 200
    assert_close(host(S)[:, 3].astype(np.float64), cabs, 1e-4, 16 * 2.0 ** -23 * scale + 1e-12, "abs grad")


@pytest.mark.parametrize("n", [1, 777, 20011])
def test_densify_and_prune_parity(B, n):
    rng = np.random.default_rng(n + 3)
    p = synth.gaussians(n, 31)
    p[6:10] *= rng.uniform(0.5, 2.0, n).astype(np.float32)          # unnormalised quaternions
    m = rng.normal(size=(59, n)).astype(np.float32)
    v = rng.uniform(0, 1, (59, n)).astype(np.float32)
    keep = (rng.uniform(0, 1, n) < 0.8).astype(np.uint8)
    dens = (rng.uniform(0, 1, n) < 0.3).astype(np.uint8)
    if n == 1:
        keep[:], dens[:] = 1, 1
    z = rng.normal(size=(n, 3)).astype(np.float32)
    log_split = float(np.float32(np.median(p[3:6].max(axis=0))))
    want = density.apply_topology(p, m, v, keep, dens, z, log_split)
    ws = torch.empty(B.tgs_density_topology_workspace_size(n), dtype=torch.uint8, device="cuda")
    nk, nn = B.tgs_density_topology_count(dev(keep), dev(dens), n, ws)
    assert (nk, nn) == (want["n_keep"], want["n_new"])
    n_out = nk + nn
    po = torch.full((59, n_out), np.nan, dtype=torch.float32, device="cuda")
    mo, vo = (torch.full((n_out, B.MOMENT_STRIDE), np.nan, dtype=torch.float32, device="cuda") for _ in range(2))
    B.tgs_density_topology_apply(dev(p), dev(moments_gaussian_major(m)), dev(moments_gaussian_major(v)), n, dev(z),
                                 log_split, ws, po, mo, vo, n_out)
    got, gm, gv = host(po), moments_rows(host(mo)), moments_rows(host(vo))
    ref = want["params"]
    # rows copied as they are, and the moments: bit for bit
    assert np.array_equal(got[6:], ref[6:].astype(np.float32))
    assert np.array_equal(gm, want["m"].astype(np.float32)) and np.array_equal(gv, want["v"].astype(np.float32))
    # split means and log-scales: FP32 arithmetic against FP64
    assert_close(got[3:6], ref[3:6], 0.0, 1e-6, "log-scales")
    o_scale = np.abs(ref[0:3]) + np.exp(ref[3:6].max(axis=0)) * 1.6 * 4.0
    assert_close(got[0:3], ref[0:3], 0.0, 1e-6 * o_scale, "means")
    if n > 1:
        assert want["split"].sum() > 10 and (dens & keep & ~want["split"]).sum() > 10


def test_trainer_densify_and_prune_then_step(B):
    """Select, densify and prune at 300k Gaussians, then train on: the count
    follows the selections and the next step runs on the new Gaussians."""
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    from support import scene_scaling
    p, cam = scene_scaling()
    H, W = cam.height, cam.width
    gt = dev(synth.image(H, W, 191))
    E = [dev(synth.error_map(H, W, 192).view(np.int16))]
    A = [dev(synth.age_map(H, W, 193).view(np.int16))]
    tr = Trainer(dev(p), [cam], [gt], StepConfig(rate_permille=250, density_stats=True), E=E, A=A)
    tr.step([0])
    dm, km, thr, _ = tr.density_select(0.5, 0.3, eta_topk=0.95, eta_final=0.85)
    # prune a random fifth of the Gaussians the score would keep
    keep = km * (torch.rand(tr.n, device="cuda") > 0.2).to(torch.uint8)
    n_keep, n_new = int(keep.sum()), int((keep * dm).sum())
    z = torch.randn((tr.n, 3), device="cuda")
    n_out = tr.densify_and_prune(dm, keep, z, float(np.log(0.02)))
    assert n_out == n_keep + n_new == tr.n and tr.params.shape == (59, n_out)
    used = tr.step([0])
    assert torch.isfinite(tr.params).all()
    assert used[0].n == n_out and tr.dstats.shape == (n_out, 4) and float(tr.dstats[:, 1].sum()) > 0


def test_grad_screen_statistics_parity(B):
    rng = np.random.default_rng(21)
    n = 50021
    acc = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    want = np.zeros((n, 4))
    for view in range(3):
        g = (rng.normal(size=(n, 9)) * 10.0 ** rng.uniform(-6, 0, (n, 1))).astype(np.float32)
        r = np.where(rng.uniform(0, 1, n) < 0.6, rng.integers(1, 200, n), 0).astype(np.int32)
        B.tgs_grad_screen_accumulate(dev(g), dev(r), n, 1296, 840, acc)
        want = density.grad_screen_accumulate(want, g, r, 1296, 840)
    got = host(acc).astype(np.float64)
    assert_close(got[:, 0], want[:, 0], 1e-6, 0.0, "norm sum")
    assert np.array_equal(got[:, 1:3], want[:, 1:3]) and not got[:, 3].any()
    mean = torch.empty(n, dtype=torch.float32, device="cuda")
    B.tgs_grad_screen_mean(acc, n, mean)
    assert_close(host(mean), density.grad_screen_mean(want), 2e-6, 0.0, "mean")


def test_trainer_grad_screen_statistics(B):
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    p, cams = scene_c1()
    H, W = cams[0].height, cams[0].width
    gts = [dev(synth.image(H, W, 200 + k)) for k in range(len(cams))]
    E = [dev(synth.error_map(H, W, 210 + k).view(np.int16)) for k in range(len(cams))]
    A = [dev(synth.age_map(H, W, 220 + k).view(np.int16)) for k in range(len(cams))]
    tr = Trainer(dev(p), cams, gts, StepConfig(rate_permille=250, density_stats=True), E=E, A=A)
    used = tr.step([0, 1, 2])
    vis = sum((host(vb.radius) > 0).astype(np.int64) for vb in used)
    gs = host(tr.gstats)
    assert np.array_equal(gs[:, 1], vis) and vis.max() == 3
    assert (gs[:, 0] >= 0).all() and (gs[:, 0][vis == 0] == 0).all() and gs[:, 0].max() > 0
    m = host(tr.grad_screen_mean())
    assert np.isfinite(m).all() and (m[vis == 0] == 0).all()
    tr.reset_density()
    assert not tr.gstats.any()


@pytest.mark.parametrize("prune", [True, False])
def test_density_masks_bit_exact(B, prune):
    """The fused selection kernel against the oracle's gated percentile
    selection, on the same FP32 statistics (scores with ties and zeros,
    Gaussians never projected, means on both sides of the thresholds)."""
    rng = np.random.default_rng(31 + prune)
    n = 200003
    sc = rng.exponential(1.0, n).astype(np.float32)
    sc[rng.integers(0, n, n // 5)] = 0.0
    sc[rng.integers(0, n, n // 10)] = np.float32(0.5)
    views = rng.integers(0, 4, n).astype(np.float32)
    gacc = np.zeros((n, 4), np.float32)
    gacc[:, 1] = views
    gacc[:, 0] = (views * rng.exponential(2e-4, n)).astype(np.float32)
    dst = np.zeros((n, 4), np.float32)
    dst[:, 3] = (views * rng.exponential(4e-4, n)).astype(np.float32)
    eta_topk, eta_final = 0.9, 0.8
    want_gate = density.gradient_gate(gacc, dst[:, 3], 2e-4, 4e-4)
    assert 0.2 < want_gate.mean() < 0.8
    want = density.select_masks(sc, eta_topk, eta_final, gate=want_gate, prune=prune)
    thr = dev(np.array([want["thr_densify"], want["thr_keep"]], np.float32))
    dm = torch.empty(n, dtype=torch.uint8, device="cuda")
    km = torch.empty(n, dtype=torch.uint8, device="cuda")
    B.tgs_density_masks(dev(sc), dev(gacc), dev(dst), n, thr, 2e-4, 4e-4, prune, dm, km)
    assert np.array_equal(host(km).astype(bool), want["keep"])
    assert np.array_equal(host(dm).astype(bool), want["densify"])
    assert want["densify"].sum() > 1000
    # without the absolute statistic only tau_grad gates
    B.tgs_density_masks(dev(sc), dev(gacc), None, n, thr, 2e-4, 4e-4, prune, dm, km)
    g2 = density.gradient_gate(gacc, np.zeros(n), 2e-4, np.inf)
    want2 = density.select_masks(sc, eta_topk, eta_final, gate=g2, prune=prune)
    assert np.array_equal(host(dm).astype(bool), want2["densify"])
