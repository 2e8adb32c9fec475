"""Depth-prefix lists (the nearest Gaussians first, a continuation for the
tiles where a pixel runs past them) against whole lists: the lists are the
exact depth prefix and rest of the whole lists, and the forward, its
counters, the backward and the density sums come out as with whole lists."""
import math

import numpy as np
import pytest
import torch

import synth
from support import assert_close, scene_c1, scene_scaling

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


def _depth_rank(rect, depth):
    """Rank of every Gaussian with a non-empty rectangle in (depth bits, id)
    order among those Gaussians (the binning puts the others last)."""
    r = rect.astype(np.int64)
    ids = np.nonzero((r[:, 2] > r[:, 0]) & (r[:, 3] > r[:, 1]))[0]
    bits = depth.view(np.uint32)[ids].astype(np.int64)
    order = ids[np.lexsort((ids, bits))]
    rank = np.full(depth.size, -1, dtype=np.int64)
    rank[order] = np.arange(order.size)
    return rank


def _tiles_of(ranges, n_pairs):
    r = ranges.astype(np.int64)
    cnt = r[:, 1] - r[:, 0]
    t = np.repeat(np.arange(r.shape[0]), cnt)
    pos = np.concatenate([np.arange(a, b) for a, b in r if b > a]) if n_pairs else np.zeros(0, np.int64)
    return t, pos


@pytest.mark.parametrize("case", ["scaling_sparse", "scaling_dense", "c1_tile_subset"])
@pytest.mark.parametrize("frac", [0.05, 0.3])
def test_prefix_lists_render_like_whole_lists(B, case, frac):
    from paper_2606_15924_amd.pipeline import StepConfig, ViewBuffers
    if case.startswith("scaling"):
        p, cam = scene_scaling()
    else:
        p, cams = scene_c1()
        cam = cams[1]
    n = p.shape[1]
    W, H = cam.width, cam.height
    rp = B.raster_params()
    dense = case == "scaling_dense"
    n_sel = 64 if case == "c1_tile_subset" else -1
    cfg = StepConfig(rate_permille=250, n_tiles_sel=n_sel)
    vb = ViewBuffers(n, W, H, None if dense else B.tgs_pixels_per_tile(250), n_sel, torch.device("cuda"))
    if not dense:
        totals = torch.zeros(2, dtype=torch.int64, device="cuda")
        E = synth.error_map(H, W, 41)
        A = synth.age_map(H, W, 42)
        vb.sample(dev(E.view(np.int16)), dev(A.view(np.int16)), cfg, 1, 0, totals)
    vb.project(dev(p), B.camera(cam), rp)
    P = vb.P_cap
    g = torch.Generator(device="cuda").manual_seed(5)
    dL = torch.randn((P, 4), generator=g, device="cuda")
    err = torch.rand(P, generator=g, device="cuda")

    def run(prefix):
        cnt = torch.zeros((2, B.COUNTER_SLOTS), dtype=torch.int64, device="cuda")
        if prefix is None:
            vb.bin_sort()
            vb.render_fwd(rp, cnt)
        else:
            vb.bin_sort_prefix(prefix, wait=True)
            vb.render_fwd_two_part(rp, cnt, wait=True)
        vb.dL.copy_(dL)
        vb.err.copy_(err)
        vb.render_bwd(rp, zero=True)
        stats = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
        vb.density(rp, stats)
        return dict(out=host(vb.out).copy(), nc=host(vb.ncontrib).copy(), cnt=host(cnt).sum(axis=1),
                    g2d=host(vb.g2d).copy(), stats=host(stats).copy())

    whole = run(None)
    vals_w, rng_w, np_w = host(vb.vals).copy(), host(vb.ranges).copy(), vb.n_pairs
    m = max(1, int(math.ceil(frac * n)))
    part = run(m)
    # the forward bit for bit, its evaluation and blend counts exactly
    assert np.array_equal(part["out"].view(np.uint32), whole["out"].view(np.uint32))
    assert np.array_equal(part["nc"], whole["nc"])
    assert np.array_equal(part["cnt"], whole["cnt"])
    # the backward and density sums up to the order of the float atomics
    scale = np.abs(whole["g2d"]).max(axis=0, keepdims=True) + 1e-30
    assert np.all(np.abs(part["g2d"] - whole["g2d"]) <= 1e-4 * np.abs(whole["g2d"]) + 1e-5 * scale)
    assert_close(part["stats"], whole["stats"], 1e-4, 1e-6 * (np.abs(whole["stats"]).max() + 1e-30),
                 "density sums")
    # the lists: the first part is the depth prefix of every whole list,
    # the continuation the rest of every marked tile's list
    depth = host(vb.depth)
    rank = _depth_rank(host(vb.rect), depth)
    t_w, _ = _tiles_of(rng_w, np_w)
    vw = vals_w[:np_w].astype(np.int64)
    keep = rank[vw] < m
    n1 = int(host(vb.counts)[0])
    v1, r1 = host(vb.vals)[:n1].astype(np.int64), host(vb.ranges)
    assert np.array_equal(v1, vw[keep])
    t1, _ = _tiles_of(r1, n1)
    assert np.array_equal(t1, t_w[keep])
    marked = host(vb.cont_slot) >= 0
    n_marked = int(host(vb.cont_count)[0])
    assert n_marked == int(marked.sum())
    slots = np.sort(host(vb.cont_list)[:n_marked])
    tiles = np.arange(vb.n_t) if dense else host(vb.valid_tiles)
    assert np.array_equal(np.sort(tiles[slots]), np.nonzero(marked)[0])
    n2 = int(host(vb.counts2)[0])
    v2, r2 = host(vb.vals2)[:n2].astype(np.int64), host(vb.ranges2)
    rest = ~keep & marked[t_w]
    assert np.array_equal(v2, vw[rest])
    t2, _ = _tiles_of(r2, n2)
    assert np.array_equal(t2, t_w[rest])
    assert vb.n_pairs == n1 + n2
    if frac == 0.05 and case.startswith("scaling"):
        assert n1 < 0.5 * np_w          # the prefix is the smaller part of the pairs


@pytest.mark.parametrize("streams", [1, 2])
def test_trainer_prefix_binning_matches_whole_lists(B, streams):
    """Two sparse steps of the rasterizer-scaling scene over two views (the
    first sizing the arrays with host waits, the second queued without),
    the parameters reset to the same values before each: outputs and
    counters bit for bit and the second step's gradient as with whole
    lists; streams: the views' chains on that many streams."""
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer, ViewBuffers
    p, cam = scene_scaling()
    cams = [cam, synth.look_at((2.0, -1.6, 1.4), fx=cam.fx, fy=cam.fy, width=cam.width, height=cam.height)]
    rp = B.raster_params()
    P = dev(synth.perturb(p))
    vb = ViewBuffers(p.shape[1], cam.width, cam.height, None, -1, torch.device("cuda"))
    gts = []
    for c in cams:
        vb.project(P, B.camera(c), rp)
        vb.bin_sort()
        vb.render_fwd(rp)
        gts.append(vb.out[: c.width * c.height, :3].T.reshape(3, c.height, c.width).contiguous())
    del vb
    res = []
    for frac in (None, 0.1):
        cfg = StepConfig(rate_permille=200, fuse_optimizer=False, prefix_fraction=frac, view_streams=streams)
        E = [torch.zeros((c.height, c.width), dtype=torch.int16, device="cuda") for c in cams]
        A = [torch.zeros((c.height, c.width), dtype=torch.int16, device="cuda") for c in cams]
        tr = Trainer(dev(p), cams, gts, cfg, E=E, A=A)
        tr.init_error_maps([0, 1])
        outs = []
        for _ in range(2):
            tr.params.copy_(dev(p))
            used = tr.step([0, 1])
            outs.append([host(vb.out).copy() for vb in used])
        tr.check_counts(wait_all=True)
        res.append((outs, host(tr.grad).copy(), host(tr.counters).sum(axis=1)))
        if frac is not None:
            assert all(vb.two_part for vb in used)
        del tr
    (o0, g0, c0), (o1, g1, c1) = res
    for s0, s1 in zip(o0, o1):
        for a, b in zip(s0, s1):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(c0, c1)
    scale = np.abs(g0).max(axis=1, keepdims=True) + 1e-30
    assert np.all(np.abs(g1 - g0) <= 1e-4 * np.abs(g0) + 1e-5 * scale)
