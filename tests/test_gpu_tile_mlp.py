"""GPU parity of the learned tile-priority model against its oracle: the
tile features, the bfloat16-MFMA forward and the training step (gradient
and Adam update), plus a property of online training."""
import numpy as np
import pytest
import torch

import synth
from oracle import binning, project
from oracle import tile_mlp as T
from oracle.params import RasterParams

from support import small_scene

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


def _params(seed):
    rng = np.random.default_rng(seed)
    p = T.init_params(seed)
    p[T.OFF_W3:T.OFF_B3] = rng.normal(0, 1.0 / 8.0, T.HID)
    p[T.OFF_B1:T.OFF_W2] = rng.normal(0, 0.2, T.HID)
    p[T.OFF_B2:T.OFF_W3] = rng.normal(0, 0.2, T.HID)
    p[T.OFF_B3] = 0.1
    return p.astype(np.float32)


def _features(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, T.N_FEAT), np.float32)
    X[:, :21] = rng.normal(0, 1, (n, 21))
    return X


def test_tile_features_parity(B):
    p, cam = small_scene(n=2000, seed=41)
    pr = project.project(p, cam, RasterParams())
    _, _, ranges = binning.bin_and_sort(pr)
    H, W = cam.height, cam.width
    E = synth.error_map(H, W, 61)
    A = synth.age_map(H, W, 62)
    ref = T.tile_features(ranges, E, A, H, W, project.camera_center(cam))
    X = torch.empty((ranges.shape[0], 32), dtype=torch.float32, device="cuda")
    B.tgs_tile_features(dev(ranges.astype(np.uint32)), dev(E.view(np.int16)), dev(A.view(np.int16)), H, W,
                        B.camera(cam), X)
    got = host(X).astype(np.float64)
    assert np.allclose(got[:, :18], ref[:, :18], rtol=0, atol=2e-7)
    assert np.allclose(got[:, 18:21], ref[:, 18:21], rtol=1e-6, atol=1e-7)
    assert not got[:, 21:].any()


def _mlp_bounds(p, X):
    """Per-row error scales of the two hidden layers and the output."""
    q = T.unpack(p)
    f = T.forward(p, X)
    s1 = np.abs(f["xb"]) @ np.abs(T.bf16(q["W1"])) + np.abs(q["b1"])
    s2 = np.abs(f["h1b"]) @ np.abs(f["W2b"]) + np.abs(q["b2"])
    sy = np.abs(T.gelu(f["z2"])) @ np.abs(q["w3"]) + abs(q["b3"][0]) + np.abs(X[:, 19])
    return f, s1, s2, sy


@pytest.mark.parametrize("n", [37, 1000, 4293])
def test_tile_mlp_fwd_parity(B, n):
    p = _params(5)
    X = _features(n, 6)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    act = torch.empty((n, 128), dtype=torch.float32, device="cuda")
    B.tgs_tile_mlp_fwd(dev(p), dev(X), n, y, act)
    f, s1, s2, sy = _mlp_bounds(p, X)
    a = host(act).astype(np.float64)
    # layer 1: identical bfloat16 operands, float32 against FP64 sums
    assert (np.abs(a[:, :64] - f["z1"]) <= 1e-5 * s1).all()
    # layer 2 and the output: an FP32-vs-FP64 difference in gelu(z1) can move
    # a bfloat16 rounding of h1 by one step (2^-8 relative) in a few elements
    d2 = np.abs(a[:, 64:] - f["z2"])
    assert (d2 <= 1e-5 * s2).mean() > 0.99
    assert (d2 <= 2.0 ** -6 * s2).all()
    dy = np.abs(host(y) - f["y"])
    assert (dy <= 1e-5 * sy).mean() > 0.99
    assert (dy <= 2.0 ** -6 * sy).all()


def test_tile_mlp_train_step_parity(B):
    n = 4293
    p = _params(8)
    X = _features(n, 9)
    t = np.random.default_rng(10).uniform(0, 1, n).astype(np.float32)
    P, M, V = dev(p), torch.zeros(T.N_PARAMS, device="cuda"), torch.zeros(T.N_PARAMS, device="cuda")
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    act = torch.empty((n, 128), dtype=torch.float32, device="cuda")
    ws = torch.empty(B.tgs_tile_mlp_workspace_size(n), dtype=torch.uint8, device="cuda")
    G = torch.empty(T.N_PARAMS, dtype=torch.float32, device="cuda")
    Xd, td = dev(X), dev(t)
    B.tgs_tile_mlp_fwd(P, Xd, n, y, act)
    B.tgs_tile_mlp_train_step(P, M, V, Xd, act, y, td, n, 1, 1e-3, ws, grad=G)
    _, g_ref = T.loss_grad(p, X, t)
    g = host(G).astype(np.float64)
    # gradient per parameter group within 1e-4 of the group's largest entry
    # plus 1e-3 relative (the few flipped bfloat16 roundings of h1 above)
    for lo, hi in ((T.OFF_W1, T.OFF_B1), (T.OFF_B1, T.OFF_W2), (T.OFF_W2, T.OFF_B2), (T.OFF_B2, T.OFF_W3),
                   (T.OFF_W3, T.OFF_B3), (T.OFF_B3, T.N_PARAMS)):
        scale = np.abs(g_ref[lo:hi]).max()
        assert (np.abs(g[lo:hi] - g_ref[lo:hi]) <= 1e-3 * np.abs(g_ref[lo:hi]) + 1e-4 * scale).all(), (lo, hi)
    # Adam step on the GPU's own gradient (FP64 inside, rounded to float32;
    # the learning rate is the float32 the kernel receives)
    p1, m1, v1 = T.adam(p, g, np.zeros(T.N_PARAMS), np.zeros(T.N_PARAMS), 1, lr=float(np.float32(1e-3)))
    for name, a, b in (("params", host(P), p1), ("m", host(M), m1), ("v", host(V), v1)):
        b32 = b.astype(np.float32)
        assert (np.abs(a.astype(np.float64) - b32) <= np.abs(np.spacing(b32))).all(), name


def test_online_training_fits_a_tile_error_field(B):
    """Targets that move away from the stale error (feature 19) by a smooth
    function of the features: 200 Adam steps on the GPU cut the mean squared
    error several-fold (the model starts as the error-map predictor)."""
    n = 4293
    X = _features(n, 12)
    t = (X[:, 19] + 0.2 * np.tanh(X[:, 0] - 0.5 * X[:, 19]) + 0.1 * np.sin(X[:, 18])).astype(np.float32)
    P = dev(T.init_params(13))
    M, V = torch.zeros(T.N_PARAMS, device="cuda"), torch.zeros(T.N_PARAMS, device="cuda")
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    act = torch.empty((n, 128), dtype=torch.float32, device="cuda")
    ws = torch.empty(B.tgs_tile_mlp_workspace_size(n), dtype=torch.uint8, device="cuda")
    Xd, td = dev(X), dev(t)
    losses = []
    for step in range(1, 201):
        B.tgs_tile_mlp_fwd(P, Xd, n, y, act)
        if step in (1, 200):
            losses.append(float(((y - td) ** 2).mean()))
        B.tgs_tile_mlp_train_step(P, M, V, Xd, act, y, td, n, step, 3e-3, ws)
    assert np.isfinite(losses).all() and losses[1] < 0.2 * losses[0], losses


def test_trainer_tile_pass_uses_the_learned_priority(B):
    """A training step with the learned tile priority: the tiles drawn are
    those the oracle sampler draws from the model's predictions; at the first
    step the zero output layer makes them the tile means of the error map;
    the step trains the model."""
    from oracle import sampler
    from oracle.params import SampleParams
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer, init_tile_params
    from support import scene_c1
    p, cams = scene_c1()
    H, W = cams[0].height, cams[0].width
    gts = [dev(synth.image(H, W, 70 + k)) for k in range(len(cams))]
    E = [synth.error_map(H, W, 80 + k) for k in range(len(cams))]
    A = [synth.age_map(H, W, 90 + k) for k in range(len(cams))]
    Eg = [dev(e.view(np.int16)) for e in E]
    Ag = [dev(a.view(np.int16)) for a in A]
    cfg = StepConfig(rate_permille=250, n_tiles_sel=64, learned_tiles=True)
    tr = Trainer(dev(p), cams, gts, cfg, E=Eg, A=Ag)
    used = tr.step([2])
    y = host(tr.tiles.slot(0)["y"])
    ref = sampler.sample_view(E[2], A[2], SampleParams(n_pix=64, n_tiles_sel=64), cfg.seed, 1, 2, tile_pred=y)
    assert np.array_equal(host(used[0].valid_tiles), ref["valid_tiles"])
    X = T.tile_features(np.zeros((y.size, 2)), E[2], A[2], H, W, project.camera_center(cams[2]))
    assert np.allclose(y, X[:, 19], rtol=1e-6, atol=1e-7)
    assert not torch.equal(tr.tiles.params.cpu(), init_tile_params(cfg.tile_seed))
    assert np.array_equal(host(tr.tiles.ranges[2]), host(used[0].ranges))
