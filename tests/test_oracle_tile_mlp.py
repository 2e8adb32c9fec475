"""Pins of the tile-priority model's oracle against library routines,
closed forms and finite differences (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import tile_mlp as T


def test_bf16_rounding_equals_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.uniform(-6, 6, 5000),
                        # exact ties between two bfloat16 neighbours, both parities
                        (np.arange(1, 200, dtype=np.float64) * 2 + 1) * 2.0 ** -8,
                        [0.0, -0.0, 1.0, -3.5]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(T.bf16(x), ref)


def test_gelu_identities_and_derivative():
    z = np.linspace(-6, 6, 241)
    # z Phi(z) - (-z) Phi(-z) = z (Phi(z) + Phi(-z) = 1)
    assert np.allclose(T.gelu(z) - T.gelu(-z), z, atol=1e-15, rtol=0)
    assert T.gelu(np.array([0.0]))[0] == 0.0
    assert abs(T.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15   # Phi(1)
    h = 1e-6
    fd = (T.gelu(z + h) - T.gelu(z - h)) / (2 * h)
    assert np.allclose(T.gelu_grad(z), fd, atol=1e-9)


def _problem(n=40, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, T.N_FEAT))
    X[:, 21:] = 0.0
    p = T.init_params(seed).astype(np.float64)
    p[T.OFF_B1:T.OFF_W2] = rng.normal(0, 0.1, T.HID)
    p[T.OFF_B2:T.OFF_W3] = rng.normal(0, 0.1, T.HID)
    p[T.OFF_W3:T.OFF_B3] = rng.normal(0, 0.125, T.HID)   # the initial output layer is zero
    p[T.OFF_B3] = 0.2
    t = rng.uniform(0, 1, n)
    return p, X, t


def test_gradient_equals_finite_differences_without_rounding():
    p, X, t = _problem()
    _, g = T.loss_grad(p, X, t, rounding=False)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(np.arange(T.OFF_W1, T.OFF_B1), 20), rng.choice(np.arange(T.OFF_W2, T.OFF_B2), 20),
                          np.arange(T.OFF_B1, T.OFF_B1 + 5), np.arange(T.OFF_B2, T.OFF_B2 + 5),
                          np.arange(T.OFF_W3, T.OFF_W3 + 5), [T.OFF_B3]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (T.loss_grad(pp, X, t, rounding=False)[0] - T.loss_grad(pm, X, t, rounding=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_forward_of_a_single_unit_closed_form():
    """Only x0 -> unit 0 -> unit 0 -> output, plus the stale error x19:
    y = x19 + w3 g(W2 g(W1 x + b1) + b2) + b3."""
    p = np.zeros(T.N_PARAMS)
    p[T.OFF_W1 + 0 * T.HID + 0] = 0.5
    p[T.OFF_B1] = 0.25
    p[T.OFF_W2 + 0 * T.HID + 0] = 2.0
    p[T.OFF_B2] = -0.5
    p[T.OFF_W3] = 3.0
    p[T.OFF_B3] = 0.125
    X = np.zeros((3, T.N_FEAT))
    X[:, 0] = [0.0, 1.0, -2.0]   # all exact in bfloat16
    X[:, 19] = [0.5, -0.25, 0.0]
    Phi = lambda z: 0.5 * (1 + math.erf(z / math.sqrt(2)))
    for r in range(3):
        h1 = (0.5 * X[r, 0] + 0.25) * Phi(0.5 * X[r, 0] + 0.25)
        h1b = T.bf16(np.array([h1]))[0]
        z2 = 2.0 * h1b - 0.5
        # the other 63 units of each layer give g(0) = 0, and layer 2 sees their 0
        y = X[r, 19] + (3.0 * z2 * Phi(z2) + 0.125)
        assert abs(T.forward(p, X)["y"][r] - y) < 1e-15
    # the initial parameters give the stale error itself
    assert np.array_equal(T.forward(T.init_params(1), X)["y"], X[:, 19])


def test_adam_equals_torch_adam():
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=50)
    g1, g2 = rng.normal(size=50), rng.normal(size=50)
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0, np.zeros(50), np.zeros(50)
    for s, g in enumerate((g1, g2), start=1):
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = T.adam(p, g, m, v, s)
        assert np.allclose(p, w.detach().numpy(), rtol=0, atol=1e-15)


def test_tile_features_brute_force():
    H, W = 40, 37                     # partial tiles at the right and bottom
    TX, TY = 3, 3
    rng = np.random.default_rng(9)
    E = rng.uniform(0, 1, (H, W)).astype(np.float16)
    A = rng.integers(0, 50, (H, W)).astype(np.uint16)
    ranges = np.stack([np.arange(TX * TY) * 10, np.arange(TX * TY) * 10 + np.arange(TX * TY)], axis=1)
    c = np.array([0.0, 0.0, 3.0])
    X = T.tile_features(ranges, E, A, H, W, c)
    for t in range(TX * TY):
        tx, ty = t % TX, t // TX
        es, as_, cnt = [], [], 0
        for y in range(ty * 16, min(H, ty * 16 + 16)):
            for x in range(tx * 16, min(W, tx * 16 + 16)):
                es.append(float(E[y, x]))
                as_.append(float(A[y, x]))
        assert abs(X[t, 19] - sum(es) / len(es)) < 1e-12
        assert abs(X[t, 20] - math.log1p(sum(as_) / len(as_))) < 1e-12
        assert X[t, 18] == math.log1p(t)
        assert X[t, 0] == (tx * 16 + 8) / W and X[t, 1] == (ty * 16 + 8) / H
    # camera on the +z axis at radius 3: d = (0, 0, 1)
    want = [0, 0, 1, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0, -1, 0, 1]
    assert np.allclose(X[0, 2:18], want, atol=1e-15)
    assert not X[:, 21:].any()


def test_ranking_scores_against_scipy():
    from scipy.stats import kendalltau
    rng = np.random.default_rng(11)
    a, b = rng.normal(size=200), rng.normal(size=200)
    assert abs(T.kendall_tau(a, b) - kendalltau(a, b).statistic) < 1e-12
    assert T.kendall_tau(a, a) == 1.0 and T.kendall_tau(a, -a) == -1.0
    assert T.top_k_recall(a, a, 10) == 1.0
