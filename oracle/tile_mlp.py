"""Oracle of the learned tile-priority model (test infrastructure: only the
tests, the smoke check and the benchmark's CPU leg use it).

The model is not in the paper.  It is a small network that predicts each
tile's reconstruction error from cheap per-(view, tile) features.  It is
trained online on the errors the method itself measures (the tile means of
the error map E of Sec. 3.3), so tile selection can favour tiles it expects
to be poor in views not rendered recently.  The error-map sampler
(Sec. 3.3) stays the reference its ranking is scored against.

Readings (none of this is fixed by the paper):
* features, 32 per (view, tile):
  - 0, 1: tile centre x / W, y / H;
  - 2-17: camera pose features of the camera centre c: d = c / |c| (3),
    |c| / 3 (1), sin(pi d_j), cos(pi d_j), sin(2 pi d_j), cos(2 pi d_j)
    for j = 0, 1, 2 (12);
  - 18: log(1 + pairs listed for the tile);
  - 19: mean of E over the tile's in-image pixels;
  - 20: log(1 + mean of A over the same pixels);
  - 21-31: zero.
* model: y = x_19 + w3 . g(W2^T g(W1^T x + b1) + b2) + b3, g(z) = z Phi(z)
  (GELU, erf form), widths 32 -> 64 -> 64 -> 1: the network predicts the
  change of the tile's error since its error map was written, so with w3
  and b3 at zero (the initial state) it is exactly the error-map predictor
  and training refines it.
* precision: the two 64-wide layers take bfloat16 operands (x, W1, the
  first activation h1, W2; round to nearest even) with sums in float32;
  biases, GELU and the last layer are float32.  The oracle applies the same
  roundings and sums in FP64.
* training: loss = mean over the step's tiles of (y - e)^2, e the tile's
  measured error (feature 19 after the step); the gradient is that of the
  forward above with each rounding taken as the identity; Adam
  (0.9, 0.999, 1e-8, lr 1e-3, bias-corrected) on FP32 master weights.

Parameter vector (FP32, 6337): W1[32][64] at 0, b1 at 2048, W2[64][64] at
2112, b2 at 6208, w3 at 6272, b3 at 6336.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 32
HID = 64
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 2048, 2112, 6208, 6272, 6336
N_PARAMS = 6337
TILE = 16


def bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float64.  The bfloat16 of a float32 keeps its top 16 bits."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz z Phi(z) = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0))) + z * phi


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return dict(W1=p[OFF_W1:OFF_B1].reshape(N_FEAT, HID), b1=p[OFF_B1:OFF_W2],
                W2=p[OFF_W2:OFF_B2].reshape(HID, HID), b2=p[OFF_B2:OFF_W3], w3=p[OFF_W3:OFF_B3],
                b3=p[OFF_B3:OFF_B3 + 1])


def init_params(seed: int) -> np.ndarray:
    """Seeded initial weights: N(0, 1/fan_in) hidden weights, zero biases
    and a zero output layer (the model starts as the error-map predictor)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS, dtype=np.float32)
    p[OFF_W1:OFF_B1] = rng.normal(0.0, 1.0 / math.sqrt(N_FEAT), N_FEAT * HID)
    p[OFF_W2:OFF_B2] = rng.normal(0.0, 1.0 / math.sqrt(HID), HID * HID)
    return p


def pose_features(center) -> np.ndarray:
    c = np.asarray(center, dtype=np.float64)
    r = float(np.linalg.norm(c))
    d = c / r
    f = [d[0], d[1], d[2], r / 3.0]
    for j in range(3):
        f += [math.sin(math.pi * d[j]), math.cos(math.pi * d[j]),
              math.sin(2.0 * math.pi * d[j]), math.cos(2.0 * math.pi * d[j])]
    return np.array(f)


def tile_features(ranges, E, A, height: int, width: int, center) -> np.ndarray:
    """[n_t][32] features of every tile of one view (row-major tile order).

    ranges: [n_t][2] pair ranges; E: half error map as uint16 bits or
    float16 [H][W]; A: uint16 age map [H][W]."""
    TX, TY = (width + TILE - 1) // TILE, (height + TILE - 1) // TILE
    Ef = np.asarray(E)
    Ef = (Ef.view(np.float16) if Ef.dtype != np.float16 else Ef).astype(np.float64)
    Af = np.asarray(A).view(np.uint16).astype(np.float64)
    pose = pose_features(center)
    X = np.zeros((TX * TY, N_FEAT))
    for ty in range(TY):
        for tx in range(TX):
            t = ty * TX + tx
            y0, x0 = ty * TILE, tx * TILE
            e = Ef[y0:y0 + TILE, x0:x0 + TILE]
            a = Af[y0:y0 + TILE, x0:x0 + TILE]
            X[t, 0] = (x0 + 0.5 * TILE) / width
            X[t, 1] = (y0 + 0.5 * TILE) / height
            X[t, 2:18] = pose
            X[t, 18] = math.log1p(float(ranges[t][1]) - float(ranges[t][0]))
            X[t, 19] = e.mean()
            X[t, 20] = math.log1p(a.mean())
    return X


def forward(p, X, rounding: bool = True) -> dict:
    """Predictions y [n] and the intermediate values the backward needs."""
    q = unpack(p)
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    xb, W1b, W2b = rnd(X), rnd(q["W1"]), rnd(q["W2"])
    z1 = xb @ W1b + q["b1"]
    h1 = gelu(z1)
    h1b = rnd(h1)
    z2 = h1b @ W2b + q["b2"]
    h2 = gelu(z2)
    y = X[:, 19] + (h2 @ q["w3"] + q["b3"][0])
    return dict(y=y, z1=z1, h1b=h1b, z2=z2, h2=h2, xb=xb, W2b=W2b)


def loss_grad(p, X, target, rounding: bool = True):
    """Loss mean (y - e)^2 over the rows and its gradient (N_PARAMS,)."""
    f = forward(p, X, rounding)
    q = unpack(p)
    n = f["y"].size
    r = f["y"] - np.asarray(target, dtype=np.float64)
    dy = 2.0 * r / n
    g = np.zeros(N_PARAMS)
    g[OFF_B3] = dy.sum()
    g[OFF_W3:OFF_B3] = f["h2"].T @ dy
    dz2 = np.outer(dy, q["w3"]) * gelu_grad(f["z2"])
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    g[OFF_W2:OFF_B2] = (f["h1b"].T @ dz2).ravel()
    dz1 = (dz2 @ f["W2b"].T) * gelu_grad(f["z1"])
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    g[OFF_W1:OFF_B1] = (f["xb"].T @ dz1).ravel()
    return float((r * r).mean()), g


def adam(p, g, m, v, step: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One bias-corrected Adam step; returns new (p, m, v) in FP64."""
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def kendall_tau(a, b) -> float:
    """Kendall's tau-a of two score vectors (pairs with a tie in either count as 0)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = a.size
    s = 0.0
    for i in range(n - 1):
        s += np.sum(np.sign(a[i + 1:] - a[i]) * np.sign(b[i + 1:] - b[i]))
    return float(2.0 * s / (n * (n - 1)))


def top_k_recall(pred, ref, k: int) -> float:
    """Share of the k highest-``ref`` items among the k highest-``pred`` ones."""
    tp = set(np.argsort(-np.asarray(pred), kind="stable")[:k].tolist())
    tr = set(np.argsort(-np.asarray(ref), kind="stable")[:k].tolist())
    return len(tp & tr) / float(k)
