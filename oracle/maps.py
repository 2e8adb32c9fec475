"""Persistent per-pixel error and age maps (Sec. 3.3).

* Eq. (ema_err): E(p) <- (1 - beta) E(p) + beta e(p) at sampled pixels only.
  E is stored in half precision (Sec. 3.3 storage); the blend is computed in
  FP32 as fl(fl(fl(1 - beta) * E) + fl(beta * e)), each product and the sum
  rounded separately, then rounded to half to nearest-even.  This is a
  quantised code: both sides take it in the same (FP32) precision.
* Eq. (age_update): A(p) <- 0 at sampled pixels, A(p) + 1 elsewhere, for the
  views selected this step; saturating at 65535 (uint16 storage).
* Dense initialisation (Sec. 3.3, first paragraph; Alg. 1 initialisation):
  E_v(p) = e_0(p) = |I_hat(p) - I(p)|_1 over every pixel, rounded to half.
"""
from __future__ import annotations

import numpy as np


def ema_age_update(E_bits: np.ndarray, A: np.ndarray, xs, ys, err, beta: float):
    E = np.asarray(E_bits, dtype=np.uint16).view(np.float16).astype(np.float32).copy()
    A_new = np.minimum(np.asarray(A, dtype=np.int64) + 1, 65535)
    b32 = np.float32(beta)
    omb = np.float32(np.float32(1.0) - b32)
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    e32 = np.asarray(err, dtype=np.float32)
    t1 = (omb * E[ys, xs]).astype(np.float32)
    t2 = (b32 * e32).astype(np.float32)
    E[ys, xs] = (t1 + t2).astype(np.float32)
    A_new[ys, xs] = 0
    E_out = E.astype(np.float16).view(np.uint16)
    # pixels not sampled keep their exact half bits
    keep = np.ones(E.shape, dtype=bool)
    keep[ys, xs] = False
    E_out[keep] = np.asarray(E_bits, dtype=np.uint16)[keep]
    return E_out, A_new.astype(np.uint16)


def dense_error_init(rgb_dense: np.ndarray, gt: np.ndarray) -> np.ndarray:
    """E_0 from a dense render: rgb_dense [H, W, 3], gt [3, H, W] -> half bits.
    The L1 sum over channels is taken in FP32 left to right, |dr| + |dg| + |db|."""
    x = np.asarray(rgb_dense, dtype=np.float32)
    y = np.moveaxis(np.asarray(gt, dtype=np.float32), 0, -1)
    d = np.abs(x - y).astype(np.float32)
    e = ((d[..., 0] + d[..., 1]).astype(np.float32) + d[..., 2]).astype(np.float32)
    return e.astype(np.float16).view(np.uint16)
