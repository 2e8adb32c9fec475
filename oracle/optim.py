"""Hybrid moment-damped Levenberg-Marquardt / Adam update (Sec. 3.9,
Eq. moment_damped_lm, and App. A "Details of our moment-damped LM optimizer").

Per Gaussian, the geometry block g (position 3, log-scale 3, quaternion 4)
and the base-appearance block a (SH DC 3, opacity logit 1) each solve
    (J^T J + diag(sqrt(v) + eps)) Delta = -m
with the Adam moments m, v of that block; the higher SH coefficients take a
plain Adam step.  Readings:

* m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2 for every row of a touched
  Gaussian ("sparse": untouched Gaussians keep parameters and moments);
* the "local Jacobian estimated from the accumulated gradients" is the
  step's block gradient itself: J^T J = g g^T (mode 0) or its diagonal g^2
  (mode 1); mode 2 replaces the LM blocks by Adam (sparse-Adam baseline);
* LM uses the raw m, v as written; the parameter moves by lr_row * Delta
  (the equation has no step size; per-group learning rates as in 3DGS);
* Adam for SH rest: theta -= lr m_hat / (sqrt(v_hat) + eps) with bias
  corrections 1 - b^t at the global step t >= 1.

The oracle solves each system with numpy's dense solver (a library step; the
paper's Cholesky gives the same solution up to rounding).
"""
from __future__ import annotations

import numpy as np

from .params import OptimParams

GEOM_ROWS = list(range(0, 10))
APP_ROWS = [11, 12, 13, 10]
REST_ROWS = list(range(14, 59))


def _lm_block(gb, mb, vb, eps, mode):
    """Delta for one block: gb, mb, vb are [n, N] (rows of the block)."""
    n, N = gb.shape
    D = np.sqrt(vb) + eps
    if mode == 1:
        return -mb / (gb * gb + D)
    Hm = np.einsum("in,jn->nij", gb, gb)
    Hm[:, np.arange(n), np.arange(n)] += D.T
    return np.linalg.solve(Hm, -mb.T[:, :, None])[:, :, 0].T


def optimizer_step(params, grad, m, v, touched, op: OptimParams, step: int):
    """Returns updated (params, m, v) as FP64 arrays; inputs are not modified."""
    P = np.asarray(params, dtype=np.float64).copy()
    g = np.asarray(grad, dtype=np.float64)
    M = np.asarray(m, dtype=np.float64).copy()
    V = np.asarray(v, dtype=np.float64).copy()
    tmask = np.ones(P.shape[1], dtype=bool) if touched is None else np.asarray(touched).astype(bool)
    idx = np.nonzero(tmask)[0]
    gs = g[:, idx]
    M[:, idx] = op.beta1 * M[:, idx] + (1.0 - op.beta1) * gs
    V[:, idx] = op.beta2 * V[:, idx] + (1.0 - op.beta2) * gs * gs
    lr = op.row_lr()
    bc1 = 1.0 - op.beta1 ** step
    bc2 = 1.0 - op.beta2 ** step

    def adam(rows):
        mh = M[rows][:, idx] / bc1
        vh = V[rows][:, idx] / bc2
        return -lr[rows][:, None] * mh / (np.sqrt(vh) + op.eps_adam)

    upd = np.zeros((59, idx.size))
    upd[REST_ROWS] = adam(REST_ROWS)
    for rows in (GEOM_ROWS, APP_ROWS):
        if op.lm_mode == 2:
            upd[rows] = adam(rows)
        else:
            delta = _lm_block(gs[rows], M[rows][:, idx], V[rows][:, idx], op.eps_lm, op.lm_mode)
            upd[rows] = lr[rows][:, None] * delta
    P[:, idx] += upd
    return P, M, V
