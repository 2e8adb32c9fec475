"""Chain rule from screen-space splat gradients to the Gaussian parameters
(the backward of ``oracle.project``; the paper differentiates the standard
3DGS pipeline, Sec. 3.1 "this pipeline is differentiable").

Input g2d [9, N] = dL/d(mean2d x, y; conic a, b, c; opacity; rgb r, g, b).
Output dL/dparams [59, N] in the parameter-store layout.  Every step is the
derivative of the matching forward line, written with scalar formulas:

* rgb = max(sum_k Y_k(dir) sh_k + 1/2, 0): dL/dsh_k = Y_k dL/drgb (unclamped
  channels); dir = (mu - centre)/|mu - centre| feeds mu through the basis;
* opacity = sigmoid(logit): d/dlogit = o (1 - o);
* centre p = f t_xy / t_z + c - 1/2, t = W mu + t_cam;
* conic (ca, cb, cc) = (c, -b, a)/det of Sigma' = [[a, b], [b, c]];
* Sigma' = T Sigma T^T (+ dilation), T = J W:
  dL/dSigma = T^T G T and dL/dT = 2 G T Sigma with G the symmetric gradient
  matrix [[dL/da, dL/db / 2], [dL/db / 2, dL/dc]];
* J depends on t; Sigma = M M^T, M = R(q) diag(s): dL/dM = 2 dL/dSigma M;
* s = exp(log s); q_n = q/|q|: dL/dq = (I - q_n q_n^T) dL/dq_n / |q|.
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh
from .params import RasterParams


def _drot_dq(qn):
    """dR[i, j]/dq[a] for unit quaternions, shape [3, 3, 4, N]."""
    w, x, y, z = qn
    Z = np.zeros_like(w)
    d = np.empty((3, 3, 4) + w.shape)
    d[0, 0] = [Z, Z, -4 * y, -4 * z]
    d[0, 1] = [-2 * z, 2 * y, 2 * x, -2 * w]
    d[0, 2] = [2 * y, 2 * z, 2 * w, 2 * x]
    d[1, 0] = [2 * z, 2 * y, 2 * x, 2 * w]
    d[1, 1] = [Z, -4 * x, Z, -4 * z]
    d[1, 2] = [-2 * x, -2 * w, 2 * z, 2 * y]
    d[2, 0] = [-2 * y, 2 * z, -2 * w, 2 * x]
    d[2, 1] = [2 * x, 2 * w, 2 * z, 2 * y]
    d[2, 2] = [Z, -4 * x, -4 * y, Z]
    return d


def project_bwd(params: np.ndarray, cam, proj: dict, g2d: np.ndarray,
                rp: RasterParams = RasterParams()) -> np.ndarray:
    rp = rp.f64()
    p = np.asarray(params, dtype=np.float64)
    N = p.shape[1]
    grad = np.zeros((59, N))
    vis = proj["visible"]
    g = np.where(vis[None, :], np.asarray(g2d, dtype=np.float64), 0.0)
    fx, fy = float(cam.fx), float(cam.fy)
    Wc = np.asarray(cam.R, dtype=np.float64)
    tx, ty, tz = proj["t"]
    tz = np.where(vis, tz, 1.0)

    # --- colour -> SH coefficients and view direction
    nk = _sh.n_coeffs(rp.sh_degree)
    drgb = g[6:9] * (~proj["clamp"])                          # [3, N]
    Y = proj["Y"]
    for k in range(nk):
        for ch in range(3):
            grad[11 + 3 * k + ch] = Y[k] * drgb[ch]
    coeffs = p[11:11 + 3 * nk].reshape(nk, 3, N)
    dL_dY = np.einsum("kcn,cn->kn", coeffs, drgb)             # [k, N]
    dY_du = _sh.basis_grad(proj["dirs"], rp.sh_degree)        # [k, 3, N]
    dL_du = np.einsum("kn,kan->an", dL_dY, dY_du)
    dmu = dL_du / proj["dnorm"][None, :]

    # --- opacity
    o = proj["opacity"]
    grad[10] = g[5] * o * (1.0 - o)

    # --- centre
    dt = np.zeros((3, N))
    dt[0] += g[0] * fx / tz
    dt[1] += g[1] * fy / tz
    dt[2] += g[0] * (-fx * tx / (tz * tz)) + g[1] * (-fy * ty / (tz * tz))

    # --- conic -> Sigma' entries
    a, b, c = proj["S2"]
    det = a * c - b * b
    d2 = det * det
    gca, gcb, gcc = g[2], g[3], g[4]
    dL_da = gca * (-c * c / d2) + gcb * (b * c / d2) + gcc * (1.0 / det - a * c / d2)
    dL_db = gca * (2.0 * b * c / d2) + gcb * (-1.0 / det - 2.0 * b * b / d2) + gcc * (2.0 * a * b / d2)
    dL_dc = gca * (1.0 / det - a * c / d2) + gcb * (a * b / d2) + gcc * (-a * a / d2)
    Gs = np.empty((2, 2, N))
    Gs[0, 0] = dL_da
    Gs[0, 1] = Gs[1, 0] = 0.5 * dL_db
    Gs[1, 1] = dL_dc

    T = proj["T"]
    Sigma = proj["Sigma"]
    dSigma = np.einsum("kin,kln,ljn->ijn", T, Gs, T)          # T^T G T
    dT = 2.0 * np.einsum("ikn,kln,ljn->ijn", Gs, T, Sigma)    # 2 G T Sigma
    dJ = np.einsum("ikn,jk->ijn", dT, Wc)                     # dL/dT W^T
    dt[0] += dJ[0, 2] * (-fx / (tz * tz))
    dt[1] += dJ[1, 2] * (-fy / (tz * tz))
    dt[2] += (dJ[0, 0] * (-fx / (tz * tz)) + dJ[0, 2] * (2.0 * fx * tx / (tz ** 3))
              + dJ[1, 1] * (-fy / (tz * tz)) + dJ[1, 2] * (2.0 * fy * ty / (tz ** 3)))
    dmu += Wc.T @ dt

    # --- Sigma = M M^T, M = R(q) diag(s)
    Rq, s, qn = proj["Rq"], proj["s"], proj["qn"]
    M = Rq * s[None, :, :]
    dM = 2.0 * np.einsum("ikn,kjn->ijn", dSigma, M)
    ds = np.einsum("ijn,ijn->jn", Rq, dM)
    dR = dM * s[None, :, :]
    grad[3:6] = ds * s
    dqn = np.einsum("ijn,ijan->an", dR, _drot_dq(qn))
    qraw = p[6:10]
    qnorm = np.sqrt(np.sum(qraw * qraw, axis=0))
    grad[6:10] = (dqn - qn * np.sum(qn * dqn, axis=0)[None, :]) / qnorm[None, :]
    grad[0:3] = dmu
    grad[:, ~vis] = 0.0
    return grad
