"""EWA projection of 3D Gaussians to 2D splats with SH colour (Sec. 3.1:
each primitive has a centre, a covariance from scale and rotation, an opacity
and colour coefficients, and is projected to the image plane as a 2D splat
whose footprint and opacity give alpha).  The paper prints no projection
formula; it is the EWA splatting of the original 3D Gaussian Splatting, which
the paper builds on.  Readings used here:

* activations: scale = exp(log-scale), opacity = sigmoid(logit), rotation from
  the normalised quaternion (w, x, y, z);
* camera space t = R mu + t_cam; cull t_z <= z_near;
* Sigma = M M^T with M = R(q) diag(s); Sigma' = J W Sigma W^T J^T + dil * I
  with J the perspective Jacobian at t and W the camera rotation;
* conic = inverse of Sigma'; radius = ceil(3 sqrt(lambda_max));
* splat centre in pixel-index space p = (fx tx/tz + cx - 1/2, fy ty/tz + cy - 1/2),
  pixel (i, j) is evaluated at d = (i, j) - p;
* tile rectangle [trunc((p - r)/16), trunc((p + r + 15)/16)) clamped to the grid;
  cull when it is empty;
* colour = sum_k sh_k Y_k(dir) + 1/2 with dir = normalise(mu - camera centre),
  clamped at 0 per channel.

Everything is FP64.  The values that decide integers exactly (the camera-
space depth, whose FP32 rounding is the sort key, and the splat centre, which
places the tile rectangle) are written out term by term with a fixed
operation order and no fused multiply-add, so any IEEE implementation of the
same sequence reproduces them bit for bit.  The radius goes through exp and
sqrt; it is an FP64 value rounded up to an integer, so two faithful FP64
implementations disagree on it only when 3 sqrt(lambda_max) lies within a few
ulp of an integer.  ``radius_margin`` reports that distance so tests can
assert it is far from zero.
"""
from __future__ import annotations

import math

import numpy as np

from . import sh as _sh
from .params import RasterParams

TILE = 16


def quat_to_rot(qn: np.ndarray) -> np.ndarray:
    """Rotation matrix [3, 3, N] of unit quaternions qn[4, N] = (w, x, y, z)."""
    w, x, y, z = qn
    R = np.empty((3, 3) + w.shape)
    R[0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[0, 1] = 2.0 * (x * y - w * z)
    R[0, 2] = 2.0 * (x * z + w * y)
    R[1, 0] = 2.0 * (x * y + w * z)
    R[1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[1, 2] = 2.0 * (y * z - w * x)
    R[2, 0] = 2.0 * (x * z - w * y)
    R[2, 1] = 2.0 * (y * z + w * x)
    R[2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R


def camera_center(cam) -> np.ndarray:
    """World position of the camera: -R^T t."""
    R = np.asarray(cam.R, dtype=np.float64)
    t = np.asarray(cam.t, dtype=np.float64)
    return -(R.T @ t)


def _cam_space(mu: np.ndarray, cam) -> np.ndarray:
    """t = R mu + t_cam, each row summed left to right: ((R0 mx + R1 my) + R2 mz) + t."""
    R = np.asarray(cam.R, dtype=np.float64)
    tc = np.asarray(cam.t, dtype=np.float64)
    out = np.empty_like(mu)
    for r in range(3):
        out[r] = ((R[r, 0] * mu[0] + R[r, 1] * mu[1]) + R[r, 2] * mu[2]) + tc[r]
    return out


def covariance3d(log_scale: np.ndarray, quat: np.ndarray):
    """Sigma = R S S^T R^T (Sec. 3.1: covariance via scale and rotation)."""
    s = np.exp(log_scale)
    n = np.sqrt(((quat[0] * quat[0] + quat[1] * quat[1]) + quat[2] * quat[2]) + quat[3] * quat[3])
    qn = quat / n
    Rq = quat_to_rot(qn)
    M = Rq * s[None, :, :]                       # M[i, j] = R[i, j] s_j
    Sigma = np.einsum("ikn,jkn->ijn", M, M)      # M M^T
    return Sigma, s, qn, Rq


def project(params: np.ndarray, cam, rp: RasterParams = RasterParams()) -> dict:
    """Project every Gaussian of ``params[59, N]`` into ``cam``.

    Returns a dict of per-Gaussian arrays (FP64 unless stated):
      depth (t_z), depth32 (float32 t_z), mean2d [2, N], conic [3, N] = (a, b, c)
      of Q = [[a, b], [b, c]], opacity, rgb [3, N], radius (int), rect [4, N]
      (xmin, ymin, xmax, ymax; int), visible (bool), clamp [3, N] (bool: channel
      was clamped at 0), plus intermediates the backward pass re-uses.
    """
    rp = rp.f64()
    p = np.asarray(params, dtype=np.float64)
    N = p.shape[1]
    mu = p[0:3]
    W, H = cam.width, cam.height
    TX, TY = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)

    t = _cam_space(mu, cam)
    tx, ty, tz = t
    in_front = tz > rp.z_near
    tzs = np.where(in_front, tz, 1.0)  # placeholder depth for culled ones

    Sigma, s, qn, Rq = covariance3d(p[3:6], p[6:10])

    # Perspective Jacobian J (2x3) at t and T = J W (W = camera rotation).
    Wc = np.asarray(cam.R, dtype=np.float64)
    J = np.zeros((2, 3, N))
    J[0, 0] = fx / tzs
    J[0, 2] = -(fx * tx) / (tzs * tzs)
    J[1, 1] = fy / tzs
    J[1, 2] = -(fy * ty) / (tzs * tzs)
    T = np.einsum("ikn,kj->ijn", J, Wc)
    # Sigma' = T Sigma T^T, then the low-pass dilation.
    TS = np.einsum("ikn,kjn->ijn", T, Sigma)
    S2 = np.einsum("ikn,jkn->ijn", TS, T)
    a = S2[0, 0] + rp.dilation
    b = S2[0, 1]
    c = S2[1, 1] + rp.dilation
    det = a * c - b * b
    ok_det = det > 0.0
    dets = np.where(ok_det, det, 1.0)
    conic = np.stack([c / dets, -b / dets, a / dets])

    mid = 0.5 * (a + c)
    lam1 = mid + np.sqrt(np.maximum(0.1, mid * mid - det))
    radius = np.ceil(3.0 * np.sqrt(lam1))

    px = ((fx * tx) / tzs + cx) - 0.5
    py = ((fy * ty) / tzs + cy) - 0.5

    def trunc_clamp(v, hi):
        return np.clip(np.trunc(v), 0, hi).astype(np.int64)

    xmin = trunc_clamp((px - radius) / TILE, TX)
    xmax = trunc_clamp((px + radius + (TILE - 1)) / TILE, TX)
    ymin = trunc_clamp((py - radius) / TILE, TY)
    ymax = trunc_clamp((py + radius + (TILE - 1)) / TILE, TY)
    area = (xmax - xmin) * (ymax - ymin)
    visible = in_front & ok_det & (area > 0)

    # View-dependent colour from SH (degree rp.sh_degree), +1/2 offset, clamp at 0.
    cc = camera_center(cam)
    dvec = mu - cc[:, None]
    dn = np.sqrt(np.sum(dvec * dvec, axis=0))
    dirs = dvec / dn
    nk = _sh.n_coeffs(rp.sh_degree)
    Y = _sh.basis(dirs, rp.sh_degree)                  # [nk, N]
    coeffs = p[11:11 + 3 * nk].reshape(nk, 3, N)       # [k, ch, N]
    rgb_raw = np.einsum("kn,kcn->cn", Y, coeffs) + 0.5
    if rp.clamp_color:
        clamp = rgb_raw < 0.0
        rgb = np.maximum(rgb_raw, 0.0)
    else:
        clamp = np.zeros_like(rgb_raw, dtype=bool)
        rgb = rgb_raw

    opacity = 1.0 / (1.0 + np.exp(-p[10]))

    rect = np.stack([xmin, ymin, xmax, ymax])
    rect[:, ~visible] = 0
    radius_i = np.where(visible, radius, 0).astype(np.int64)
    return dict(
        depth=tz, depth32=tz.astype(np.float32), mean2d=np.stack([px, py]), conic=conic,
        opacity=opacity, rgb=rgb, radius=radius_i, rect=rect, visible=visible, clamp=clamp,
        # intermediates for the backward pass
        t=t, Sigma=Sigma, S2=np.stack([a, b, c]), s=s, qn=qn, Rq=Rq, J=J, T=T,
        dirs=dirs, dnorm=dn, Y=Y, TX=TX, TY=TY,
        radius_margin=np.abs(3.0 * np.sqrt(lam1) - np.round(3.0 * np.sqrt(lam1))),
    )


def rect_of(mean2d, radius, TX, TY):
    """Tile rectangle of a splat, as in ``project`` (used by brute-force checks)."""
    px, py = mean2d
    xmin = min(TX, max(0, math.trunc((px - radius) / TILE)))
    xmax = min(TX, max(0, math.trunc((px + radius + TILE - 1) / TILE)))
    ymin = min(TY, max(0, math.trunc((py - radius) / TILE)))
    ymax = min(TY, max(0, math.trunc((py + radius + TILE - 1) / TILE)))
    return xmin, ymin, xmax, ymax
