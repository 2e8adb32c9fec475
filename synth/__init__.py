"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and lays out scene data (Gaussian
parameters, pinhole cameras, error/age maps, target images).  It holds none of
the method's arithmetic: no projection, compositing, sampling, loss or update.

Parameter store layout (one contiguous float32 array ``params[59, N]``):

======  =====================================================================
rows    meaning
======  =====================================================================
0..2    mean (x, y, z), world space
3..5    log-scale (the activation is exp)
6..9    rotation quaternion (w, x, y, z), unnormalised (activation: q/|q|)
10      opacity logit (activation: sigmoid)
11..58  SH coefficients, coefficient-major: row 11 + 3*k + ch for basis
        function k = 0..15 (order l, then m = -l..l) and colour channel ch
======  =====================================================================

Cameras are OpenCV pinhole cameras: x right, y down, z forward.  ``R`` is the
world-to-camera rotation (row-major 3x3), ``t`` the translation, so a world
point X maps to R @ X + t in camera space.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

N_ROWS = 59
ROW_MEAN = 0
ROW_LOGSCALE = 3
ROW_QUAT = 6
ROW_OPACITY = 10
ROW_SH = 11
TILE = 16

# Seeds of the workload recipe: scene, perturbation, pixel noise, sampler, view order.
SEED_SCENE, SEED_PERTURB, SEED_NOISE, SEED_SAMPLER, SEED_VIEWS = 0, 1, 2, 3, 4


@dataclass
class Camera:
    R: np.ndarray  # (3, 3) float64, world -> camera rotation
    t: np.ndarray  # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def tiles(self) -> tuple[int, int]:
        return (self.width + TILE - 1) // TILE, (self.height + TILE - 1) // TILE


def gaussians(n: int, seed: int = SEED_SCENE, extent: float = 1.0,
              logscale_mean: float = -4.0, logscale_std: float = 0.5,
              sh_std: float = 0.2) -> np.ndarray:
    """Random Gaussians: means U[-extent, extent]^3, log-scales N(mean, std),
    uniformly random unit quaternions (normalised 4-D normal), opacity logits
    N(0, 1), all 48 SH coefficients N(0, sh_std).  Returns float32 [59, n]."""
    rng = np.random.default_rng(seed)
    p = np.empty((N_ROWS, n), dtype=np.float32)
    p[0:3] = rng.uniform(-extent, extent, size=(3, n))
    p[3:6] = rng.normal(logscale_mean, logscale_std, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    p[6:10] = q
    p[10] = rng.normal(0.0, 1.0, size=n)
    p[11:59] = rng.normal(0.0, sh_std, size=(48, n))
    return p


def perturb(params: np.ndarray, seed: int = SEED_PERTURB) -> np.ndarray:
    """Seeded perturbation of a scene (the recovery target differs from the
    initial model by these amounts): mean += N(0, 0.01), log-scale += N(0, 0.05),
    quaternion += N(0, 0.05) then renormalised, logit += N(0, 0.2), SH += N(0, 0.02)."""
    rng = np.random.default_rng(seed)
    n = params.shape[1]
    p = params.astype(np.float64).copy()
    p[0:3] += rng.normal(0, 0.01, size=(3, n))
    p[3:6] += rng.normal(0, 0.05, size=(3, n))
    q = p[6:10] + rng.normal(0, 0.05, size=(4, n))
    p[6:10] = q / np.linalg.norm(q, axis=0, keepdims=True)
    p[10] += rng.normal(0, 0.2, size=n)
    p[11:59] += rng.normal(0, 0.02, size=(48, n))
    return p.astype(np.float32)


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0), *, fx: float, fy: float,
            width: int, height: int, cx: float | None = None, cy: float | None = None) -> Camera:
    """OpenCV camera at ``eye`` looking at ``target`` with world ``up`` pointing
    to the top of the image.  Principal point defaults to the image centre."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, dtype=np.float64)
    right = np.cross(fwd, upv)
    if np.linalg.norm(right) < 1e-8:  # looking along +-up: pick another up
        right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    return Camera(R=R, t=t, fx=float(fx), fy=float(fy),
                  cx=float(width / 2 if cx is None else cx),
                  cy=float(height / 2 if cy is None else cy),
                  width=int(width), height=int(height))


def tetra_cameras(radius: float = 3.0, size: int = 256, focal: float = 300.0) -> list[Camera]:
    """Four cameras on a sphere at the regular-tetrahedron directions
    (+-1, +-1, +-1)/sqrt(3) with an even number of minus signs, looking at the origin."""
    dirs = [(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]
    cams = []
    for d in dirs:
        e = radius * np.asarray(d, dtype=np.float64) / math.sqrt(3.0)
        cams.append(look_at(e, fx=focal, fy=focal, width=size, height=size))
    return cams


def hemisphere_cameras(n: int, radius: float = 3.0, width: int = 1600, height: int = 1060,
                       focal: float = 1875.0) -> list[Camera]:
    """``n`` cameras on the upper hemisphere (Fibonacci lattice, z in (0.05, 0.95))."""
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for i in range(n):
        z = 0.05 + 0.9 * (i + 0.5) / n
        r = math.sqrt(1.0 - z * z)
        phi = golden * i
        e = radius * np.array([r * math.cos(phi), r * math.sin(phi), z])
        cams.append(look_at(e, fx=focal, fy=focal, width=width, height=height))
    return cams


def corridor_gaussians(n: int, seed: int = SEED_SCENE, length: float = 50.0, width: float = 8.0,
                       height: float = 3.0, logscale_mean: float = -4.0) -> np.ndarray:
    """Random Gaussians filling a corridor along the x axis: means uniform in
    [-length/2, length/2] x [-width/2, width/2] x [-height/2, height/2], the
    other distributions as in ``gaussians``.  Float32 [59, n]."""
    p = gaussians(n, seed, logscale_mean=logscale_mean)
    rng = np.random.default_rng(seed + 1000)
    p[0] = rng.uniform(-length / 2, length / 2, n)
    p[1] = rng.uniform(-width / 2, width / 2, n)
    p[2] = rng.uniform(-height / 2, height / 2, n)
    return p


def trajectory_cameras(n: int, length: float = 50.0, offset: float = 6.0, elevation: float = 1.5,
                       width: int = 1920, height: int = 1080, focal: float = 1100.0) -> list[Camera]:
    """``n`` cameras spread along a 50-unit trajectory beside the corridor:
    x from -length/2 to length/2, alternately on either side (y = -+offset)
    at z = elevation with a slow sinusoidal sway, each looking at the
    corridor's axis a little ahead of itself."""
    cams = []
    for i in range(n):
        x = -length / 2 + length * (i + 0.5) / n
        side = -1.0 if i % 2 == 0 else 1.0
        y = side * offset * (1.0 + 0.1 * math.sin(0.7 * i))
        z = elevation + 0.5 * math.sin(0.31 * i)
        cams.append(look_at((x, y, z), (x + 1.5 * math.sin(0.13 * i), 0.0, 0.0), fx=focal, fy=focal,
                            width=width, height=height))
    return cams


def config_camera(name: str) -> Camera:
    """The single view of the rasterizer-scaling workload (1296x840, focal kept
    from the 256x256/f=300 field of view) or a tetrahedron view."""
    if name == "scaling":
        e = 3.0 * np.ones(3) / math.sqrt(3.0)
        return look_at(e, fx=300.0 * 1296 / 256, fy=300.0 * 1296 / 256, width=1296, height=840)
    raise KeyError(name)


def error_map(height: int, width: int, seed: int, zero_frac: float = 0.1) -> np.ndarray:
    """Half-precision error map (returned as uint16 bit patterns): smooth
    blob-structured positive values with a heavy tail, a fraction of exact
    zeros (whole blocks) so zero-weight tiles and pixels occur."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:height, 0:width].astype(np.float64)
    e = np.zeros((height, width))
    for _ in range(8):
        cx, cy = rng.uniform(0, width), rng.uniform(0, height)
        s = rng.uniform(0.05, 0.3) * max(width, height)
        e += rng.uniform(0.05, 0.5) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
    e *= rng.gamma(2.0, 0.5, size=e.shape)
    if zero_frac > 0:
        by, bx = (height + 31) // 32, (width + 31) // 32
        zmask = rng.uniform(size=(by, bx)) < zero_frac
        e[np.kron(zmask, np.ones((32, 32), dtype=bool))[:height, :width]] = 0.0
    return e.astype(np.float16).view(np.uint16)


def age_map(height: int, width: int, seed: int, max_age: int = 40) -> np.ndarray:
    """uint16 age map with many ties (small integer range)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, max_age + 1, size=(height, width), dtype=np.uint16)


def image(height: int, width: int, seed: int) -> np.ndarray:
    """Smooth random RGB image in [0, 1], float32 [3, H, W]."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:height, 0:width].astype(np.float64)
    img = np.zeros((3, height, width))
    for c in range(3):
        for _ in range(6):
            kx, ky = rng.normal(0, 0.05, size=2)
            img[c] += rng.uniform(0.05, 0.2) * np.sin(kx * x + ky * y + rng.uniform(0, 6.3))
    img += 0.5 + rng.normal(0, 0.01, size=img.shape)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def pixel_noise(shape, seed: int = SEED_NOISE, std: float = 0.01) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, std, size=shape).astype(np.float32)

