"""Real spherical-harmonic basis up to degree 3 (the colour coefficients of
Sec. 3.1 are SH coefficients; the paper names them but not the basis).

Reading: the orthonormal real basis with the Condon-Shortley phase kept in
the associated Legendre functions, ordered by degree l, then m = -l..l:

    Y_l0  = K_l^0 P_l^0(cos t)
    Y_lm  = sqrt(2) K_l^m P_l^m(cos t) cos(m p)        (m > 0)
    Y_l-m = sqrt(2) K_l^m P_l^m(cos t) sin(m p)        (m > 0)
    K_l^m = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!)

This is the basis the original 3D Gaussian Splatting colour model uses.  The
oracle evaluates it from its definition (Legendre recurrence, spherical
angles), not from Cartesian polynomials.
"""
from __future__ import annotations

import math

import numpy as np


def assoc_legendre(l: int, m: int, x: np.ndarray) -> np.ndarray:
    """P_l^m(x) for 0 <= m <= l, Condon-Shortley phase included, by the
    standard upward recurrence in l."""
    x = np.asarray(x, dtype=np.float64)
    somx2 = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.ones_like(x)
    fact = 1.0
    for _ in range(m):
        pmm = -pmm * fact * somx2
        fact += 2.0
    if l == m:
        return pmm
    pmmp1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pmmp1
    pll = pmmp1
    for ll in range(m + 2, l + 1):
        pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pmmp1 = pmmp1, pll
    return pll


def norm_const(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def n_coeffs(degree: int) -> int:
    return (degree + 1) ** 2


def basis(dirs: np.ndarray, degree: int = 3) -> np.ndarray:
    """Y[k, ...] for unit directions ``dirs[3, ...]``, k = l*l + l + m."""
    d = np.asarray(dirs, dtype=np.float64)
    x, y, z = d[0], d[1], d[2]
    cost = np.clip(z, -1.0, 1.0)
    phi = np.arctan2(y, x)
    out = np.zeros((n_coeffs(degree),) + x.shape, dtype=np.float64)
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            k = l * l + l + m
            am = abs(m)
            p = assoc_legendre(l, am, cost)
            if m == 0:
                out[k] = norm_const(l, 0) * p
            elif m > 0:
                out[k] = math.sqrt(2.0) * norm_const(l, am) * p * np.cos(am * phi)
            else:
                out[k] = math.sqrt(2.0) * norm_const(l, am) * p * np.sin(am * phi)
    return out


def basis_grad(dirs: np.ndarray, degree: int = 3, h: float = 1e-6) -> np.ndarray:
    """dY_k/d(dir) for unit directions, as the gradient of the basis extended
    off the sphere as a function of the Cartesian direction *before*
    normalisation is not needed: the caller chains through the normalisation.

    The basis is evaluated from spherical angles, which makes an analytic
    Cartesian derivative awkward; Y_lm(d/|d|) is smooth in d, so its gradient
    with respect to the unit vector is taken by FP64 central differences of
    the normalised function and is exact to ~1e-9.  Returns [k, 3, ...] with
    the derivative of Y_k(u / |u|) at u = dir (tangential to the sphere)."""
    d = np.asarray(dirs, dtype=np.float64)
    g = np.zeros((n_coeffs(degree), 3) + d.shape[1:], dtype=np.float64)
    for a in range(3):
        e = np.zeros_like(d)
        e[a] = h
        dp = d + e
        dm = d - e
        dp = dp / np.linalg.norm(dp, axis=0, keepdims=True)
        dm = dm / np.linalg.norm(dm, axis=0, keepdims=True)
        g[:, a] = (basis(dp, degree) - basis(dm, degree)) / (2 * h)
    return g
