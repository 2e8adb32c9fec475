"""Pins of the oracle's SH basis and EWA projection against closed forms,
exact quadrature and finite differences (no GPU)."""
import math

import numpy as np
import pytest

import synth
from oracle import project as P
from oracle import sh
from oracle.params import RasterParams


def _quadrature(n_theta=10, n_phi=24):
    """Gauss-Legendre in cos(theta) x uniform phi: exact for the products of
    two degree-3 harmonics (degree <= 6 in cos(theta), frequency <= 6 in phi)."""
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct]).reshape(3, -1)
    w = (wg[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).ravel()
    return dirs, w


def test_sh_orthonormal_by_exact_quadrature():
    dirs, w = _quadrature()
    Y = sh.basis(dirs, 3)
    gram = (Y * w[None, :]) @ Y.T
    assert np.allclose(gram, np.eye(16), atol=1e-12)


def test_sh_low_degree_closed_forms():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(3, 50))
    d /= np.linalg.norm(d, axis=0)
    Y = sh.basis(d, 3)
    assert np.allclose(Y[0], 0.5 / math.sqrt(math.pi))
    c1 = math.sqrt(3 / (4 * math.pi))
    # Condon-Shortley phase kept: (m=-1, 0, 1) -> (-y, z, -x)
    assert np.allclose(Y[1], -c1 * d[1])
    assert np.allclose(Y[2], c1 * d[2])
    assert np.allclose(Y[3], -c1 * d[0])
    # a degree-2 member: Y_{2,0} = sqrt(5/(16 pi)) (3 z^2 - 1)
    assert np.allclose(Y[6], math.sqrt(5 / (16 * math.pi)) * (3 * d[2] ** 2 - 1))


def test_sh_gradient_degree1_closed_form():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(3, 20))
    d /= np.linalg.norm(d, axis=0)
    g = sh.basis_grad(d, 1)
    c1 = math.sqrt(3 / (4 * math.pi))
    # Y_{1,0}(u/|u|) = c1 u_z/|u| -> gradient c1 (e_z - u_z u) at |u| = 1
    ez = np.zeros_like(d)
    ez[2] = 1
    assert np.allclose(g[2], c1 * (ez - d[2] * d), atol=1e-8)


def test_quaternion_rotation_orthonormal_and_sign_invariant():
    p = synth.gaussians(200, 3)
    Sigma, s, qn, R = P.covariance3d(p[3:6].astype(np.float64), p[6:10].astype(np.float64))
    Rt = np.moveaxis(R, -1, 0)
    assert np.allclose(Rt @ np.transpose(Rt, (0, 2, 1)), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(Rt), 1.0)
    Sigma2, *_ = P.covariance3d(p[3:6].astype(np.float64), -p[6:10].astype(np.float64))
    assert np.allclose(Sigma, Sigma2, rtol=1e-12, atol=0)
    ev = np.linalg.eigvalsh(np.moveaxis(Sigma, -1, 0))
    assert (ev > 0).all()
    # eigenvalues are the squared scales
    assert np.allclose(np.sort(ev, axis=1), np.sort((s ** 2).T, axis=1), rtol=1e-10)


def _axis_camera(f=300.0, W=64, H=48):
    return synth.Camera(R=np.eye(3), t=np.zeros(3), fx=f, fy=f, cx=W / 2, cy=H / 2, width=W, height=H)


def test_ewa_isotropic_on_axis_closed_form():
    cam = _axis_camera()
    d, sig = 2.5, 0.01
    p = np.zeros((59, 1), dtype=np.float32)
    p[2] = d
    p[3:6] = np.float32(math.log(sig))
    p[6] = 1.0
    rp = RasterParams(dilation=0.3)
    pr = P.project(p, cam, rp)
    dil = float(np.float32(0.3))
    var = (cam.fx * math.exp(float(np.float32(math.log(sig)))) / d) ** 2 + dil
    assert np.allclose(pr["conic"][:, 0], [1 / var, 0.0, 1 / var], rtol=1e-12)
    assert np.allclose(pr["mean2d"][:, 0], [cam.cx - 0.5, cam.cy - 0.5])
    # lambda_max = mid + sqrt(max(0.1, mid^2 - det)) and mid^2 = det when isotropic
    assert pr["radius"][0] == math.ceil(3 * math.sqrt(var + math.sqrt(0.1)))
    assert pr["depth32"][0] == np.float32(d)


def test_ewa_jacobian_matches_finite_differences_of_the_projection():
    """Sigma' = J W Sigma W^T J^T with J the derivative of the pinhole map at
    the camera-space centre: compare against J from central differences."""
    cams = synth.tetra_cameras()
    p = synth.gaussians(64, 4)
    rp = RasterParams(dilation=0.0)
    for cam in cams[:2]:
        pr = P.project(p, cam, rp)
        t = pr["t"]

        def pix(tt):
            return np.stack([cam.fx * tt[0] / tt[2] + cam.cx, cam.fy * tt[1] / tt[2] + cam.cy])

        h = 1e-6
        J = np.zeros((2, 3, t.shape[1]))
        for a in range(3):
            e = np.zeros_like(t)
            e[a] = h
            J[:, a] = (pix(t + e) - pix(t - e)) / (2 * h)
        T = np.einsum("ikn,kj->ijn", J, cam.R)
        S2 = np.einsum("ikn,kln,jln->ijn", T, pr["Sigma"], T)
        vis = pr["visible"]
        a, b, c = pr["S2"]
        assert np.allclose(S2[0, 0][vis], a[vis], rtol=1e-6)
        assert np.allclose(S2[0, 1][vis], b[vis], rtol=1e-6, atol=1e-9 * np.abs(a[vis]).max())
        assert np.allclose(S2[1, 1][vis], c[vis], rtol=1e-6)
        # centre: pinhole map minus the half-pixel shift
        assert np.allclose(pix(t)[:, vis] - 0.5, pr["mean2d"][:, vis], rtol=1e-13)


def test_conic_is_inverse_and_radius_covers_three_sigma():
    p = synth.gaussians(500, 5)
    cam = synth.tetra_cameras()[1]
    pr = P.project(p, cam)
    vis = pr["visible"]
    a, b, c = pr["S2"][:, vis]
    ca, cb, cc = pr["conic"][:, vis]
    assert np.allclose(a * ca + b * cb, 1.0)
    assert np.allclose(b * ca + c * cb, 0.0, atol=1e-9)
    lam = np.linalg.eigvalsh(np.moveaxis(np.array([[a, b], [b, c]]), -1, 0))[:, 1]
    assert (pr["radius"][vis] >= 3 * np.sqrt(lam) - 1e-9).all()


def test_colour_degree0_and_sigmoid():
    cam = _axis_camera()
    p = np.zeros((59, 3), dtype=np.float32)
    p[2] = 2.0
    p[3:6] = -4.0
    p[6] = 1.0
    p[10] = [0.0, 2.0, -30.0]
    p[11:14] = [[0.3, -2.0, 0.1], [0.0, 0.0, 0.0], [1.0, -1.5, 0.2]]   # [channel, gaussian]
    pr = P.project(p, cam, RasterParams(sh_degree=0))
    expect = p[11:14].astype(np.float64) * 0.5 / math.sqrt(math.pi) + 0.5
    assert np.allclose(pr["rgb"], np.maximum(expect, 0.0))
    assert pr["clamp"][0, 1] and pr["clamp"].sum() == 1
    assert np.allclose(pr["opacity"], 1 / (1 + np.exp(-p[10].astype(np.float64))))


def test_near_plane_and_offscreen_culling():
    cam = _axis_camera()
    p = synth.gaussians(3, 1)
    p[0:3, 0] = [0, 0, 0.1]      # in front of the camera but inside z_near
    p[0:3, 1] = [0, 0, -1.0]     # behind
    p[0:3, 2] = [50.0, 0, 1.0]   # far outside the image
    pr = P.project(p, cam)
    assert not pr["visible"].any()
    assert (pr["radius"] == 0).all() and (pr["rect"] == 0).all()
