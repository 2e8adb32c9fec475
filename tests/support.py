"""Helpers shared by the GPU parity tests: seeded scenes, conversion of oracle
stage outputs into the library's input layouts, and tolerance checks.

Every GPU stage is fed inputs that come from ``synth`` or from the oracle,
never from another GPU stage, so each comparison isolates one kernel."""
from __future__ import annotations

import numpy as np

import synth
from oracle import binning, project, render, sampler
from oracle.params import RasterParams, SampleParams

TILE = 16


def scene_c1(n=10000):
    """The tiny workload: 10k Gaussians, four 256x256 tetrahedron views."""
    return synth.gaussians(n, synth.SEED_SCENE), synth.tetra_cameras()


def scene_scaling(n=300000):
    """The rasterizer-scaling workload: 300k Gaussians, one 1296x840 view."""
    return synth.gaussians(n, synth.SEED_SCENE), synth.config_camera("scaling")


def small_scene(n=400, seed=21, W=150, H=107):
    """A few hundred Gaussians over a ragged image (partial edge tiles)."""
    p = synth.gaussians(n, seed, logscale_mean=-3.3)
    cam = synth.look_at((2.4, -1.1, 1.3), fx=W * 1.2, fy=W * 1.2, width=W, height=H)
    return p, cam


def splat_record(pr: dict) -> np.ndarray:
    """The library's [N, 12] splat record built from an oracle projection."""
    N = pr["opacity"].size
    s = np.zeros((N, 12), dtype=np.float32)
    px, py = pr["mean2d"]
    fx, fy = np.floor(px), np.floor(py)
    s[:, 0], s[:, 1] = fx, fy
    s[:, 2], s[:, 3] = px - fx, py - fy
    s[:, 4:7] = pr["conic"].T
    s[:, 7] = pr["opacity"]
    s[:, 8:11] = pr["rgb"].T
    s[:, 11] = pr["depth32"]
    vis = pr["visible"]
    s[~vis, :11] = 0.0
    return s


def splat_as_oracle(pr: dict, rec: np.ndarray) -> dict:
    """An oracle projection dict whose 2D splat values are the FP32 record
    widened back to FP64 (so both sides composite identical splats)."""
    q = dict(pr)
    q["mean2d"] = np.stack([rec[:, 0].astype(np.float64) + rec[:, 2], rec[:, 1].astype(np.float64) + rec[:, 3]])
    q["conic"] = rec[:, 4:7].T.astype(np.float64)
    q["opacity"] = rec[:, 7].astype(np.float64)
    q["rgb"] = rec[:, 8:11].T.astype(np.float64)
    return q


def samples_dict(s: dict):
    return s["valid_tiles"], s["tile_off"], s["pix"]


def close(a, b, rtol, atol=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b)
    bound = rtol * np.abs(b) + atol
    bad = err > bound
    return (~bad).all(), err, bound, bad


def assert_close(a, b, rtol, atol=0.0, what=""):
    ok, err, bound, bad = close(a, b, rtol, atol)
    if not ok:
        i = np.argmax(err - bound)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside tolerance; worst index {i}: "
                             f"got {np.asarray(a).ravel()[i]!r}, want {np.asarray(b).ravel()[i]!r}, "
                             f"max rel {np.max(err / np.maximum(np.abs(b), 1e-30)):.3g}")
