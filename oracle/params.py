"""Parameter records of the oracle (values the paper leaves open are readings;
each default is the value stated for the reading).

The rasterizer thresholds are stored as the FP32 numbers the GPU kernels
receive, then widened to FP64, so both sides compare against the same value.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _f32(x: float) -> float:
    return float(np.float32(x))


@dataclass
class RasterParams:
    sh_degree: int = 3
    z_near: float = 0.2          # near-plane cull (3DGS convention)
    dilation: float = 0.3        # low-pass added to the 2D covariance diagonal, px^2
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    clamp_color: bool = True     # clamp the SH colour at 0 (oracle-only switch for FD tests)

    def f64(self) -> "RasterParams":
        """The same record with every threshold rounded through FP32."""
        return RasterParams(self.sh_degree, _f32(self.z_near), _f32(self.dilation),
                            _f32(self.alpha_min), _f32(self.alpha_max), _f32(self.T_min),
                            tuple(_f32(b) for b in self.bg), self.clamp_color)


@dataclass
class SampleParams:
    n_pix: int                   # pixels per full tile, N_pix
    hard_permille: int = 400     # r_hard
    stable_permille: int = 300   # r_stable
    n_tiles_sel: int = -1        # tiles drawn per view (-1: every tile)


@dataclass
class LossParams:
    eps_charb: float = 1e-3
    eps_ncc: float = 1e-6
    eps_lambda: float = 1e-8
    structure: str = "ncc"       # tile structure term: "ncc" (S-NCC) or "ssim" (the S-SSIM ablation)


@dataclass
class OptimParams:
    lr_mean: float = 1.6e-4
    lr_scale: float = 5e-3
    lr_quat: float = 1e-3
    lr_opacity: float = 2.5e-2
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20.0
    beta1: float = 0.9
    beta2: float = 0.999
    eps_adam: float = 1e-15
    eps_lm: float = 1e-8
    lm_mode: int = 0             # 0: J^T J = g g^T, 1: J^T J = diag(g^2), 2: Adam everywhere

    def row_lr(self) -> np.ndarray:
        lr = np.empty(59)
        lr[0:3] = self.lr_mean
        lr[3:6] = self.lr_scale
        lr[6:10] = self.lr_quat
        lr[10] = self.lr_opacity
        lr[11:14] = self.lr_sh_dc
        lr[14:59] = self.lr_sh_rest
        return lr


def pixels_per_tile(rate_permille: int, tile: int = 16) -> int:
    """N_pix = max(1, floor(r_t * S^2)) (Sec. 3.5) with r_t in per-mille, in integers."""
    return max(1, (rate_permille * tile * tile) // 1000)


def split_counts(n: int, hard_permille: int, stable_permille: int) -> tuple[int, int, int]:
    """N_hard = round(r_hard * n), N_stable = round(r_stable * n) (Sec. 3.5),
    rounding half up in integer arithmetic; the rest of the tile budget goes to
    the mixed set."""
    n_hard = (hard_permille * n + 500) // 1000
    n_stable = (stable_permille * n + 500) // 1000
    if n_hard + n_stable > n:
        n_stable = n - n_hard
    return n_hard, n_stable, n - n_hard - n_stable
