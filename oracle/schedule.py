"""Training-loop scheduling: anchor view, geometry-aware view sampling
(Sec. 3.4, Eq. anchor_view, Eq. view_sampling) and the adaptive view budget
and pixel rate (App. A, Eq. sin_rate and the schedule of r_tile and K_t).

Readings (the paper leaves these open):

* E_bar_v is the mean of the half error map over the image with each value
  taken exactly; negative, NaN and infinite entries count 0 (the sampler's
  weight convention).  It is computed as the integer sum of the values scaled
  by 2^24 (every finite non-negative half is then an integer), divided by
  2^24 |Omega| in FP64;
* the view stack is the set of views not yet drawn; when fewer than K remain
  it is refilled with every view (the anchor is an argmax and the companions
  are drawn by weight, so the stack's order plays no part);
* the anchor is the stack's view of largest E_bar (lowest index on ties);
* the K - 1 companions are drawn one at a time without replacement from the
  rest of the stack with weights pi(u | v*) in FP64 (math.exp); a draw takes
  the 64-bit counter value u = draw(seed, t, 0, V, j) for companion j,
  r = (u >> 11) 2^-53 W_rem, and picks the first candidate in ascending view
  index whose running weight exceeds r;
* lambda_d and lambda_theta are inputs (the paper gives no values);
* E_bar_t is the mean of the views' E_bar, E_bar_init its value after the
  dense initialisation; eps = 1e-8; round() is floor(x + 1/2); the pixel
  rate in permille is floor(1000 r_tile + 1/2) clipped to [1, 1000];
* rho_t = 1 - clip(t / tau_until, 0, 1) (the appendix's definition);
* random view sampling (the "Geo-VS -> RVS" ablation baseline of Tab.
  ablation_main) draws the step's K views uniformly without replacement
  from all views, with no anchor and no stack: draw j takes the 64-bit
  counter value u = draw(seed, t, 1, V, j) and picks the
  floor(u m / 2^64)-th of the m views not yet drawn, in ascending order.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np

from .rng import below, draw

SCALE = 1 << 24


def half_weight_sum(E_bits: np.ndarray) -> int:
    """Exact sum of the map's values times 2^24 (non-finite or negative: 0)."""
    h = np.asarray(E_bits, dtype=np.uint16).view(np.float16).astype(np.float64).ravel()
    ok = np.isfinite(h) & (h >= 0)
    return int(sum(int(x) for x in (h[ok] * SCALE)))


def mean_view_error(E_bits: np.ndarray) -> float:
    """Eq. anchor_view: E_bar_v = (1 / |Omega|) sum_p E_v(p)."""
    return half_weight_sum(E_bits) / (SCALE * np.asarray(E_bits).size)


def view_weight(c_u, d_u, c_a, d_a, lam_d: float, lam_t: float) -> float:
    """Eq. view_sampling: exp(-lam_d |c_u - c_a| - lam_t (1 - <d_u, d_a>))."""
    dist = math.sqrt(sum((float(c_u[k]) - float(c_a[k])) ** 2 for k in range(3)))
    cos = sum(float(d_u[k]) * float(d_a[k]) for k in range(3))
    return math.exp(-lam_d * dist - lam_t * (1.0 - cos))


def select_views(stack: list, means, centres, dirs, K: int, lam_d: float, lam_t: float, seed: int, t: int):
    """One step's view set: (views [anchor first, then companions], new stack)."""
    V = len(means)
    K = min(K, V)
    if len(stack) < K:
        stack = list(range(V))
    stack = sorted(stack)
    anchor = max(stack, key=lambda v: (means[v], -v))
    chosen = [anchor]
    rest = [u for u in stack if u != anchor]
    for j in range(K - 1):
        w = [view_weight(centres[u], dirs[u], centres[anchor], dirs[anchor], lam_d, lam_t) for u in rest]
        total = sum(w)
        r = (draw(seed, t, 0, V, j) >> 11) * 2.0 ** -53 * total
        acc, pick = 0.0, len(rest) - 1
        for i, wi in enumerate(w):
            acc += wi
            if acc > r:
                pick = i
                break
        chosen.append(rest.pop(pick))
    return chosen, [u for u in stack if u not in chosen]


def schedule(t: int, E_t: float, E_init: float, tau_until: int, K_min: int, K_max: int, lam: float,
             alpha: float, eps: float = 1e-8) -> dict:
    """Eq. sin_rate and the schedule of r_tile and K_t."""
    r = min(max(E_t / (E_init + eps), 0.0), 1.0)
    phi = math.sin(math.pi / 2.0 * math.sqrt(r))
    rho = 1.0 - min(max(t / tau_until, 0.0), 1.0)
    a = 1.0 - rho * phi
    r_min, r_max = lam / K_max, lam / K_min
    r_tile = r_min + (r_max - r_min) * a
    K = int(math.floor(K_min + (K_max - K_min) * math.exp(-alpha * a) + 0.5))
    permille = min(max(int(math.floor(1000.0 * r_tile + 0.5)), 1), 1000)
    return dict(r=r, phi=phi, rho=rho, r_tile=r_tile, K=K, permille=permille)


def random_views(V: int, K: int, seed: int, t: int) -> list:
    """Random view sampling: K distinct views uniformly at random (draw order)."""
    K = min(K, V)
    rest = list(range(V))
    chosen = []
    for j in range(K):
        chosen.append(rest.pop(below(draw(seed, t, 1, V, j), len(rest))))
    return chosen
