"""Training-loop scheduling on the host (Sec. 3.4, Eq. anchor_view and
Eq. view_sampling; App. A, Eq. sin_rate and the schedule of the pixel rate
r_tile and the view budget K_t).  The per-view mean errors come from the GPU
(tgs_view_error_sums); the rest is a handful of scalars per step.

Conventions (fixed so that runs are reproducible):
* E_bar_v = (exact sum of E_v * 2^24) / (2^24 |Omega|) in FP64;
* the view stack is the set of views not yet drawn, refilled with every
  view when fewer than K remain;
* the anchor is the stack's view of largest E_bar (lowest index on ties);
* K - 1 companions are drawn without replacement from the rest of the stack
  with weights exp(-lambda_d |c_u - c_a| - lambda_theta (1 - <d_u, d_a>))
  (FP64): companion j takes the SplitMix64 counter value of
  (seed, t, 0, V, j), r = (u >> 11) 2^-53 W_rem, and the first candidate in
  ascending view index whose running weight exceeds r;
* rho_t = 1 - clip(t / tau_until, 0, 1), r_t = clip(E_bar_t / (E_bar_init
  + 1e-8), 0, 1), phi = sin(pi/2 sqrt(r_t)), a = 1 - rho_t phi;
  r_tile = r_min + (r_max - r_min) a, K_t = floor(K_min + (K_max - K_min)
  exp(-alpha a) + 1/2), r_min = lambda / K_max, r_max = lambda / K_min; the
  pixel rate in permille is floor(1000 r_tile + 1/2) clipped to [1, 1000];
* that rho_t (the appendix's) lives inside the schedule only; the density
  score of Eq. gauss_score takes the training progress of Alg. 1,
  min(1, t / tau_until);
* random view sampling (the ablation baseline that replaces the
  geometry-aware sampling): K distinct views uniformly at random, draw j
  picking the floor(u m / 2^64)-th of the m views left (ascending), u the
  counter value of (seed, t, 1, V, j).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import binding as B

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def _finalise(z: int) -> int:
    """SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def counter_draw(seed: int, *fields: int) -> int:
    """The 64-bit value of a counter tuple: each field absorbed as
    h <- finalise(h + golden * (field + 1)), from h = seed."""
    h = seed & _M64
    for f in fields:
        h = _finalise((h + _GOLDEN * (f + 1)) & _M64)
    return h


def view_errors(E_maps, pixels: int, dev, views=None, means=None) -> list:
    """E_bar_v of the views' half error maps (one GPU reduction per map, one
    device-to-host copy).  With ``views`` and ``means`` only those views'
    entries of ``means`` are refreshed (the maps of the other views have not
    changed since they were last reduced)."""
    views = list(range(len(E_maps))) if views is None else list(views)
    sums = torch.empty(max(len(views), 1), dtype=torch.int64, device=dev)
    for j, v in enumerate(views):
        B.tgs_view_error_sums(E_maps[v], 1, pixels, sums[j:j + 1])
    out = list(means) if means is not None else [0.0] * len(E_maps)
    for v, s in zip(views, sums.cpu().tolist()):
        out[v] = int(s) / (float(1 << 24) * pixels)
    return out


def _weight(cu, du, ca, da, lam_d, lam_t) -> float:
    dx, dy, dz = cu[0] - ca[0], cu[1] - ca[1], cu[2] - ca[2]
    dist = math.sqrt(dx * dx + dy * dy + dz * dz)
    return math.exp(-lam_d * dist - lam_t * (1.0 - (du[0] * da[0] + du[1] * da[1] + du[2] * da[2])))


def pick_views(stack, means, centres, dirs, K, lam_d, lam_t, seed, t):
    """Anchor and companions of step t; returns (views, stack left)."""
    V = len(means)
    K = min(K, V)
    pool = sorted(stack) if len(stack) >= K else list(range(V))
    anchor = pool[0]
    for u in pool[1:]:
        if means[u] > means[anchor]:
            anchor = u
    views = [anchor]
    cand = [u for u in pool if u != anchor]
    ca, da = [float(x) for x in centres[anchor]], [float(x) for x in dirs[anchor]]
    for j in range(K - 1):
        w = [_weight([float(x) for x in centres[u]], [float(x) for x in dirs[u]], ca, da, lam_d, lam_t)
             for u in cand]
        r = (counter_draw(seed, t, 0, V, j) >> 11) * 2.0 ** -53 * sum(w)
        run, k = 0.0, len(cand) - 1
        for i, wi in enumerate(w):
            run += wi
            if run > r:
                k = i
                break
        views.append(cand.pop(k))
    return views, [u for u in pool if u not in views]


def pick_views_random(V: int, K: int, seed: int, t: int) -> list:
    """Random view sampling: K distinct views, uniformly, in draw order."""
    K = min(K, V)
    rest = list(range(V))
    views = []
    for j in range(K):
        views.append(rest.pop((counter_draw(seed, t, 1, V, j) * len(rest)) >> 64))
    return views


@dataclass
class Schedule:
    tau_until: int = 3500
    K_min: int = 3
    K_max: int = 10
    lam: float = 1.0        # tile sampling scale
    alpha: float = 3.0

    def at(self, t: int, E_t: float, E_init: float) -> tuple:
        """(K_t, pixel rate in permille) of step t."""
        r = min(max(E_t / (E_init + 1e-8), 0.0), 1.0)
        phi = math.sin(math.pi / 2.0 * math.sqrt(r))
        rho = 1.0 - min(max(t / self.tau_until, 0.0), 1.0)
        a = 1.0 - rho * phi
        r_min, r_max = self.lam / self.K_max, self.lam / self.K_min
        r_tile = r_min + (r_max - r_min) * a
        K = int(math.floor(self.K_min + (self.K_max - self.K_min) * math.exp(-self.alpha * a) + 0.5))
        return K, min(max(int(math.floor(1000.0 * r_tile + 0.5)), 1), 1000)


def camera_pose(cam) -> tuple:
    """Centre c = -R^T t and unit viewing direction (the camera's +z axis,
    the third row of the world-to-camera R) of a tgs_camera."""
    R = [[cam.R[3 * i + j] for j in range(3)] for i in range(3)]
    t = [cam.t[i] for i in range(3)]
    c = [-(R[0][k] * t[0] + R[1][k] * t[1] + R[2][k] * t[2]) for k in range(3)]
    d = R[2]
    n = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    return c, [x / n for x in d]


@dataclass
class DensityPlan:
    """When and how density control runs inside the loop (the hyper-parameter
    table: tau_from, tau_until, Delta_dens, Delta_prune, eta_topk, eta_final,
    tau_grad, tau_grad^abs, rho_dense, lambda_base).  Every ``every`` steps in
    [t_from, t_until] the accumulated statistics select and densify; on the
    steps that are also multiples of ``prune_every`` the final pruning keeps
    the top eta_final of the scores.  A densified Gaussian is split when its
    largest scale exceeds percent_dense times the scene extent (1.1 times the
    largest distance of a camera centre from their mean), else cloned.  The
    trainer needs density_stats on."""
    t_from: int = 200
    t_until: int = 3500
    every: int = 100
    prune_every: int = 500
    eta_topk: float = 0.9
    eta_final: float = 0.9
    tau_grad: float = 2e-4
    tau_grad_abs: float = 4e-4
    percent_dense: float = 0.01
    lambda_base: float = 0.8
    seed: int = 11


def scene_extent(cams) -> float:
    """1.1 times the largest distance of a camera centre from the mean centre."""
    cs = [camera_pose(c)[0] for c in cams]
    m = [sum(c[k] for c in cs) / len(cs) for k in range(3)]
    return 1.1 * max(math.sqrt(sum((c[k] - m[k]) ** 2 for k in range(3))) for c in cs)


def density_step(tr, t: int, tau_until: int, plan: DensityPlan, extent: float):
    """One density-control step at iteration t: the score at the training
    progress rho = min(1, t / tau_until) of Alg. 1, the gated selections, the
    topology change (split draws from a seeded generator) and a restart of
    the sums.  Returns (densify mask, keep mask, rho) as used."""
    rho = min(1.0, t / tau_until)
    prune = plan.prune_every > 0 and t % plan.prune_every == 0
    dm, km, _, _ = tr.density_select(plan.lambda_base, rho, plan.eta_topk, plan.eta_final,
                                     tau_grad=plan.tau_grad, tau_grad_abs=plan.tau_grad_abs, prune=prune)
    gen = torch.Generator(device=tr.dev).manual_seed(plan.seed + t)
    z = torch.randn((tr.n, 3), generator=gen, device=tr.dev)
    tr.densify_and_prune(dm, km, z, math.log(plan.percent_dense * extent))
    return dm, km, rho


def run_schedule(tr, steps: int, sch: Schedule, lam_d: float, lam_t: float, seed: int, t0: int = 1,
                 density: DensityPlan | None = None, on_density=None, view_sampling: str = "geometry"):
    """Sparse training driven by the schedule: each step takes K_t and the
    pixel rate from the schedule, picks the anchor and its companions from
    the views' mean errors and runs the step at that rate; afterwards only
    the stepped views' mean errors are reduced again (the other maps are
    unchanged).  With ``density``, every ``every`` steps from ``t_from`` to
    ``t_until`` a density step runs (``density_step``); ``on_density(t, tr)``
    is called just before it (e.g. to read the statistics).
    ``view_sampling`` = "random" replaces the anchor and companion draws by
    random view sampling (``pick_views_random``).  E_bar_init is
    the mean error when the run starts.  Returns the per-step (views, K_t,
    rate in permille, the views' mean errors before the step, Gaussians
    after it)."""
    cams = tr.cams
    pixels = cams[0].width * cams[0].height
    assert all(c.width * c.height == pixels for c in cams), "one image size"
    poses = [camera_pose(c) for c in cams]
    centres, dirs = [p[0] for p in poses], [p[1] for p in poses]
    means = view_errors(tr.E, pixels, tr.dev)
    e_init = sum(means) / len(means)
    extent = scene_extent(cams)
    stack = list(range(len(cams)))
    log = []
    for t in range(t0, t0 + steps):
        K, permille = sch.at(t, sum(means) / len(means), e_init)
        if view_sampling == "random":
            views = pick_views_random(len(cams), K, seed, t)
        elif view_sampling == "geometry":
            views, stack = pick_views(stack, means, centres, dirs, K, lam_d, lam_t, seed, t)
        else:
            raise ValueError(f"unknown view sampling {view_sampling!r}")
        tr.step(views, rate_permille=permille)
        if density is not None and density.t_from <= t <= density.t_until and t % density.every == 0:
            if on_density is not None:
                on_density(t, tr)
            density_step(tr, t, sch.tau_until, density, extent)
        log.append((views, K, permille, means, tr.n))
        means = view_errors(tr.E, pixels, tr.dev, views, means)
    return log
