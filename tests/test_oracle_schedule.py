"""Pins of the training-loop scheduling oracle (Sec. 3.4, App. A) against
closed forms, brute force and the limits the formulas fix (CPU only)."""
import math

import numpy as np

from oracle import schedule as S


def test_mean_view_error_exact():
    E = np.array([[0.5, 1.0], [np.inf, -2.0]], dtype=np.float16)
    assert S.mean_view_error(E.view(np.uint16)) == 1.5 / 4
    rng = np.random.default_rng(3)
    E = rng.uniform(0, 3, (64, 48)).astype(np.float16)
    assert abs(S.mean_view_error(E.view(np.uint16)) - E.astype(np.float64).mean()) < 1e-15
    tiny = np.full((4, 4), np.float16(2.0 ** -24))                 # the smallest subnormal
    assert S.half_weight_sum(tiny.view(np.uint16)) == 16


def test_schedule_limits_and_closed_forms():
    # start of training at the initial error: r = 1, phi = 1, rho = 1 -> a = 0:
    # the most views at the lowest per-view rate
    s = S.schedule(0, 1.0, 1.0, 3500, 3, 10, 1.0, 3.0, eps=0.0)
    assert s["phi"] == 1.0 and s["rho"] == 1.0
    assert s["K"] == 10 and abs(s["r_tile"] - 0.1) < 1e-15 and s["permille"] == 100
    # after tau_until: rho = 0 -> a = 1 whatever the error
    s = S.schedule(4000, 0.3, 1.0, 3500, 3, 10, 1.0, 3.0)
    assert s["rho"] == 0.0 and abs(s["r_tile"] - 1 / 3) < 1e-15 and s["permille"] == 333
    assert s["K"] == round(3 + 7 * math.exp(-3.0))                 # 3.35 -> 3
    # halfway, error ratio 1/4: phi = sin(pi/4)
    s = S.schedule(1750, 0.25, 1.0, 3500, 3, 10, 0.5, 3.0, eps=0.0)
    a = 1 - 0.5 * math.sqrt(0.5)
    assert abs(s["phi"] - math.sqrt(0.5)) < 1e-15
    assert abs(s["r_tile"] - (0.05 + (0.5 / 3 - 0.05) * a)) < 1e-15
    assert s["K"] == math.floor(3 + 7 * math.exp(-3 * a) + 0.5)
    # the error ratio is clipped
    assert S.schedule(10, 5.0, 1.0, 3500, 3, 10, 1.0, 3.0)["r"] == 1.0


def test_view_selection_brute_force_frequencies():
    """Companion draws follow pi(u | v*): over many steps the first
    companion's frequencies match the normalised weights."""
    rng = np.random.default_rng(5)
    V = 6
    c = rng.normal(size=(V, 3))
    d = rng.normal(size=(V, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    means = [0.1, 0.5, 0.2, 0.3, 0.05, 0.4]
    w = np.array([S.view_weight(c[u], d[u], c[1], d[1], 0.7, 2.0) for u in range(V) if u != 1])
    counts = np.zeros(V - 1)
    T = 4000
    for t in range(T):
        views, _ = S.select_views(list(range(V)), means, c, d, 2, 0.7, 2.0, seed=9, t=t)
        assert views[0] == 1                                         # the anchor: largest mean error
        counts[[u for u in range(V) if u != 1].index(views[1])] += 1
    p = w / w.sum()
    assert np.all(np.abs(counts / T - p) < 4 * np.sqrt(p * (1 - p) / T) + 1e-3)


def test_stack_refills_and_draws_without_replacement():
    V = 7
    c = np.eye(3)[np.arange(V) % 3] * (1 + np.arange(V))[:, None]
    d = np.eye(3)[np.arange(V) % 3]
    means = list(np.linspace(0.1, 0.7, V))
    stack = list(range(V))
    seen = []
    for t in range(3):
        views, stack = S.select_views(stack, means, c, d, 3, 1.0, 1.0, seed=1, t=t)
        assert len(set(views)) == 3
        seen.append(views)
    # first step: the stack holds every view; the anchor is view 6; second
    # step draws from the four left; third finds one view left and refills
    assert seen[0][0] == 6 and set(seen[0]).isdisjoint(seen[1])
    assert seen[2][0] == 6


def test_random_view_sampling_is_uniform_without_replacement():
    """Random view sampling: K distinct views per step; over many steps each
    view is drawn with frequency K/V, and on V = 4, K = 2 each of the six
    unordered pairs with frequency 1/6 (chi-squared, seeded)."""
    from scipy.stats import chi2
    V, K, T = 30, 7, 3000
    counts = np.zeros(V)
    for t in range(T):
        v = S.random_views(V, K, seed=9, t=t)
        assert len(v) == K == len(set(v)) and all(0 <= x < V for x in v)
        counts[v] += 1
    exp = T * K / V
    stat = ((counts - exp) ** 2 / exp).sum()
    assert stat < chi2.ppf(0.999, V - 1)
    pairs = {}
    for t in range(6000):
        a, b = sorted(S.random_views(4, 2, seed=10, t=t))
        pairs[(a, b)] = pairs.get((a, b), 0) + 1
    assert len(pairs) == 6
    c = np.array(list(pairs.values()), dtype=float)
    assert ((c - 1000) ** 2 / 1000).sum() < chi2.ppf(0.999, 5)
    assert sorted(S.random_views(5, 9, seed=1, t=0)) == list(range(5))
