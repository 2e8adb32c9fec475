"""The host view scheduler against the oracle (CPU only): the same view sets
step after step, and the same view budget and pixel rate."""
import numpy as np

from oracle import schedule as S
from paper_2606_15924_amd import schedule as H


def test_counter_draws_equal_the_oracle_generator():
    from oracle import rng
    for f in [(1, 2, 3, 4), (0, 0, 0, 0), (2 ** 40, 7, 99, 3)]:
        assert H.counter_draw(12345, *f) == rng.draw(12345, *f)


def test_view_sets_equal_the_oracle_over_many_steps():
    gen = np.random.default_rng(2)
    V = 40
    c = gen.normal(size=(V, 3))
    d = gen.normal(size=(V, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    means = list(gen.uniform(0, 1, V))
    means[7] = means[3]                               # a tie: the lower index wins
    so, sh = list(range(V)), list(range(V))
    for t in range(300):
        K = 3 + t % 8
        vo, so = S.select_views(so, means, c, d, K, 0.8, 1.5, seed=4, t=t)
        vh, sh = H.pick_views(sh, means, c, d, K, 0.8, 1.5, seed=4, t=t)
        assert vo == vh and so == sh, t
        means[vo[0]] *= 0.9                           # the anchor's error drops after training


def test_schedule_equals_the_oracle():
    sch = H.Schedule(tau_until=3500, K_min=3, K_max=10, lam=0.8, alpha=3.0)
    for t in range(0, 5000, 37):
        for e in (1.2, 1.0, 0.6, 0.2, 0.01):
            ref = S.schedule(t, e, 1.0, 3500, 3, 10, 0.8, 3.0)
            assert sch.at(t, e, 1.0) == (ref["K"], ref["permille"])


def test_camera_pose_matches_the_oracle_centre_and_looks_at_the_target():
    import synth
    from oracle import project
    from paper_2606_15924_amd.binding import camera
    for eye in [(2.4, -1.1, 1.3), (0.0, 0.0, 3.0), (-1.0, 2.0, 0.5)]:
        cam = synth.look_at(eye, fx=300.0, fy=300.0, width=64, height=48)
        c, d = H.camera_pose(camera(cam))
        assert np.allclose(c, project.camera_center(cam), atol=1e-12)
        # a look-at camera views the origin: the direction points from the centre to it
        to_origin = -np.asarray(c) / np.linalg.norm(c)
        assert np.allclose(d, to_origin, atol=1e-9), (eye, d, to_origin)


def test_view_sets_at_the_edges():
    c = np.zeros((3, 3))
    d = np.tile([0.0, 0.0, 1.0], (3, 1))
    means = [0.2, 0.2, 0.1]
    for K in (1, 3, 7):                                  # K above the view count is clamped
        vo, so = S.select_views([], means, c, d, K, 1.0, 1.0, seed=2, t=1)
        vh, sh = H.pick_views([], means, c, d, K, 1.0, 1.0, seed=2, t=1)
        assert vo == vh and so == sh and vh[0] == 0 and len(vh) == min(K, 3)
    assert H.pick_views([0], [0.5], [[0, 0, 0]], [[0, 0, 1]], 1, 1.0, 1.0, 0, 0) == ([0], [])


def test_random_view_sampling_equals_the_oracle():
    for t in range(300):
        for V, K in ((150, 3), (150, 10), (7, 7), (4, 9)):
            assert H.pick_views_random(V, K, 5, t) == S.random_views(V, K, 5, t)
