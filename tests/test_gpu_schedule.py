"""GPU per-view error sums for the anchor view (Sec. 3.4, Eq. anchor_view):
exact, so bit for bit against the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import schedule as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15924_amd import binding
    binding.lib()
    return binding


def test_view_error_sums_exact(B):
    H, W, V = 840, 1296, 3
    maps = [synth.error_map(H, W, 300 + v) for v in range(V)]
    maps[1] = maps[1].copy()
    flat = maps[1].reshape(-1)
    flat[:5] = np.array([np.inf, np.nan, -1.0, 2.0 ** -24, 65504.0], np.float16).view(np.uint16)
    E = torch.from_numpy(np.stack(maps).view(np.int16)).cuda()
    sums = torch.empty(V, dtype=torch.int64, device="cuda")
    B.tgs_view_error_sums(E, V, H * W, sums)
    got = sums.cpu().numpy().astype(np.uint64)
    for v in range(V):
        assert int(got[v]) == S.half_weight_sum(maps[v]), v


def test_host_view_errors_equal_the_oracle_means(B):
    from paper_2606_15924_amd.schedule import view_errors
    H, W = 256, 256
    maps = [synth.error_map(H, W, 310 + v) for v in range(4)]
    got = view_errors([torch.from_numpy(m.view(np.int16)).cuda() for m in maps], H * W, "cuda")
    assert got == [S.mean_view_error(m) for m in maps]


def test_schedule_driven_training(B):
    """Twelve steps of sparse training driven by the schedule on four views:
    each step trains K_t distinct views at the scheduled rate, the first
    anchor is the view of largest mean error, and the maps and parameters
    move."""
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    from paper_2606_15924_amd.schedule import Schedule, run_schedule
    from support import scene_c1
    p, cams = scene_c1()
    H, W = cams[0].height, cams[0].width
    gts = [torch.from_numpy(synth.image(H, W, 320 + k)).cuda() for k in range(len(cams))]
    E = [torch.zeros((H, W), dtype=torch.int16, device="cuda") for _ in cams]
    A = [torch.zeros((H, W), dtype=torch.int16, device="cuda") for _ in cams]
    tr = Trainer(torch.from_numpy(p).cuda(), cams, gts, StepConfig(rate_permille=250), E=E, A=A)
    tr.init_error_maps(list(range(len(cams))))
    p0 = tr.params.clone()
    sch = Schedule(tau_until=10, K_min=1, K_max=3, lam=0.75, alpha=3.0)
    log = run_schedule(tr, 12, sch, lam_d=0.5, lam_t=1.0, seed=7)
    for t, (views, K, permille, means, _) in enumerate(log, start=1):
        assert len(views) == K == len(set(views)) and 1 <= K <= 3
        assert 250 <= permille <= 750                       # r_min = 0.25, r_max = 0.75
        assert all(0 <= v < 4 for v in views)
    e_init = float(np.mean(log[0][3]))
    for t, (views, K, permille, means, _) in enumerate(log, start=1):
        assert (K, permille) == sch.at(t, float(np.mean(means)), e_init), t
    views, K, permille, means, _ = log[0]
    assert K == 2 and permille == 300                       # t = 1: rho = 0.9, phi = 1, a = 0.1
    assert views[0] == int(np.argmax(means))
    assert log[-1][1] == 1 and log[-1][2] == 750            # after tau_until: a = 1
    assert torch.isfinite(tr.params).all() and not torch.equal(tr.params, p0)
    # buffers: one set per slot, keyed by the slot, at the last step's pixels per tile
    assert sorted(tr._bufs) == list(range(len(tr._bufs))) and len(tr._bufs) <= 3
    assert tr._bufs[0].n_pix == B.tgs_pixels_per_tile(log[-1][2])


def test_schedule_driven_training_with_random_view_sampling(B):
    """The same loop with random view sampling (the ablation baseline): each
    step trains the oracle's uniform draw of K_t distinct views, K_t and the
    rate still from the schedule."""
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    from paper_2606_15924_amd.schedule import Schedule, run_schedule
    from support import scene_c1
    p, cams = scene_c1()
    H, W = cams[0].height, cams[0].width
    gts = [torch.from_numpy(synth.image(H, W, 330 + k)).cuda() for k in range(len(cams))]
    E = [torch.zeros((H, W), dtype=torch.int16, device="cuda") for _ in cams]
    A = [torch.zeros((H, W), dtype=torch.int16, device="cuda") for _ in cams]
    tr = Trainer(torch.from_numpy(p).cuda(), cams, gts, StepConfig(rate_permille=250), E=E, A=A)
    tr.init_error_maps(list(range(len(cams))))
    p0 = tr.params.clone()
    sch = Schedule(tau_until=10, K_min=1, K_max=3, lam=0.75, alpha=3.0)
    log = run_schedule(tr, 12, sch, lam_d=0.5, lam_t=1.0, seed=8, view_sampling="random")
    e_init = float(np.mean(log[0][3]))
    for t, (views, K, permille, means, _) in enumerate(log, start=1):
        assert views == S.random_views(len(cams), K, 8, t), t
        assert (K, permille) == sch.at(t, float(np.mean(means)), e_init), t
    assert torch.isfinite(tr.params).all() and not torch.equal(tr.params, p0)


def test_schedule_driven_training_with_density_control(B):
    """The loop with density control every four steps from step 4 to 10 and
    final pruning at step 8 only: the Gaussian count changes only there, and
    at each density step the selections equal the oracle's on the same
    statistics: the score at the training progress rho = t / tau_until of
    Alg. 1 (lambda_eff = lambda_base (1 - rho)), the percentile thresholds,
    the gradient gate, and n_out = #keep + #(keep and densify)."""
    from oracle import density as D
    from paper_2606_15924_amd.pipeline import StepConfig, Trainer
    from paper_2606_15924_amd.schedule import DensityPlan, Schedule, run_schedule, scene_extent
    from support import scene_c1
    p, cams = scene_c1()
    H, W = cams[0].height, cams[0].width
    gts = [torch.from_numpy(synth.image(H, W, 330 + k)).cuda() for k in range(len(cams))]
    E = [torch.zeros((H, W), dtype=torch.int16, device="cuda") for _ in cams]
    A = [torch.zeros((H, W), dtype=torch.int16, device="cuda") for _ in cams]
    tr = Trainer(torch.from_numpy(p).cuda(), cams, gts, StepConfig(rate_permille=250, density_stats=True),
                 E=E, A=A)
    tr.init_error_maps(list(range(len(cams))))
    n0 = tr.n
    plan = DensityPlan(t_from=4, t_until=10, every=4, prune_every=8, eta_topk=0.9, eta_final=0.95,
                       tau_grad=1e-5, tau_grad_abs=2e-5, percent_dense=0.005, lambda_base=0.8)
    tau_until = 10
    seen = {}

    def check(t, tr):
        st = tr.dstats.cpu().numpy().astype(np.float64)
        gs = tr.gstats.cpu().numpy()
        rho = t / tau_until
        sc = D.score(st[:, :3].T, plan.lambda_base, rho)
        assert abs(sc["lambda_eff"] - plan.lambda_base * (1 - rho)) < 1e-15
        gate = D.gradient_gate(gs, st[:, 3], plan.tau_grad, plan.tau_grad_abs)
        # the selection on the GPU's FP32 scores (the score itself is pinned
        # elsewhere to 1e-6): thresholds and masks bit for bit
        dm, km, thr, (_, _, s32) = tr.density_select(plan.lambda_base, rho, plan.eta_topk, plan.eta_final,
                                                     tau_grad=plan.tau_grad, tau_grad_abs=plan.tau_grad_abs,
                                                     prune=t % plan.prune_every == 0)
        s32 = s32.cpu().numpy()
        assert np.allclose(s32, sc["s"], rtol=1e-5, atol=1e-7)
        want = D.select_masks(s32, plan.eta_topk, plan.eta_final, gate=gate, prune=t % plan.prune_every == 0)
        assert np.array_equal(thr.cpu().numpy(), np.array([want["thr_densify"], want["thr_keep"]], np.float32))
        assert np.array_equal(dm.cpu().numpy().astype(bool), want["densify"])
        assert np.array_equal(km.cpu().numpy().astype(bool), want["keep"])
        seen[t] = (int(want["keep"].sum()) + int(want["densify"].sum()), int(want["densify"].sum()))

    log = run_schedule(tr, 12, Schedule(tau_until=tau_until, K_min=1, K_max=3, lam=0.75), 0.5, 1.0, seed=7,
                       density=plan, on_density=check)
    counts = [n0] + [entry[4] for entry in log]
    changed = [t for t in range(1, 13) if counts[t] != counts[t - 1]]
    assert sorted(seen) == [4, 8] and changed == [4, 8]
    for t in (4, 8):
        assert counts[t] == seen[t][0] and seen[t][1] > 0
    assert counts[8] < counts[7] + seen[8][1]                # step 8 prunes
    assert counts[4] == counts[3] + seen[4][1]               # step 4 only densifies
    assert abs(scene_extent(tr.cams) - 1.1 * 3.0) < 1e-9     # tetrahedron cameras at radius 3
    assert tr.n == counts[-1] and tr.params.shape == (59, tr.n) and tr.dstats.shape == (tr.n, 4)
    assert torch.isfinite(tr.params).all()
