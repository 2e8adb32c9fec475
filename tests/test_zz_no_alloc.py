"""The sampler entry point that allocates nothing (tgs_sample_noalloc,
static per-GPU scratch) against tgs_sample with a caller workspace: two
calls in a row, the second on a smaller image, with the tile pass drawing
from the error map and then from predicted tile errors; every output bit
for bit.  And the size limit: an image of more tiles than the static
scratch holds is rejected before anything is queued."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_15924_amd import binding
    binding.lib()
    return binding


def _sample(B, noalloc, E, A, H, W, sp, pred):
    n_st = B.tgs_sample_tile_count(H, W, sp)
    n_t = ((W + 15) // 16) * ((H + 15) // 16)
    d = torch.device("cuda")
    vt = torch.full((max(n_st, 1),), -7, dtype=torch.int32, device=d)
    off = torch.full((n_st + 1,), -7, dtype=torch.int32, device=d)
    pix = torch.zeros(max(n_st * sp.n_pix, 1), dtype=torch.uint8, device=d)
    slot = torch.full((n_t,), -7, dtype=torch.int32, device=d)
    totals = torch.zeros(2, dtype=torch.int64, device=d)
    if noalloc:
        B.tgs_sample_noalloc(E, A, H, W, sp, vt, off, pix, slot, totals, tile_pred=pred)
    else:
        ws = torch.empty(B.tgs_sample_workspace_size(H, W), dtype=torch.uint8, device=d)
        B.tgs_sample(E, A, H, W, sp, vt, off, pix, slot, totals, ws, tile_pred=pred)
    torch.cuda.synchronize()
    P = int(off[-1].item())
    return vt.cpu().numpy(), off.cpu().numpy(), pix[:P].cpu().numpy(), slot.cpu().numpy(), totals.cpu().numpy()


def test_sample_noalloc_matches_sample_on_two_calls(B):
    cases = [(840, 1296, 64, 1073, False), (256, 200, 51, 40, True)]   # the second call is smaller
    for k, (H, W, n_pix, n_sel, with_pred) in enumerate(cases):
        print(f"noalloc sampler case {k}: {W}x{H}, {n_pix} px, {n_sel} tiles, pred={with_pred}", flush=True)
        E = torch.from_numpy(synth.error_map(H, W, 81 + k).view(np.int16)).cuda()
        A = torch.from_numpy(synth.age_map(H, W, 91 + k).view(np.int16)).cuda()
        n_t = ((W + 15) // 16) * ((H + 15) // 16)
        pred = None
        if with_pred:
            pred = torch.from_numpy(np.random.default_rng(k).uniform(0, 2, n_t).astype(np.float32)).cuda()
        sp = B.sample_params(n_pix, n_tiles_sel=n_sel, seed=3, step=5 + k, view=2)
        want = _sample(B, False, E, A, H, W, sp, pred)
        got = _sample(B, True, E, A, H, W, sp, pred)
        assert want[1][-1] > 0 and want[0].size == n_sel
        for a, b in zip(got, want):
            assert np.array_equal(a, b)


def test_sample_noalloc_rejects_images_beyond_its_scratch(B):
    d = torch.device("cuda")
    t = torch.zeros(16, dtype=torch.int32, device=d)
    sp = B.sample_params(64, n_tiles_sel=10)
    with pytest.raises(RuntimeError, match="exceed the static scratch"):
        B.tgs_sample_noalloc(t, t, 4112, 4112, sp, t, t, t, t, torch.zeros(2, dtype=torch.int64, device=d))
