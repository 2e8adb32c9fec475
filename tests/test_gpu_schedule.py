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
