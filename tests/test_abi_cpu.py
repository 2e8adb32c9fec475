"""The C-ABI library loads and exports every symbol its header declares; host
logic (argument checks, sizes, counts) behaves as documented.  No GPU work:
every call here returns before anything is enqueued."""
import ctypes
import os
import re

import pytest

from oracle.params import pixels_per_tile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "turbogs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tgs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def B():
    from paper_2606_15924_amd import binding
    binding.lib()
    return binding


def test_header_symbols_exported(B):
    names = _declared()
    assert len(names) >= 16
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(B.PROTOTYPES), set(names) ^ set(B.PROTOTYPES)


def test_version_and_counts(B):
    assert B.tgs_version() == 12
    for r in (1, 100, 150, 200, 250, 500, 1000):
        assert B.tgs_pixels_per_tile(r) == pixels_per_tile(r)
    sp = B.sample_params(64, n_tiles_sel=64)
    assert B.tgs_sample_tile_count(256, 256, sp) == 64
    sp.n_tiles_sel = -1
    assert B.tgs_sample_tile_count(840, 1296, sp) == 81 * 53
    sp.n_tiles_sel = 10 ** 6
    assert B.tgs_sample_tile_count(20, 20, sp) == 4


def test_workspace_sizes_grow(B):
    assert B.tgs_sample_workspace_size(256, 256) >= 256 * 8
    a = B.tgs_bin_sort_workspace_size(1000, 10000, 256)
    b = B.tgs_bin_sort_workspace_size(1000, 100000, 256)
    assert 0 < a < b
    assert b >= 100000 * 12


def _null_call(B, name, *args):
    f = getattr(B.lib(), name)
    return f(*args)


def test_invalid_arguments_are_rejected_before_any_launch(B):
    lib = B.lib()
    cam = B.tgs_camera()
    cam.width, cam.height = 64, 48
    rp = B.raster_params()
    # null output pointers
    st = lib.tgs_project(ctypes.c_void_p(16), 10, ctypes.byref(cam), ctypes.byref(rp), None, None, None,
                         None, None, None, None)
    assert st == B.TGS_ERR_INVALID
    assert "null" in lib.tgs_last_error().decode()
    # bad SH degree
    rp.sh_degree = 4
    st = lib.tgs_project(ctypes.c_void_p(16), 10, ctypes.byref(cam), ctypes.byref(rp), None, None, None,
                         None, None, None, None)
    assert st == B.TGS_ERR_INVALID and "sh_degree" in lib.tgs_last_error().decode()
    rp.sh_degree = 3
    # tile grid inconsistent with the image
    st = lib.tgs_render_fwd(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 3, 3, 64, 48,
                            None, None, None, 0, 0, ctypes.byref(rp), ctypes.c_void_p(16),
                            ctypes.c_void_p(16), None, None, None)
    assert st == B.TGS_ERR_INVALID and "tile grid" in lib.tgs_last_error().decode()
    # sampler: n_pix out of range, then too-small workspace
    sp = B.sample_params(300)
    st = lib.tgs_sample(ctypes.c_void_p(16), ctypes.c_void_p(16), 48, 64, ctypes.byref(sp), None,
                        *([ctypes.c_void_p(16)] * 6), 1 << 20, None)
    assert st == B.TGS_ERR_INVALID and "n_pix" in lib.tgs_last_error().decode()
    sp = B.sample_params(64)
    st = lib.tgs_sample(ctypes.c_void_p(16), ctypes.c_void_p(16), 48, 64, ctypes.byref(sp), None,
                        *([ctypes.c_void_p(16)] * 6), 8, None)
    assert st == B.TGS_ERR_INVALID and "workspace" in lib.tgs_last_error().decode()
    # optimizer: step 0 and bad mode
    op = B.optim_params()
    st = lib.tgs_optimizer_step(*([ctypes.c_void_p(16)] * 4), 10, None, ctypes.byref(op), 0, None)
    assert st == B.TGS_ERR_INVALID and "step" in lib.tgs_last_error().decode()
    op.lm_mode = 7
    st = lib.tgs_optimizer_step(*([ctypes.c_void_p(16)] * 4), 10, None, ctypes.byref(op), 1, None)
    assert st == B.TGS_ERR_INVALID
    # misaligned splat record
    st = lib.tgs_render_fwd(ctypes.c_void_p(20), ctypes.c_void_p(16), ctypes.c_void_p(16), 4, 3, 64, 48,
                            None, None, None, 0, 0, ctypes.byref(rp), ctypes.c_void_p(16),
                            ctypes.c_void_p(16), None, None, None)
    assert st == B.TGS_ERR_INVALID and "aligned" in lib.tgs_last_error().decode()


def test_density_and_schedule_arguments_are_rejected_before_any_launch(B):
    lib = B.lib()
    P = ctypes.c_void_p(16)

    def err(st, word):
        assert st == B.TGS_ERR_INVALID and word in lib.tgs_last_error().decode(), lib.tgs_last_error()

    rp = B.raster_params()
    # stats slot array must be 16-byte aligned
    err(lib.tgs_density_accumulate(P, P, P, 4, 3, 64, 48, None, None, None, 0, 0, ctypes.byref(rp), P, P, None,
                                   10, ctypes.c_void_p(20), None), "aligned")
    err(lib.tgs_density_score(P, 10, 0.5, 1.5, 1e-8, None, None, P, None), "rho")
    err(lib.tgs_density_score(P, 10, 0.5, 0.5, 0.0, None, None, P, None), "eps")
    ws = B.tgs_select_workspace_size()
    assert ws >= 256 * 4
    err(lib.tgs_select_kth_largest(P, 10, 0, P, P, ws, None), "k")
    err(lib.tgs_select_kth_largest(P, 10, 11, P, P, ws, None), "k")
    err(lib.tgs_select_kth_largest(P, 10, 3, P, P, 8, None), "workspace")
    nk, nn = ctypes.c_int64(0), ctypes.c_int64(0)
    tws = lib.tgs_density_topology_workspace_size(1000)
    assert tws >= 4 * 4 * 1000
    err(lib.tgs_density_topology_count(P, P, 1000, ctypes.byref(nk), ctypes.byref(nn), P, 16, None), "workspace")
    err(lib.tgs_density_topology_apply(P, P, P, 1000, P, 0.0, P, tws, P, P, P, 2001, None), "n_out")
    err(lib.tgs_grad_screen_accumulate(P, P, 10, 64, 48, ctypes.c_void_p(20), None), "aligned")
    err(lib.tgs_grad_screen_accumulate(P, P, 10, 0, 48, P, None), "image size")
    err(lib.tgs_density_masks(P, ctypes.c_void_p(20), None, 10, P, 1e-4, 2e-4, 1, P, P, None), "aligned")
    err(lib.tgs_view_error_sums(P, 3, 0, P, None), "pixels")
    # empty inputs: nothing to do
    assert lib.tgs_density_score(None, 0, 0.5, 0.5, 1e-8, None, None, None, None) == B.TGS_OK
    assert lib.tgs_grad_screen_accumulate(None, None, 0, 64, 48, None, None) == B.TGS_OK
    assert lib.tgs_density_masks(None, None, None, 0, None, 0.0, 0.0, 0, None, None, None) == B.TGS_OK
    assert lib.tgs_view_error_sums(None, 0, 100, None, None) == B.TGS_OK
    assert lib.tgs_density_topology_apply(P, P, P, 1000, P, 0.0, P, tws, None, None, None, 0, None) == B.TGS_OK


def test_empty_inputs_are_no_ops(B):
    lib = B.lib()
    cam = B.tgs_camera()
    cam.width, cam.height = 64, 48
    rp = B.raster_params()
    assert lib.tgs_project(None, 0, ctypes.byref(cam), ctypes.byref(rp), None, None, None, None, None,
                           None, None) == B.TGS_OK
    op = B.optim_params()
    assert lib.tgs_optimizer_step(None, None, None, None, 0, None, ctypes.byref(op), 1, None) == B.TGS_OK


def test_binding_refuses_host_tensors(B):
    import torch
    with pytest.raises(ValueError):
        B._ptr(torch.zeros(4))
