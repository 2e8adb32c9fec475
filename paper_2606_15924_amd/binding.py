"""ctypes binding of ``libturbogs.so`` with the C entry points' names.

Argument marshalling only: tensors are passed as device pointers
(``data_ptr()``), records as ctypes structures, and every call runs on
torch's current HIP stream.  All work happens in the HIP kernels; a missing
library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libturbogs.so")

TGS_OK = 0
TGS_ERR_CAPACITY = 1
TGS_ERR_INVALID = -1
TGS_ERR_HIP = -2
SPLAT_FLOATS = 12
G2D_FLOATS = 9
PARAM_ROWS = 59
MOMENT_STRIDE = 64   # floats per Gaussian in the optimizer moments m, v ([n][64], Gaussian-major)
TILE = 16
COUNTER_SLOTS = 64
RENDER_CHUNKS = 8
RENDER_CHUNK_LEN = 32


class tgs_camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class tgs_raster_params(ctypes.Structure):
    _fields_ = [("sh_degree", ctypes.c_int32), ("z_near", ctypes.c_float), ("dilation", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("T_min", ctypes.c_float),
                ("bg", ctypes.c_float * 3)]


class tgs_sample_params(ctypes.Structure):
    _fields_ = [("n_pix", ctypes.c_int32), ("hard_permille", ctypes.c_int32),
                ("stable_permille", ctypes.c_int32), ("n_tiles_sel", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("step", ctypes.c_uint64), ("view", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class tgs_loss_params(ctypes.Structure):
    _fields_ = [("eps_charb", ctypes.c_float), ("eps_ncc", ctypes.c_float), ("eps_lambda", ctypes.c_float),
                ("structure", ctypes.c_int32)]


STRUCTURE = {"ncc": 0, "ssim": 1}   # TGS_STRUCTURE_NCC, TGS_STRUCTURE_SSIM


class tgs_optim_params(ctypes.Structure):
    _fields_ = [("lr_mean", ctypes.c_double), ("lr_scale", ctypes.c_double), ("lr_quat", ctypes.c_double),
                ("lr_opacity", ctypes.c_double), ("lr_sh_dc", ctypes.c_double),
                ("lr_sh_rest", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps_adam", ctypes.c_double), ("eps_lm", ctypes.c_double), ("lm_mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class CapacityError(RuntimeError):
    def __init__(self, msg: str, required: int):
        super().__init__(msg)
        self.required = required


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

PROTOTYPES = {
    "tgs_version": (ctypes.c_uint32, []),
    "tgs_last_error": (ctypes.c_char_p, []),
    "tgs_pixels_per_tile": (_I32, [_I32]),
    "tgs_check_finite": (_I32, [_P, _I64, _P, _P]),
    "tgs_bin_sort_async": (_I32, [_P, _P, _P, _I64, _P, _I32, _I32, ctypes.c_float, _P, _P, _I64, _P, _P, _P, _P,
                                  _SZ, _P]),
    "tgs_bin_sort_prefix_async": (_I32, [_P, _P, _P, _I64, _P, _I32, _I32, ctypes.c_float, _I64, _P, _P, _I64, _P,
                                         _P, _P, _P, _SZ, _P]),
    "tgs_bin_sort_continue_async": (_I32, [_P, _I64, _P, _P, _I32, _I32, ctypes.c_float, _I64, _I64, _P, _SZ, _P,
                                           _I64, _P, _P, _P, _SZ, _P]),
    "tgs_render_fwd_prefix": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                     ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P, _P, _P]),
    "tgs_render_fwd_cont": (_I32, [_P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                   ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P, _P]),
    "tgs_render_bwd2": (_I32, [_P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                               ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P, _P, _I64, _P, _P]),
    "tgs_density_accumulate2": (_I32, [_P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                       ctypes.POINTER(tgs_raster_params), _P, _P, _P, _I64, _P, _P]),
    "tgs_sample_noalloc": (_I32, [_P, _P, _I32, _I32, ctypes.POINTER(tgs_sample_params), _P, _P, _P, _P, _P, _P,
                                  _P]),
    "tgs_render_bwd_det_workspace_size": (_SZ, [_I64, _I32, _I32]),
    "tgs_render_bwd_deterministic": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                            ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P, _P, _P,
                                            _I64, _I64, _P, _SZ, _P]),
    "tgs_project_f64": (_I32, [_P, _I64, ctypes.POINTER(tgs_camera), ctypes.POINTER(tgs_raster_params),
                               _P, _P, _P, _P, _P, _P, _P]),
    "tgs_render_fwd_f64": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                  ctypes.POINTER(tgs_raster_params), _P, _P, _P]),
    "tgs_render_bwd_f64": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                  ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P]),
    "tgs_project_bwd_f64": (_I32, [_P, _I64, ctypes.POINTER(tgs_camera), ctypes.POINTER(tgs_raster_params),
                                   _P, _P, _P, _P, _I32, _P]),
    "tgs_sample_tile_count": (_I32, [_I32, _I32, ctypes.POINTER(tgs_sample_params)]),
    "tgs_project": (_I32, [_P, _I64, ctypes.POINTER(tgs_camera), ctypes.POINTER(tgs_raster_params),
                           _P, _P, _P, _P, _P, _P, _P]),
    "tgs_sample_workspace_size": (_SZ, [_I32, _I32]),
    "tgs_sample": (_I32, [_P, _P, _I32, _I32, ctypes.POINTER(tgs_sample_params), _P, _P, _P, _P, _P, _P,
                          _P, _SZ, _P]),
    "tgs_bin_sort_workspace_size": (_SZ, [_I64, _I64, _I32]),
    "tgs_bin_sort": (_I32, [_P, _P, _P, _I64, _P, _I32, _I32, ctypes.c_float, _P, _P, _I64, _P, _P,
                            ctypes.POINTER(_I64), _P, _SZ, _P]),
    "tgs_render_state_size": (_SZ, [_I32, _I32]),
    "tgs_render_fwd": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                              ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P]),
    "tgs_render_bwd": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                              ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P, _P]),
    "tgs_loss": (_I32, [_P, _P, _I32, _I32, _P, _P, _P, _I32, _P, ctypes.POINTER(tgs_loss_params),
                        _P, _P, _P, _P, _P]),
    "tgs_ema_age_update": (_I32, [_P, _P, _I32, _I32, _P, _P, _P, _P, ctypes.c_float, _P]),
    "tgs_error_init": (_I32, [_P, _P, _I32, _I32, _P, _P]),
    "tgs_density_accumulate": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                      ctypes.POINTER(tgs_raster_params), _P, _P, _P, _I64, _P, _P]),
    "tgs_render_bwd_density": (_I32, [_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _I32,
                                      ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P, _P, _I64, _P,
                                      _P]),
    "tgs_density_score": (_I32, [_P, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P, _P, _P, _P]),
    "tgs_density_topology_workspace_size": (_SZ, [_I64]),
    "tgs_density_topology_count": (_I32, [_P, _P, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64), _P, _SZ, _P]),
    "tgs_density_topology_apply": (_I32, [_P, _P, _P, _I64, _P, ctypes.c_float, _P, _SZ, _P, _P, _P, _I64, _P]),
    "tgs_grad_screen_accumulate": (_I32, [_P, _P, _I64, _I32, _I32, _P, _P]),
    "tgs_density_masks": (_I32, [_P, _P, _P, _I64, _P, ctypes.c_float, ctypes.c_float, _I32, _P, _P, _P]),
    "tgs_grad_screen_mean": (_I32, [_P, _I64, _P, _P]),
    "tgs_view_error_sums": (_I32, [_P, _I32, _I64, _P, _P]),
    "tgs_select_workspace_size": (_SZ, []),
    "tgs_select_kth_largest": (_I32, [_P, _I64, _I64, _P, _P, _SZ, _P]),
    "tgs_threshold_mask": (_I32, [_P, _I64, _P, _P, _P]),
    "tgs_project_bwd": (_I32, [_P, _I64, ctypes.POINTER(tgs_camera), ctypes.POINTER(tgs_raster_params),
                               _P, _P, _P, _P, _I32, _P]),
    "tgs_optimizer_step": (_I32, [_P, _P, _P, _P, _I64, _P, ctypes.POINTER(tgs_optim_params), _I64, _P]),
    "tgs_tile_features": (_I32, [_P, _P, _P, _I32, _I32, ctypes.POINTER(tgs_camera), _P, _P]),
    "tgs_tile_mlp_fwd": (_I32, [_P, _P, _I64, _P, _P, _P]),
    "tgs_tile_mlp_workspace_size": (_SZ, [_I64]),
    "tgs_tile_mlp_train_step": (_I32, [_P, _P, _P, _P, _P, _P, _P, _I64, _I64, ctypes.c_float, _P, _P, _SZ, _P]),
    "tgs_project_bwd_optimizer_workspace_size": (_SZ, [_I64]),
    "tgs_project_bwd_optimizer_views_workspace_size": (_SZ, [_I64, _I32]),
    "tgs_project_bwd_optimizer_step_views": (_I32, [_P, _I64, _I32, ctypes.POINTER(tgs_camera),
                                                    ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P,
                                                    ctypes.POINTER(tgs_optim_params), _I64, _P, _SZ, _P]),
    "tgs_project_bwd_optimizer_step": (_I32, [_P, _I64, ctypes.POINTER(tgs_camera),
                                              ctypes.POINTER(tgs_raster_params), _P, _P, _P, _P, _P, _P, _P,
                                              ctypes.POINTER(tgs_optim_params), _I64, _P, _SZ, _P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_15924_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(status: int, name: str, required: int | None = None):
    if status == TGS_OK:
        return
    msg = lib().tgs_last_error().decode()
    if status == TGS_ERR_CAPACITY:
        raise CapacityError(f"{name}: {msg}", int(required or 0))
    raise RuntimeError(f"{name} failed ({status}): {msg}")


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream():
    # the raw handle of the current stream (no Stream object per call)
    return ctypes.c_void_p(torch._C._cuda_getCurrentRawStream(torch.cuda.current_device()))


# ------------------------------------------------------------------ records
def camera(cam) -> tgs_camera:
    """A ``tgs_camera`` from any object with R, t, fx, fy, cx, cy, width, height."""
    c = tgs_camera()
    R = [float(v) for row in cam.R for v in row]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = float(cam.t[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def raster_params(sh_degree=3, z_near=0.2, dilation=0.3, alpha_min=1.0 / 255.0, alpha_max=0.99,
                  T_min=1e-4, bg=(0.0, 0.0, 0.0)) -> tgs_raster_params:
    r = tgs_raster_params()
    r.sh_degree, r.z_near, r.dilation = sh_degree, z_near, dilation
    r.alpha_min, r.alpha_max, r.T_min = alpha_min, alpha_max, T_min
    for i in range(3):
        r.bg[i] = bg[i]
    return r


def sample_params(n_pix, hard_permille=400, stable_permille=300, n_tiles_sel=-1, seed=0, step=0,
                  view=0) -> tgs_sample_params:
    s = tgs_sample_params()
    s.n_pix, s.hard_permille, s.stable_permille, s.n_tiles_sel = n_pix, hard_permille, stable_permille, n_tiles_sel
    s.seed, s.step, s.view = seed, step, view
    return s


def loss_params(eps_charb=1e-3, eps_ncc=1e-6, eps_lambda=1e-8, structure="ncc") -> tgs_loss_params:
    """Loss constants; ``structure`` is the tile term, "ncc" (S-NCC) or "ssim" (S-SSIM)."""
    p = tgs_loss_params()
    p.eps_charb, p.eps_ncc, p.eps_lambda = eps_charb, eps_ncc, eps_lambda
    p.structure = STRUCTURE[structure] if isinstance(structure, str) else int(structure)
    return p


def optim_params(lr_mean=1.6e-4, lr_scale=5e-3, lr_quat=1e-3, lr_opacity=2.5e-2, lr_sh_dc=2.5e-3,
                 lr_sh_rest=2.5e-3 / 20.0, beta1=0.9, beta2=0.999, eps_adam=1e-15, eps_lm=1e-8,
                 lm_mode=0) -> tgs_optim_params:
    o = tgs_optim_params()
    o.lr_mean, o.lr_scale, o.lr_quat, o.lr_opacity = lr_mean, lr_scale, lr_quat, lr_opacity
    o.lr_sh_dc, o.lr_sh_rest, o.beta1, o.beta2 = lr_sh_dc, lr_sh_rest, beta1, beta2
    o.eps_adam, o.eps_lm, o.lm_mode = eps_adam, eps_lm, lm_mode
    return o


# ------------------------------------------------------------------ entry points
def tgs_version() -> int:
    return int(lib().tgs_version())


def tgs_check_finite(x, count):
    """count (one device int64) <- number of NaN / infinite entries of x (float32)."""
    if x.dtype != torch.float32 or count.dtype != torch.int64:
        raise TypeError("tgs_check_finite: x float32, count int64")
    _check(lib().tgs_check_finite(_ptr(x), x.numel(), _ptr(count), _stream()), "tgs_check_finite")


def check_finite(x) -> int:
    """The number of non-finite entries of a float32 device tensor (synchronises)."""
    count = torch.empty(1, dtype=torch.int64, device=x.device)
    tgs_check_finite(x, count)
    return int(count.item())


def tgs_pixels_per_tile(rate_permille: int) -> int:
    return int(lib().tgs_pixels_per_tile(rate_permille))


def tgs_sample_tile_count(height: int, width: int, sp: tgs_sample_params) -> int:
    return int(lib().tgs_sample_tile_count(height, width, ctypes.byref(sp)))


def tgs_project(params, n, cam: tgs_camera, rp: tgs_raster_params, splat, depth, radius, rect, clamp,
                g2d_clear=None):
    _check(lib().tgs_project(_ptr(params), n, ctypes.byref(cam), ctypes.byref(rp), _ptr(splat), _ptr(depth),
                             _ptr(radius), _ptr(rect), _ptr(clamp), _ptr(g2d_clear), _stream()), "tgs_project")


def tgs_project_f64(params, n, cam: tgs_camera, rp: tgs_raster_params, rec64, splat, depth, radius, rect, clamp):
    _check(lib().tgs_project_f64(_ptr(params), n, ctypes.byref(cam), ctypes.byref(rp), _ptr(rec64), _ptr(splat),
                                 _ptr(depth), _ptr(radius), _ptr(rect), _ptr(clamp), _stream()), "tgs_project_f64")


def tgs_render_fwd_f64(rec64, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                       n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib):
    _check(lib().tgs_render_fwd_f64(_ptr(rec64), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height,
                                    _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                    ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _stream()), "tgs_render_fwd_f64")


def tgs_render_bwd_f64(rec64, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                       n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib, dL, g2d):
    _check(lib().tgs_render_bwd_f64(_ptr(rec64), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height,
                                    _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                    ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _ptr(dL), _ptr(g2d), _stream()),
           "tgs_render_bwd_f64")


def tgs_project_bwd_f64(params, n, cam: tgs_camera, rp: tgs_raster_params, radius, clamp, g2d, grad,
                        accumulate: bool = False):
    _check(lib().tgs_project_bwd_f64(_ptr(params), n, ctypes.byref(cam), ctypes.byref(rp), _ptr(radius),
                                     _ptr(clamp), _ptr(g2d), _ptr(grad), int(bool(accumulate)), _stream()),
           "tgs_project_bwd_f64")


def tgs_sample_workspace_size(height: int, width: int) -> int:
    return int(lib().tgs_sample_workspace_size(height, width))


def tgs_sample(E, A, height, width, sp: tgs_sample_params, valid_tiles, tile_off, pix, tile_slot,
               totals, ws, tile_pred=None):
    _check(lib().tgs_sample(_ptr(E), _ptr(A), height, width, ctypes.byref(sp), _ptr(tile_pred), _ptr(valid_tiles),
                            _ptr(tile_off), _ptr(pix), _ptr(tile_slot), _ptr(totals), _ptr(ws),
                            ws.numel() * ws.element_size(), _stream()), "tgs_sample")


def tgs_sample_noalloc(E, A, height, width, sp: tgs_sample_params, valid_tiles, tile_off, pix, tile_slot, totals,
                       tile_pred=None):
    """tgs_sample without a workspace (the library's static per-GPU scratch)."""
    _check(lib().tgs_sample_noalloc(_ptr(E), _ptr(A), height, width, ctypes.byref(sp), _ptr(tile_pred),
                                    _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), _ptr(tile_slot), _ptr(totals),
                                    _stream()), "tgs_sample_noalloc")


def tgs_bin_sort_workspace_size(n: int, capacity: int, n_tiles: int) -> int:
    return int(lib().tgs_bin_sort_workspace_size(n, capacity, n_tiles))


def tgs_bin_sort(rect, splat, depth, n, tile_slot, tiles_x, tiles_y, alpha_min, keys, vals, capacity, ranges,
                 touched, ws) -> int:
    """Returns the pair count; raises CapacityError(required) when it exceeds capacity."""
    n_pairs = _I64(0)
    st = lib().tgs_bin_sort(_ptr(rect), _ptr(splat), _ptr(depth), n, _ptr(tile_slot), tiles_x, tiles_y,
                            float(alpha_min), _ptr(keys), _ptr(vals), capacity, _ptr(ranges), _ptr(touched),
                            ctypes.byref(n_pairs), _ptr(ws), ws.numel() * ws.element_size(), _stream())
    _check(st, "tgs_bin_sort", n_pairs.value)
    return int(n_pairs.value)


def tgs_bin_sort_async(rect, splat, depth, n, tile_slot, tiles_x, tiles_y, alpha_min, keys, vals, capacity, ranges,
                       touched, counts, ws):
    """tgs_bin_sort without a host wait: counts (device int64[2]) receives the
    list length and the capacity needed."""
    _check(lib().tgs_bin_sort_async(_ptr(rect), _ptr(splat), _ptr(depth), n, _ptr(tile_slot), tiles_x, tiles_y,
                                    float(alpha_min), _ptr(keys), _ptr(vals), capacity, _ptr(ranges), _ptr(touched),
                                    _ptr(counts), _ptr(ws), ws.numel() * ws.element_size(), _stream()),
           "tgs_bin_sort_async")


def tgs_bin_sort_prefix_async(rect, splat, depth, n, tile_slot, tiles_x, tiles_y, alpha_min, prefix, keys, vals,
                              capacity, ranges, touched, counts, ws):
    """tgs_bin_sort_async restricted to the first ``prefix`` Gaussians in
    depth order; the workspace keeps the depth order for a continuation."""
    _check(lib().tgs_bin_sort_prefix_async(_ptr(rect), _ptr(splat), _ptr(depth), n, _ptr(tile_slot), tiles_x,
                                           tiles_y, float(alpha_min), int(prefix), _ptr(keys), _ptr(vals), capacity,
                                           _ptr(ranges), _ptr(touched), _ptr(counts), _ptr(ws),
                                           ws.numel() * ws.element_size(), _stream()),
           "tgs_bin_sort_prefix_async")


def tgs_bin_sort_continue_async(splat, n, flag_slot, tiles_x, tiles_y, alpha_min, prefix, capacity, ws, vals2,
                                capacity2, ranges2, counts2, ws2, n_flagged=None):
    """The continuation lists of the flagged tiles (Gaussians from depth rank
    ``prefix`` on) from a prefix call's workspace ``ws``."""
    _check(lib().tgs_bin_sort_continue_async(_ptr(splat), n, _ptr(flag_slot), _ptr(n_flagged), tiles_x, tiles_y,
                                             float(alpha_min),
                                             int(prefix), capacity, _ptr(ws), ws.numel() * ws.element_size(),
                                             _ptr(vals2), capacity2, _ptr(ranges2), _ptr(counts2), _ptr(ws2),
                                             ws2.numel() * ws2.element_size(), _stream()),
           "tgs_bin_sort_continue_async")


def tgs_render_fwd_prefix(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                          n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib, counters, state, cont_slot,
                          cont_list, cont_count):
    _check(lib().tgs_render_fwd_prefix(_ptr(splat), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height,
                                       _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                       ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _ptr(counters), _ptr(state),
                                       _ptr(cont_slot), _ptr(cont_list), _ptr(cont_count), _stream()),
           "tgs_render_fwd_prefix")


def tgs_render_fwd_cont(splat, vals, ranges, vals2, ranges2, tiles_x, tiles_y, width, height, valid_tiles, tile_off,
                        pix, n_st, max_per_tile, rp: tgs_raster_params, cont_list, cont_count, out, ncontrib,
                        counters=None, state=None):
    _check(lib().tgs_render_fwd_cont(_ptr(splat), _ptr(vals), _ptr(ranges), _ptr(vals2), _ptr(ranges2), tiles_x,
                                     tiles_y, width, height, _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st,
                                     max_per_tile, ctypes.byref(rp), _ptr(cont_list), _ptr(cont_count), _ptr(out),
                                     _ptr(ncontrib), _ptr(counters), _ptr(state), _stream()),
           "tgs_render_fwd_cont")


def tgs_render_bwd2(splat, vals, ranges, vals2, ranges2, tiles_x, tiles_y, width, height, valid_tiles, tile_off,
                    pix, n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib, dL_dout, g2d, state=None,
                    touched=None, err=None, n=0, stats=None):
    """tgs_render_bwd over two-segment lists; with ``stats`` (and err, n) it
    also adds the density-control sums like tgs_render_bwd_density."""
    _check(lib().tgs_render_bwd2(_ptr(splat), _ptr(vals), _ptr(ranges), _ptr(vals2), _ptr(ranges2), tiles_x, tiles_y,
                                 width, height, _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                 ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _ptr(dL_dout), _ptr(g2d), _ptr(state),
                                 _ptr(touched), _ptr(err), n, _ptr(stats), _stream()), "tgs_render_bwd2")


def tgs_density_accumulate2(splat, vals, ranges, vals2, ranges2, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp: tgs_raster_params, ncontrib, err, n, stats,
                            state=None):
    _check(lib().tgs_density_accumulate2(_ptr(splat), _ptr(vals), _ptr(ranges), _ptr(vals2), _ptr(ranges2), tiles_x,
                                         tiles_y, width, height, _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st,
                                         max_per_tile, ctypes.byref(rp), _ptr(ncontrib), _ptr(err), _ptr(state), n,
                                         _ptr(stats), _stream()), "tgs_density_accumulate2")


def tgs_render_state_size(n_slots: int, max_per_tile: int) -> int:
    return int(lib().tgs_render_state_size(n_slots, max_per_tile))


def tgs_render_fwd(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                   n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib, counters=None, state=None):
    _check(lib().tgs_render_fwd(_ptr(splat), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height,
                                _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _ptr(counters), _ptr(state),
                                _stream()), "tgs_render_fwd")


def tgs_render_bwd(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                   n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib, dL_dout, g2d, state=None,
                   touched=None):
    _check(lib().tgs_render_bwd(_ptr(splat), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height,
                                _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _ptr(dL_dout), _ptr(g2d),
                                _ptr(state), _ptr(touched), _stream()), "tgs_render_bwd")


def tgs_render_bwd_det_workspace_size(n_pairs: int, max_per_tile: int, dense: bool) -> int:
    return int(lib().tgs_render_bwd_det_workspace_size(n_pairs, max_per_tile, int(bool(dense))))


def tgs_render_bwd_deterministic(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                                 n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib, dL, g2d, state, touched,
                                 depth, rect, n, n_pairs, ws):
    _check(lib().tgs_render_bwd_deterministic(
        _ptr(splat), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height, _ptr(valid_tiles), _ptr(tile_off),
        _ptr(pix), n_st, max_per_tile, ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _ptr(dL), _ptr(g2d),
        _ptr(state), _ptr(touched), _ptr(depth), _ptr(rect), n, n_pairs, _ptr(ws), ws.numel() * ws.element_size(),
        _stream()), "tgs_render_bwd_deterministic")


def tgs_loss(out, gt, height, width, valid_tiles, tile_off, pix, n_st, totals, lp: tgs_loss_params,
             dL_dout, err, lam, tile_loss):
    _check(lib().tgs_loss(_ptr(out), _ptr(gt), height, width, _ptr(valid_tiles), _ptr(tile_off), _ptr(pix),
                          n_st, _ptr(totals), ctypes.byref(lp), _ptr(dL_dout), _ptr(err), _ptr(lam),
                          _ptr(tile_loss), _stream()), "tgs_loss")


def tgs_ema_age_update(E, A, height, width, tile_slot, tile_off, pix, err, beta):
    _check(lib().tgs_ema_age_update(_ptr(E), _ptr(A), height, width, _ptr(tile_slot), _ptr(tile_off),
                                    _ptr(pix), _ptr(err), beta, _stream()), "tgs_ema_age_update")


def tgs_error_init(out_dense, gt, height, width, E):
    _check(lib().tgs_error_init(_ptr(out_dense), _ptr(gt), height, width, _ptr(E), _stream()),
           "tgs_error_init")


def tgs_density_accumulate(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                           n_st, max_per_tile, rp: tgs_raster_params, ncontrib, err, n, stats, state=None):
    _check(lib().tgs_density_accumulate(_ptr(splat), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height,
                                        _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                        ctypes.byref(rp), _ptr(ncontrib), _ptr(err), _ptr(state), n, _ptr(stats),
                                        _stream()),
           "tgs_density_accumulate")


def tgs_render_bwd_density(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix,
                           n_st, max_per_tile, rp: tgs_raster_params, out, ncontrib, dL_dout, g2d, err, n, stats,
                           state=None, touched=None):
    _check(lib().tgs_render_bwd_density(_ptr(splat), _ptr(vals), _ptr(ranges), tiles_x, tiles_y, width, height,
                                        _ptr(valid_tiles), _ptr(tile_off), _ptr(pix), n_st, max_per_tile,
                                        ctypes.byref(rp), _ptr(out), _ptr(ncontrib), _ptr(dL_dout), _ptr(g2d),
                                        _ptr(state), _ptr(touched), _ptr(err), n, _ptr(stats), _stream()),
           "tgs_render_bwd_density")


def tgs_density_score(stats, n, lambda_base, rho, eps, e_out, d_out, s_out):
    _check(lib().tgs_density_score(_ptr(stats), n, lambda_base, rho, eps, _ptr(e_out), _ptr(d_out), _ptr(s_out),
                                   _stream()), "tgs_density_score")


def tgs_density_topology_workspace_size(n) -> int:
    return int(lib().tgs_density_topology_workspace_size(n))


def tgs_density_topology_count(keep, densify, n, ws):
    """Returns (n_keep, n_new)."""
    nk, nn = _I64(0), _I64(0)
    _check(lib().tgs_density_topology_count(_ptr(keep), _ptr(densify), n, ctypes.byref(nk), ctypes.byref(nn),
                                            _ptr(ws), ws.numel() * ws.element_size(), _stream()),
           "tgs_density_topology_count")
    return int(nk.value), int(nn.value)


def tgs_density_topology_apply(params, m, v, n, z, log_split, ws, params_out, m_out, v_out, n_out):
    _check(lib().tgs_density_topology_apply(_ptr(params), _ptr(m), _ptr(v), n, _ptr(z), log_split, _ptr(ws),
                                            ws.numel() * ws.element_size(), _ptr(params_out), _ptr(m_out),
                                            _ptr(v_out), n_out, _stream()), "tgs_density_topology_apply")


def tgs_grad_screen_accumulate(g2d, radius, n, width, height, acc):
    _check(lib().tgs_grad_screen_accumulate(_ptr(g2d), _ptr(radius), n, width, height, _ptr(acc), _stream()),
           "tgs_grad_screen_accumulate")


def tgs_density_masks(scores, gstats, dstats, n, thr, tau_grad, tau_grad_abs, prune, densify, keep):
    _check(lib().tgs_density_masks(_ptr(scores), _ptr(gstats), _ptr(dstats), n, _ptr(thr), float(tau_grad),
                                   float(tau_grad_abs), int(prune), _ptr(densify), _ptr(keep), _stream()),
           "tgs_density_masks")


def tgs_grad_screen_mean(acc, n, out):
    _check(lib().tgs_grad_screen_mean(_ptr(acc), n, _ptr(out), _stream()), "tgs_grad_screen_mean")


def tgs_view_error_sums(E, n_views, pixels, sums):
    _check(lib().tgs_view_error_sums(_ptr(E), n_views, pixels, _ptr(sums), _stream()), "tgs_view_error_sums")


def tgs_select_workspace_size() -> int:
    return int(lib().tgs_select_workspace_size())


def tgs_select_kth_largest(values, n, k, out, ws):
    _check(lib().tgs_select_kth_largest(_ptr(values), n, k, _ptr(out), _ptr(ws), ws.numel() * ws.element_size(), _stream()),
           "tgs_select_kth_largest")


def tgs_threshold_mask(values, n, thr, mask):
    _check(lib().tgs_threshold_mask(_ptr(values), n, _ptr(thr), _ptr(mask), _stream()), "tgs_threshold_mask")


def tgs_project_bwd(params, n, cam: tgs_camera, rp: tgs_raster_params, radius, clamp, g2d, grad,
                    accumulate: bool = True):
    _check(lib().tgs_project_bwd(_ptr(params), n, ctypes.byref(cam), ctypes.byref(rp), _ptr(radius),
                                 _ptr(clamp), _ptr(g2d), _ptr(grad), int(bool(accumulate)), _stream()),
           "tgs_project_bwd")


def tgs_optimizer_step(params, grad, m, v, n, touched, op: tgs_optim_params, step):
    _check(lib().tgs_optimizer_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, _ptr(touched),
                                    ctypes.byref(op), step, _stream()), "tgs_optimizer_step")


def tgs_project_bwd_optimizer_workspace_size(n: int) -> int:
    return int(lib().tgs_project_bwd_optimizer_workspace_size(n))


def tgs_project_bwd_optimizer_step(params, n, cam: tgs_camera, rp: tgs_raster_params, radius, clamp, g2d,
                                   grad_prev, m, v, touched, op: tgs_optim_params, step, ws):
    _check(lib().tgs_project_bwd_optimizer_step(_ptr(params), n, ctypes.byref(cam), ctypes.byref(rp),
                                                _ptr(radius), _ptr(clamp), _ptr(g2d), _ptr(grad_prev),
                                                _ptr(m), _ptr(v), _ptr(touched), ctypes.byref(op), step,
                                                _ptr(ws), ws.numel() * ws.element_size(), _stream()),
           "tgs_project_bwd_optimizer_step")


def tgs_project_bwd_optimizer_views_workspace_size(n: int, n_views: int) -> int:
    return int(lib().tgs_project_bwd_optimizer_views_workspace_size(n, n_views))


def tgs_project_bwd_optimizer_step_views(params, n, cams, rp: tgs_raster_params, radius, clamp, g2d, m, v, touched,
                                         op: tgs_optim_params, step, ws):
    """Every view's projection backward and the update in one pass; cams,
    radius, clamp and g2d are per-view lists (tgs_camera records, device
    tensors)."""
    k = len(cams)
    cam_arr = (tgs_camera * k)(*cams)
    ptrs = [(ctypes.c_void_p * k)(*[_ptr(t) for t in xs]) for xs in (radius, clamp, g2d)]
    _check(lib().tgs_project_bwd_optimizer_step_views(_ptr(params), n, k, cam_arr, ctypes.byref(rp), ptrs[0], ptrs[1],
                                                      ptrs[2], _ptr(m), _ptr(v), _ptr(touched), ctypes.byref(op),
                                                      step, _ptr(ws), ws.numel() * ws.element_size(), _stream()),
           "tgs_project_bwd_optimizer_step_views")


# ------------------------------------------------------------------ learned tile priority
TILE_MLP_FEATURES = 32
TILE_MLP_PARAMS = 6337


def tgs_tile_features(ranges, E, A, height: int, width: int, cam: tgs_camera, X):
    _check(lib().tgs_tile_features(_ptr(ranges), _ptr(E), _ptr(A), height, width, ctypes.byref(cam), _ptr(X),
                                   _stream()), "tgs_tile_features")


def tgs_tile_mlp_fwd(params, X, n: int, y, act=None):
    _check(lib().tgs_tile_mlp_fwd(_ptr(params), _ptr(X), n, _ptr(y), _ptr(act), _stream()), "tgs_tile_mlp_fwd")


def tgs_tile_mlp_workspace_size(n: int) -> int:
    return int(lib().tgs_tile_mlp_workspace_size(n))


def tgs_tile_mlp_train_step(params, m, v, X, act, y, target, n: int, step: int, lr: float, ws, grad=None):
    _check(lib().tgs_tile_mlp_train_step(_ptr(params), _ptr(m), _ptr(v), _ptr(X), _ptr(act), _ptr(y), _ptr(target),
                                         n, step, float(lr), _ptr(grad), _ptr(ws), ws.numel() * ws.element_size(),
                                         _stream()), "tgs_tile_mlp_train_step")
