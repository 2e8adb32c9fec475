"""``torch.autograd.Function`` around the sparse rasterizer.

Forward: project, bin/sort and composite the given samples of one view
(``tgs_project`` -> ``tgs_bin_sort`` -> ``tgs_render_fwd``).  Backward: the
hand-written adjoint (``tgs_render_bwd`` -> ``tgs_project_bwd``).  The context
keeps only the projected splats, the sorted ids with the tile ranges, and the
per-sample outputs (final colour, transmittance, contributor count): the
backward recomputes every per-pixel quantity from them instead of storing
per-(pixel, Gaussian) state (Sec. 3.6: splat-parallel backward without a
dense replay).

Float64 parameters select the FP64 instantiation of the same kernels
(``tgs_project_f64``, ``tgs_render_fwd_f64``, ``tgs_render_bwd_f64``,
``tgs_project_bwd_f64``; the lists come from the same ``tgs_bin_sort``), so
``torch.autograd.gradcheck`` can check the adjoint against finite
differences at double precision.
"""
from __future__ import annotations

import torch

from . import binding as B
from .pipeline import ViewBuffers


class Samples:
    """A view's sample set as device tensors (``None`` valid_tiles = dense)."""

    def __init__(self, valid_tiles, tile_off, pix, n_st: int, max_per_tile: int, tile_slot=None):
        self.valid_tiles, self.tile_off, self.pix = valid_tiles, tile_off, pix
        self.n_st, self.max_per_tile, self.tile_slot = n_st, max_per_tile, tile_slot


class SparseRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, cam, samples: Samples, rp=None):
        rp = rp if rp is not None else B.raster_params()
        n = params.shape[1]
        params = params.contiguous()
        vb = ViewBuffers(n, cam.width, cam.height, None, -1, params.device)
        if samples.valid_tiles is not None:
            vb.dense = False
            vb.valid_tiles, vb.tile_off, vb.pix = samples.valid_tiles, samples.tile_off, samples.pix
            vb.tile_slot = samples.tile_slot
            vb.n_st, vb.n_pix = samples.n_st, samples.max_per_tile
            P = int(samples.tile_off[-1].item()) if samples.n_st > 0 else 0
            vb.out = torch.empty((max(P, 1), 4), dtype=torch.float32, device=params.device)
            vb.ncontrib = torch.empty(max(P, 1), dtype=torch.int32, device=params.device)
            vb.P = P
        else:
            vb.P = cam.width * cam.height
        c = B.camera(cam)
        ctx.vb, ctx.cam, ctx.rp = vb, c, rp
        ctx.save_for_backward(params)
        if params.dtype == torch.float64:
            vb.rec64 = torch.empty((n, 12), dtype=torch.float64, device=params.device)
            B.tgs_project_f64(params, n, c, rp, vb.rec64, vb.splat, vb.depth, vb.radius, vb.rect, vb.clamp)
            vb.bin_sort(alpha_min=rp.alpha_min)
            vb.out64 = torch.empty((max(vb.P, 1), 4), dtype=torch.float64, device=params.device)
            B.tgs_render_fwd_f64(vb.rec64, vb.vals, vb.ranges, vb.tiles_x, vb.tiles_y, vb.width, vb.height,
                                 vb.valid_tiles, vb.tile_off, vb.pix, vb.n_st, vb.n_pix, rp, vb.out64, vb.ncontrib)
            return vb.out64[: vb.P, :3].clone()
        if params.dtype != torch.float32:
            raise TypeError("SparseRasterize: parameters must be float32 or float64")
        vb.project(params, c, rp)
        vb.bin_sort(alpha_min=rp.alpha_min)
        vb.render_fwd(rp)
        return vb.out[: vb.P, :3].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        vb = ctx.vb
        if params.dtype == torch.float64:
            dL = torch.zeros((max(vb.P, 1), 4), dtype=torch.float64, device=params.device)
            dL[: vb.P, :3] = grad_out
            g2d = torch.zeros((vb.n, 9), dtype=torch.float64, device=params.device)
            B.tgs_render_bwd_f64(vb.rec64, vb.vals, vb.ranges, vb.tiles_x, vb.tiles_y, vb.width, vb.height,
                                 vb.valid_tiles, vb.tile_off, vb.pix, vb.n_st, vb.n_pix, ctx.rp, vb.out64,
                                 vb.ncontrib, dL, g2d)
            grad = torch.empty_like(params)
            B.tgs_project_bwd_f64(params, vb.n, ctx.cam, ctx.rp, vb.radius, vb.clamp, g2d, grad, accumulate=False)
            return grad, None, None, None
        dL = torch.zeros((max(vb.P, 1), 4), dtype=torch.float32, device=params.device)
        dL[: vb.P, :3] = grad_out
        vb.dL = dL
        vb.render_bwd(ctx.rp)
        grad = torch.empty_like(params)
        vb.project_bwd(params, ctx.cam, ctx.rp, grad, accumulate=False)
        return grad, None, None, None


def rasterize(params, cam, samples: Samples, rp=None):
    return SparseRasterize.apply(params, cam, samples, rp)
