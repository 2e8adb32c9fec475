"""Host-side orchestration of one training step on the GPU (Alg. 1, steps 3-10
for the selected views): buffers are allocated once per shape and every step
of the path runs in the HIP library through the C ABI.

A view's work, in order:
  tgs_sample -> tgs_project -> tgs_bin_sort -> tgs_render_fwd -> tgs_loss
  -> tgs_ema_age_update -> tgs_render_bwd -> tgs_project_bwd
and once per step the optimizer update, fused with the last view's
projection backward (tgs_project_bwd_optimizer_step).  The sampler of every view runs first
because the loss normalises by the step's total sample and tile counts.

Two streams (both at the default priority): the samplers run on a side
stream while the main stream projects and bins (binning needs the sample
only when it restricts the tiles), and each view's error/age update runs on
the side stream beside the backward, which does not read the maps.  Events
order the two; the step ends with the main stream waiting for the side one.
With ``density_stats`` each sparse view's backward also back-projects the
per-pixel errors onto the Gaussians (tgs_render_bwd_density, Sec. 3.8) for
the density-control score (tgs_density_score) and its percentile selections.
"""
from __future__ import annotations

import contextlib
import math
from dataclasses import dataclass, field

import torch

from . import binding as B

TILE = B.TILE


_NO_STAGE = contextlib.nullcontext()  # the stage bracket when a stage is not timed


@dataclass
class StepConfig:
    """What one step samples and how it renders (dense when ``rate_permille`` is None)."""
    rate_permille: int | None = 250
    n_tiles_sel: int = -1
    hard_permille: int = 400
    stable_permille: int = 300
    beta: float = 0.4
    seed: int = 3
    fuse_optimizer: bool = True   # last view's projection backward fused with the update
    # every view's projection backward fused with the update in one pass
    # (tgs_project_bwd_optimizer_step_views; no gradient array), one-view
    # steps included (it visits touched Gaussians only)
    fuse_views: bool = False
    # views side by side: each view's sampler and chain (projection to
    # backward) on a stream of its own, reused round-robin (1: all on the
    # current stream, in view order)
    view_streams: int = 1
    learned_tiles: bool = False   # tile pass by the learned tile priority (with n_tiles_sel > 0)
    tile_lr: float = 3e-3         # its online Adam learning rate
    tile_seed: int = 23           # its initial weights
    density_stats: bool = False   # back-project (e, w, D) onto the Gaussians each sparse view (Sec. 3.8)
    deterministic: bool = False   # bitwise-reproducible backward (tgs_render_bwd_deterministic)
    # depth-prefix binning: each view's lists hold the nearest prefix_fraction
    # of the Gaussians, plus a continuation for the tiles where a pixel ran
    # past them (the same images and gradients as whole lists; None: off)
    prefix_fraction: float | None = None
    raster: dict = field(default_factory=dict)
    loss: dict = field(default_factory=dict)
    optim: dict = field(default_factory=dict)


class ViewBuffers:
    """Per-view device buffers for one image size and sampling rate."""

    def __init__(self, n: int, width: int, height: int, n_pix: int | None, n_tiles_sel: int,
                 device, capacity: int | None = None, keep_keys: bool = False):
        self.n, self.width, self.height = n, width, height
        self.keep_keys = keep_keys
        self.tiles_x, self.tiles_y = (width + TILE - 1) // TILE, (height + TILE - 1) // TILE
        self.n_t = self.tiles_x * self.tiles_y
        self.dense = n_pix is None
        self.n_pix = 256 if n_pix is None else n_pix
        dev = device
        self.splat = torch.empty((n, B.SPLAT_FLOATS), dtype=torch.float32, device=dev)
        self.depth = torch.empty(n, dtype=torch.float32, device=dev)
        self.radius = torch.empty(n, dtype=torch.int32, device=dev)
        self.rect = torch.empty((n, 4), dtype=torch.int32, device=dev)
        self.clamp = torch.empty(n, dtype=torch.uint8, device=dev)
        if self.dense:
            self.n_st = self.n_t
            self.P_cap = width * height
            self.valid_tiles = self.tile_off = self.pix = self.tile_slot = None
        else:
            sp = B.sample_params(self.n_pix, n_tiles_sel=n_tiles_sel)
            self.n_st = B.tgs_sample_tile_count(height, width, sp)
            self.P_cap = self.n_st * self.n_pix
            self.valid_tiles = torch.empty(max(self.n_st, 1), dtype=torch.int32, device=dev)
            self.tile_off = torch.empty(self.n_st + 1, dtype=torch.int32, device=dev)
            self.pix = torch.empty(max(self.P_cap, 1), dtype=torch.uint8, device=dev)
            self.tile_slot = torch.empty(self.n_t, dtype=torch.int32, device=dev)
            self.sample_ws = torch.empty(B.tgs_sample_workspace_size(height, width), dtype=torch.uint8,
                                         device=dev)
        self.ranges = torch.empty((self.n_t, 2), dtype=torch.int32, device=dev)
        self.out = torch.empty((max(self.P_cap, 1), 4), dtype=torch.float32, device=dev)
        self.ncontrib = torch.empty(max(self.P_cap, 1), dtype=torch.int32, device=dev)
        self.dL = torch.zeros((max(self.P_cap, 1), 4), dtype=torch.float32, device=dev)
        self.err = torch.empty(max(self.P_cap, 1), dtype=torch.float32, device=dev)
        self.lam = torch.empty(max(self.n_st, 1), dtype=torch.float32, device=dev)
        self.tile_loss = torch.zeros((max(self.n_st, 1), 2), dtype=torch.float32, device=dev)
        self.g2d = torch.empty((n, B.G2D_FLOATS), dtype=torch.float32, device=dev)
        # per-pixel (T, colour) at the backward's chunk starts, kept by the forward
        n_state = B.tgs_render_state_size(self.n_st, self.n_pix) // 4
        self.state = torch.empty(max(n_state, 4), dtype=torch.float32, device=dev)
        # (list length, capacity needed[, whole-list pairs after a depth-prefix call])
        self.counts = torch.zeros(3, dtype=torch.int64, device=dev)
        # depth-prefix lists: the continuation's lists and the marked tiles
        self.two_part = False
        self.prefix = self.n
        self.counts2 = torch.zeros(2, dtype=torch.int64, device=dev)
        self.capacity2 = 0
        self.vals2 = self.ranges2 = self.sort_ws2 = None
        self.cont_slot = self.cont_list = self.cont_count = None
        self._n_pairs = 0
        self.sized = False   # whether a bin/sort has run to completion here (the capacity then fits a view)
        self._alloc_pairs(capacity if capacity is not None else max(1 << 16, 8 * n))

    @property
    def n_pairs(self) -> int:
        """Pairs in the lists of the last bin/sort (reads the device count
        after an asynchronous one; raises CapacityError if it overflowed)."""
        if self._n_pairs is None:
            valid, need = (int(x) for x in self.counts[:2].cpu().tolist())
            if need > self.capacity:
                raise B.CapacityError(f"pair lists need {need} entries, capacity {self.capacity}", need)
            if self.two_part:
                valid2, need2 = (int(x) for x in self.counts2.cpu().tolist())
                if need2 > self.capacity2:
                    raise B.CapacityError(f"continuation lists need {need2} entries, capacity {self.capacity2}",
                                          need2)
                valid += valid2
            self._n_pairs = valid
        return self._n_pairs

    @n_pairs.setter
    def n_pairs(self, v: int):
        self._n_pairs = v

    def _alloc_pairs(self, capacity: int):
        dev = self.splat.device
        if getattr(self, "vals", None) is not None:
            # the old arrays may still be in use on another stream (views
            # side by side): the allocator must not hand them out before
            # that work ends
            torch.cuda.synchronize(dev)
        self.capacity = int(capacity)
        self.keys = torch.empty(self.capacity, dtype=torch.int64, device=dev) if self.keep_keys else None
        self.vals = torch.empty(self.capacity, dtype=torch.int32, device=dev)
        self.sort_ws = torch.empty(B.tgs_bin_sort_workspace_size(self.n, self.capacity, self.n_t),
                                   dtype=torch.uint8, device=dev)

    # ---- the steps of one view
    def sample(self, E, A, cfg: StepConfig, step: int, view: int, totals, tile_pred=None):
        sp = B.sample_params(self.n_pix, cfg.hard_permille, cfg.stable_permille, cfg.n_tiles_sel,
                             cfg.seed, step, view)
        B.tgs_sample(E, A, self.height, self.width, sp, self.valid_tiles, self.tile_off, self.pix,
                     self.tile_slot, totals, self.sample_ws, tile_pred=tile_pred)

    def project(self, params, cam: B.tgs_camera, rp):
        # also clears the screen-space gradient that the backward accumulates into
        B.tgs_project(params, self.n, cam, rp, self.splat, self.depth, self.radius, self.rect, self.clamp,
                      self.g2d)

    def bin_sort_needs_samples(self) -> bool:
        """Binning reads the tile map only when the sampler keeps a subset of tiles."""
        return self.tile_slot is not None and self.n_st < self.n_t

    def bin_sort(self, touched=None, alpha_min: float = 1.0 / 255.0) -> int:
        """Bin and sort, waiting for the count: grows the pair arrays and
        repeats when they are too small.  Returns the list length."""
        while True:
            self.bin_sort_async(touched, alpha_min)
            valid, need = (int(x) for x in self.counts[:2].cpu().tolist())
            if need <= self.capacity:
                self.n_pairs = valid
                self.sized = True
                return valid
            self._alloc_pairs(int(need * 1.5) + 1024)

    def bin_sort_async(self, touched=None, alpha_min: float = 1.0 / 255.0):
        """Bin and sort without a host wait (tgs_bin_sort_async); the counts
        stay on the device until n_pairs is read."""
        # every tile is valid when the sampler keeps all of them: no tile map needed
        tile_slot = self.tile_slot if self.bin_sort_needs_samples() else None
        B.tgs_bin_sort_async(self.rect, self.splat, self.depth, self.n, tile_slot, self.tiles_x, self.tiles_y,
                             alpha_min, self.keys, self.vals, self.capacity, self.ranges, touched, self.counts,
                             self.sort_ws)
        self.two_part = False
        self._n_pairs = None

    # ---- depth-prefix lists
    def _alloc_cont(self, capacity2: int):
        dev = self.splat.device
        if self.vals2 is not None:
            torch.cuda.synchronize(dev)   # as in _alloc_pairs
        self.capacity2 = int(capacity2)
        self.vals2 = torch.empty(self.capacity2, dtype=torch.int32, device=dev)
        self.sort_ws2 = torch.empty(B.tgs_bin_sort_workspace_size(self.n, self.capacity2, self.n_t),
                                    dtype=torch.uint8, device=dev)
        if self.ranges2 is None:
            self.ranges2 = torch.empty((self.n_t, 2), dtype=torch.int32, device=dev)
            self.cont_slot = torch.empty(self.n_t, dtype=torch.int32, device=dev)
            self.cont_list = torch.empty(max(self.n_st, 1), dtype=torch.int32, device=dev)
            self.cont_count = torch.zeros(1, dtype=torch.int32, device=dev)

    # capacity margins of depth-prefix lists: views of one scene differ in
    # their prefix and continuation needs, and an overflow is only seen two
    # steps later, so both arrays keep room to spare
    PREFIX_MARGIN = 2.0       # prefix arrays: twice the need they were sized on
    CONT_MIN_SHARE = 0.35     # continuation: at least this share of the whole lists' pairs

    def bin_sort_prefix(self, prefix: int, touched=None, alpha_min: float = 1.0 / 255.0, wait: bool = False):
        """The lists of the nearest ``prefix`` Gaussians (no host wait unless
        ``wait``: then the pair arrays, and the continuation's, are sized
        from the counts)."""
        tile_slot = self.tile_slot if self.bin_sort_needs_samples() else None
        self.prefix = int(min(prefix, self.n))
        while True:
            B.tgs_bin_sort_prefix_async(self.rect, self.splat, self.depth, self.n, tile_slot, self.tiles_x,
                                        self.tiles_y, alpha_min, self.prefix, self.keys, self.vals, self.capacity,
                                        self.ranges, touched, self.counts, self.sort_ws)
            if not wait:
                break
            _, need, whole = (int(x) for x in self.counts.cpu().tolist())
            if need <= self.capacity:
                if self.capacity < self.PREFIX_MARGIN * need:
                    self._alloc_pairs(int(self.PREFIX_MARGIN * need) + 1024)
                    continue   # re-run into the new arrays
                want2 = max(1 << 16, int(self.CONT_MIN_SHARE * whole))
                if self.vals2 is None or self.capacity2 < want2:
                    self._alloc_cont(want2)
                break
            self._alloc_pairs(int(self.PREFIX_MARGIN * need) + 1024)
        self.two_part = True
        self._n_pairs = None

    def render_fwd_two_part(self, rp, counters=None, alpha_min: float = 1.0 / 255.0, wait: bool = False):
        """Forward over the prefix lists, the continuation lists of the tiles
        it marks, and the forward again for those tiles over both parts."""
        self.render_fwd_prefix(rp, counters)
        self.continue_lists(alpha_min, wait)
        self.render_fwd_cont(rp, counters)

    def render_fwd_prefix(self, rp, counters=None):
        """Forward over the prefix lists, marking the tiles that need more."""
        if self.vals2 is None:
            self._alloc_cont(max(1 << 16, self.capacity // 2))
        B.tgs_render_fwd_prefix(self.splat, self.vals, self.ranges, self.tiles_x, self.tiles_y, self.width,
                                self.height, self.valid_tiles, self.tile_off, self.pix, self.n_st, self.n_pix, rp,
                                self.out, self.ncontrib, counters, self.state, self.cont_slot, self.cont_list,
                                self.cont_count)

    def continue_lists(self, alpha_min: float = 1.0 / 255.0, wait: bool = False):
        """The continuation lists of the marked tiles (``wait``: grow their
        arrays until they fit)."""
        while True:
            B.tgs_bin_sort_continue_async(self.splat, self.n, self.cont_slot, self.tiles_x, self.tiles_y, alpha_min,
                                          self.prefix, self.capacity, self.sort_ws, self.vals2, self.capacity2,
                                          self.ranges2, self.counts2, self.sort_ws2, n_flagged=self.cont_count)
            if not wait:
                break
            need = int(self.counts2[1].item())
            if need <= self.capacity2:
                break
            self._alloc_cont(int(need * 1.5) + 1024)

    def render_fwd_cont(self, rp, counters=None):
        """The marked tiles' forward over both parts of their lists."""
        B.tgs_render_fwd_cont(self.splat, self.vals, self.ranges, self.vals2, self.ranges2, self.tiles_x,
                              self.tiles_y, self.width, self.height, self.valid_tiles, self.tile_off, self.pix,
                              self.n_st, self.n_pix, rp, self.cont_list, self.cont_count, self.out, self.ncontrib,
                              counters, self.state)

    def render_fwd(self, rp, counters=None):
        if self.two_part:
            raise RuntimeError("two-part lists: render with render_fwd_two_part")
        B.tgs_render_fwd(self.splat, self.vals, self.ranges, self.tiles_x, self.tiles_y, self.width,
                         self.height, self.valid_tiles, self.tile_off, self.pix, self.n_st, self.n_pix,
                         rp, self.out, self.ncontrib, counters, self.state)

    def loss(self, gt, totals, lp):
        B.tgs_loss(self.out, gt, self.height, self.width, self.valid_tiles, self.tile_off, self.pix,
                   self.n_st, totals, lp, self.dL, self.err, self.lam, self.tile_loss)

    def ema_age(self, E, A, beta):
        B.tgs_ema_age_update(E, A, self.height, self.width, self.tile_slot, self.tile_off, self.pix,
                             self.err, beta)

    def density(self, rp, stats):
        if self.two_part:
            B.tgs_density_accumulate2(self.splat, self.vals, self.ranges, self.vals2, self.ranges2, self.tiles_x,
                                      self.tiles_y, self.width, self.height, self.valid_tiles, self.tile_off,
                                      self.pix, self.n_st, self.n_pix, rp, self.ncontrib, self.err, self.n, stats,
                                      self.state)
            return
        B.tgs_density_accumulate(self.splat, self.vals, self.ranges, self.tiles_x, self.tiles_y, self.width,
                                 self.height, self.valid_tiles, self.tile_off, self.pix, self.n_st, self.n_pix,
                                 rp, self.ncontrib, self.err, self.n, stats, self.state)

    def render_bwd(self, rp, zero=True, stats=None, touched=None, deterministic=False):
        """The backward; with ``stats`` it also adds the density-control
        sums; ``touched`` collects the Gaussians composited at a sample;
        ``deterministic`` selects the bitwise-reproducible reduction (not
        with ``stats``)."""
        if zero:
            self.g2d.zero_()
        if self.two_part:
            if deterministic:
                raise ValueError("the deterministic backward takes whole lists, not depth-prefix lists")
            B.tgs_render_bwd2(self.splat, self.vals, self.ranges, self.vals2, self.ranges2, self.tiles_x,
                              self.tiles_y, self.width, self.height, self.valid_tiles, self.tile_off, self.pix,
                              self.n_st, self.n_pix, rp, self.out, self.ncontrib, self.dL, self.g2d, self.state,
                              touched, self.err if stats is not None else None, self.n if stats is not None else 0,
                              stats)
            return
        if deterministic:
            if stats is not None:
                raise ValueError("the deterministic backward has no density-control variant")
            pairs = self.n_pairs
            need = B.tgs_render_bwd_det_workspace_size(pairs, self.n_pix, self.dense)
            if getattr(self, "det_ws", None) is None or self.det_ws.numel() < need:
                self.det_ws = torch.empty(need, dtype=torch.uint8, device=self.splat.device)
            B.tgs_render_bwd_deterministic(self.splat, self.vals, self.ranges, self.tiles_x, self.tiles_y, self.width,
                                           self.height, self.valid_tiles, self.tile_off, self.pix, self.n_st,
                                           self.n_pix, rp, self.out, self.ncontrib, self.dL, self.g2d, self.state,
                                           touched, self.depth, self.rect, self.n, pairs, self.det_ws)
            return
        if stats is not None:
            B.tgs_render_bwd_density(self.splat, self.vals, self.ranges, self.tiles_x, self.tiles_y, self.width,
                                     self.height, self.valid_tiles, self.tile_off, self.pix, self.n_st,
                                     self.n_pix, rp, self.out, self.ncontrib, self.dL, self.g2d, self.err, self.n,
                                     stats, self.state, touched)
            return
        B.tgs_render_bwd(self.splat, self.vals, self.ranges, self.tiles_x, self.tiles_y, self.width,
                         self.height, self.valid_tiles, self.tile_off, self.pix, self.n_st, self.n_pix,
                         rp, self.out, self.ncontrib, self.dL, self.g2d, self.state, touched)

    def project_bwd(self, params, cam: B.tgs_camera, rp, grad, accumulate=True):
        B.tgs_project_bwd(params, self.n, cam, rp, self.radius, self.clamp, self.g2d, grad, accumulate)


def init_tile_params(seed: int) -> torch.Tensor:
    """Initial weights of the learned tile priority: N(0, 1/fan_in) hidden
    weights, zero biases and a zero output layer, so the model starts as the
    error-map predictor (it adds to the tile's stale mean error)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    p = np.zeros(B.TILE_MLP_PARAMS, dtype=np.float32)
    p[0:2048] = rng.normal(0.0, 1.0 / np.sqrt(32.0), 2048)
    p[2112:6208] = rng.normal(0.0, 1.0 / np.sqrt(64.0), 4096)
    return torch.from_numpy(p)


class TilePriority:
    """The learned tile priority of one training run: model, Adam state, the
    pair ranges each view had at its last binning, and per-slot scratch."""

    def __init__(self, n_views: int, n_t: int, cfg: StepConfig, dev):
        self.params = init_tile_params(cfg.tile_seed).to(dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.lr = cfg.tile_lr
        self.steps = 0
        self.n_t = n_t
        self.ranges = torch.zeros((n_views, n_t, 2), dtype=torch.int32, device=dev)
        self.ws = torch.empty(B.tgs_tile_mlp_workspace_size(n_t), dtype=torch.uint8, device=dev)
        self._slots: dict = {}

    def slot(self, k: int) -> dict:
        if k not in self._slots:
            d = self.params.device
            self._slots[k] = dict(X=torch.empty((self.n_t, 32), dtype=torch.float32, device=d),
                                  Xa=torch.empty((self.n_t, 32), dtype=torch.float32, device=d),
                                  y=torch.empty(self.n_t, dtype=torch.float32, device=d),
                                  t=torch.empty(self.n_t, dtype=torch.float32, device=d),
                                  act=torch.empty((self.n_t, 128), dtype=torch.float32, device=d))
        return self._slots[k]

    def predict(self, k, v, E, A, vb, cam):
        """Features from the view's maps and its last pair ranges; predictions."""
        s = self.slot(k)
        B.tgs_tile_features(self.ranges[v], E, A, vb.height, vb.width, cam, s["X"])
        B.tgs_tile_mlp_fwd(self.params, s["X"], self.n_t, s["y"], s["act"])
        return s["y"]

    def learn(self, k, v, E, A, vb, cam):
        """One training step towards the tile means of the updated error map;
        the view's pair ranges are kept for its next prediction."""
        s = self.slot(k)
        B.tgs_tile_features(vb.ranges, E, A, vb.height, vb.width, cam, s["Xa"])
        s["t"].copy_(s["Xa"][:, 19])
        self.steps += 1
        B.tgs_tile_mlp_train_step(self.params, self.m, self.v, s["X"], s["act"], s["y"], s["t"], self.n_t,
                                  self.steps, self.lr, self.ws)
        self.ranges[v].copy_(vb.ranges)


class Trainer:
    """Gaussians, optimizer state and per-view buffers for sparse (or dense)
    training steps over a fixed set of cameras."""

    SAMPLE_STREAMS = 4   # streams the views' samplers are spread over

    def __init__(self, params: torch.Tensor, cams, gts, cfg: StepConfig, E=None, A=None):
        if cfg.deterministic and cfg.density_stats:
            raise ValueError("the deterministic backward has no density-control variant")
        self.dev = params.device
        self.params = params.contiguous()
        self.n = params.shape[1]
        # the moments are Gaussian-major, [n][MOMENT_STRIDE] (see moments())
        self.m = torch.zeros((self.n, B.MOMENT_STRIDE), dtype=torch.float32, device=self.dev)
        self.v = torch.zeros_like(self.m)
        self.grad = torch.zeros_like(self.params)
        self.touched = torch.zeros(self.n, dtype=torch.uint8, device=self.dev)
        self.cams = [B.camera(c) for c in cams]
        self.gts = gts
        self.cfg = cfg
        self.rp = B.raster_params(**cfg.raster)
        self.lp = B.loss_params(**cfg.loss)
        self.op = B.optim_params(**cfg.optim)
        self.E, self.A = E, A
        self.totals = torch.zeros(2, dtype=torch.int64, device=self.dev)
        self.step_count = 0
        self._bufs: dict = {}
        self.counters = torch.zeros((2, B.COUNTER_SLOTS), dtype=torch.int64, device=self.dev)
        self.side = torch.cuda.Stream(device=self.dev)  # default priority
        self.fused_ws = torch.empty(B.tgs_project_bwd_optimizer_workspace_size(self.n), dtype=torch.uint8,
                                    device=self.dev)
        self.events: dict | None = None   # stage name -> [(start, end)] when timing
        self.timed_stages: set | None = None  # stages to time (all when None)
        self.tiles: TilePriority | None = None
        # density-control sums [E, W, D, -] per Gaussian (cleared by reset_density)
        self.dstats = torch.zeros((self.n, 4), dtype=torch.float32, device=self.dev) if cfg.density_stats else None
        # screen-space gradient statistics [sum |dL/d centre|, views, max radius, -]
        self.gstats = torch.zeros((self.n, 4), dtype=torch.float32, device=self.dev) if cfg.density_stats else None
        self._select_ws = None   # percentile-selection workspace, made on first use
        if cfg.learned_tiles and cfg.rate_permille is not None and cfg.n_tiles_sel > 0:
            c0 = self.cams[0]
            n_t = ((c0.width + TILE - 1) // TILE) * ((c0.height + TILE - 1) // TILE)
            assert all(c.width == c0.width and c.height == c0.height for c in self.cams), "one image size"
            self.tiles = TilePriority(len(self.cams), n_t, cfg, self.dev)
        # cross-stream events, recorded anew each step (a wait binds to the
        # record queued before it)
        self._sampled: list = []           # per view slot: its sampler's completion
        self._sample_streams: list = []
        self._view_streams: list = []
        self._lossed: list = []            # per view slot: its loss (the error maps' update waits)
        self._done: list = []              # per view slot: its loss (with view streams)
        self._cleared = None               # main after a step's clears (with view streams)
        self._pending: list = []   # (event, pinned counts, [(view buffers, capacity)]) per step

    def _stage(self, name):
        """Brackets a stage with HIP events on the current stream when timing."""
        if self.events is None or (self.timed_stages is not None and name not in self.timed_stages):
            return _NO_STAGE
        return self._timed_stage(name)

    @contextlib.contextmanager
    def _timed_stage(self, name):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        yield
        b.record()
        self.events.setdefault(name, []).append((a, b))

    def stage_ms(self) -> dict:
        """Total milliseconds per stage over the recorded events (synchronises)."""
        torch.cuda.synchronize()
        return {k: sum(a.elapsed_time(b) for a, b in v) for k, v in (self.events or {}).items()}

    def stage_samples_ms(self) -> dict:
        """Every recorded duration per stage, in milliseconds (synchronises)."""
        torch.cuda.synchronize()
        return {k: [a.elapsed_time(b) for a, b in v] for k, v in (self.events or {}).items()}

    def buffers(self, key, cam, rate_permille: int | None = None) -> ViewBuffers:
        """Buffers of view slot ``key`` at the configured rate, or at
        ``rate_permille``.  A slot keeps one buffer set, keyed by its pixels
        per tile (rates that give the same count share it); a new count
        replaces the set and starts the pair arrays at the old capacity."""
        rate = self.cfg.rate_permille if rate_permille is None else rate_permille
        n_pix = None if rate is None else B.tgs_pixels_per_tile(rate)
        old = self._bufs.get(key)
        if old is not None and old.n == self.n and old.width == cam.width and old.height == cam.height \
                and (old.n_pix if not old.dense else None) == n_pix:
            return old
        cap = old.capacity if old is not None and old.n == self.n else None
        if old is not None:
            torch.cuda.synchronize(self.dev)   # its arrays may be in use on a view stream
            del self._bufs[key]
        self._bufs[key] = ViewBuffers(self.n, cam.width, cam.height, n_pix, self.cfg.n_tiles_sel, self.dev,
                                      capacity=cap)
        return self._bufs[key]

    def init_error_maps(self, views):
        """Dense L1 error of the current model per view (Sec. 3.3 initialisation)."""
        bufs = {}   # one dense buffer set per image size
        for v in views:
            cam = self.cams[v]
            vb = bufs.get((cam.width, cam.height))
            if vb is None:
                vb = bufs[(cam.width, cam.height)] = ViewBuffers(self.n, cam.width, cam.height, None, -1, self.dev)
            vb.project(self.params, cam, self.rp)
            vb.bin_sort(alpha_min=self.rp.alpha_min)
            vb.render_fwd(self.rp)
            B.tgs_error_init(vb.out, self.gts[v], cam.height, cam.width, self.E[v])

    def step(self, views, rate_permille: int | None = None) -> list:
        """One training step over ``views`` (at ``rate_permille`` if given,
        else the configured rate); returns the per-view buffers."""
        self.check_counts()
        self.step_count += 1
        t = self.step_count
        views = list(views)
        main, side = torch.cuda.current_stream(), self.side
        if not views:
            self.grad.zero_()
        st = self._stage
        used = [self.buffers(slot, self.cams[v], rate_permille) for slot, v in enumerate(views)]
        slot_of = {id(vb): k for k, vb in enumerate(used)}
        views_fused = self.cfg.fuse_views
        self.touched.zero_()
        # the sample totals are cleared (dense views' counts added) on main;
        # then each sparse view's sampler runs on a stream of its own (which
        # sees everything queued on main so far), so the views' tile passes
        # run side by side and beside the first projection
        self.totals.zero_()
        for vb, v in zip(used, views):
            if vb.dense:
                self.totals[0] += self.cams[v].width * self.cams[v].height
                self.totals[1] += vb.n_t
        par = self.cfg.view_streams > 1
        prefix_n = None
        if self.cfg.prefix_fraction is not None and not self.cfg.deterministic:
            prefix_n = max(1, int(math.ceil(self.cfg.prefix_fraction * self.n)))
        sampled: list = []   # filled below, read by the chains' later stages
        S = self.cfg.view_streams

        def chains_of(g0):
            # the view streams wait for the previous step and this step's
            # clears (the _cleared event), not for the samplers queued on main
            out = []
            for k in range(g0, min(g0 + S, len(used))):
                vs = self._view_stream(k)
                vs.wait_event(self._cleared)
                while len(self._done) <= k:
                    self._done.append(torch.cuda.Event())
                out.append((vs, self._view_chain(k, used[k], views[k], self.cams[views[k]], sampled, prefix_n, vs,
                                                 self._done[k])))
            return out

        def advance(chains, once=False):
            while chains:
                for c in list(chains):
                    with torch.cuda.stream(c[0]):
                        if next(c[1], StopIteration) is StopIteration:
                            chains.remove(c)
                if once:
                    return

        first = []
        if par:
            if self._cleared is None:
                self._cleared = torch.cuda.Event()
            self._cleared.record(main)
            # the first views' projections are queued before the samplers
            first = chains_of(0)
            advance(first, once=True)
        for k, (vb, v) in enumerate(zip(used, views)):
            if vb.dense:
                sampled.append(None)
                continue
            # views side by side: a sampler over every tile is short and runs
            # on main (idle until the first backward) beside the projections;
            # drawing a tile subset is one long workgroup per view, so those
            # run on the view streams (after the view's projection), side by side
            if par:
                ss = self._view_stream(k) if self.cfg.n_tiles_sel > 0 else main
            else:
                ss = self._sample_stream(k)
                ss.wait_stream(main)
            with torch.cuda.stream(ss):
                cam = self.cams[v]
                pred = None
                if self.tiles is not None:
                    pred = self.tiles.predict(slot_of[id(vb)], v, self.E[v], self.A[v], vb, cam)
                with st("sample"):
                    vb.sample(self.E[v], self.A[v], self.cfg, t, v, self.totals, tile_pred=pred)
                while len(self._sampled) <= k:
                    self._sampled.append(torch.cuda.Event())
                ev = self._sampled[k]
                ev.record(ss)
            sampled.append(ev)
        # each view's chain, projection to loss: on main, or (view_streams >
        # 1) on a stream per view, the views side by side; the backward and
        # what sums over views in place (screen-gradient statistics, the
        # per-view projection backward into the gradient array) run on main
        # in view order, the backward of a view once its loss is queued
        if par:
            # enqueued breadth first, a stage of every view in turn, so each
            # stream has work queued soon after the step starts (views that
            # share a stream go in consecutive rounds)
            advance(first)
            for g0 in range(S, len(used), S):
                advance(chains_of(g0))
        for k, (vb, v) in enumerate(zip(used, views)):
            cam = self.cams[v]
            if par:
                main.wait_event(self._done[k])
            else:
                for _ in self._view_chain(k, vb, v, cam, sampled, prefix_n, main):
                    pass
            with st("render_bwd"):
                # g2d was cleared by the projection; the density sums of sparse
                # views join the backward's reduction
                vb.render_bwd(self.rp, zero=False, stats=None if vb.dense else self.dstats, touched=self.touched,
                              deterministic=self.cfg.deterministic)
            if self.gstats is not None:
                B.tgs_grad_screen_accumulate(vb.g2d, vb.radius, self.n, cam.width, cam.height, self.gstats)
            if views_fused:
                pass   # every view's chain rule joins the update after the loop
            elif k + 1 < len(used) or not self.cfg.fuse_optimizer:
                with st("project_bwd"):
                    # the first view overwrites the gradient, later views add to it
                    vb.project_bwd(self.params, cam, self.rp, self.grad, accumulate=k > 0)
            else:
                # the last view's chain rule feeds the update directly
                with st("project_bwd_optimizer"):
                    B.tgs_project_bwd_optimizer_step(self.params, self.n, cam, self.rp, vb.radius, vb.clamp,
                                                     vb.g2d, self.grad if k > 0 else None, self.m, self.v,
                                                     self.touched, self.op, t, self.fused_ws)
        if views_fused:
            need = B.tgs_project_bwd_optimizer_views_workspace_size(self.n, len(used))
            if getattr(self, "views_ws", None) is None or self.views_ws.numel() < need:
                self.views_ws = torch.empty(need, dtype=torch.uint8, device=self.dev)
            with st("project_bwd_optimizer"):
                B.tgs_project_bwd_optimizer_step_views(self.params, self.n, [self.cams[v] for v in views], self.rp,
                                                       [vb.radius for vb in used], [vb.clamp for vb in used],
                                                       [vb.g2d for vb in used], self.m, self.v, self.touched,
                                                       self.op, t, self.views_ws)
        elif not used or not self.cfg.fuse_optimizer:
            with st("optimizer"):
                B.tgs_optimizer_step(self.params, self.grad, self.m, self.v, self.n, self.touched, self.op, t)
        main.wait_stream(side)
        if par:
            for vs in self._view_streams:
                main.wait_stream(vs)   # their error-map updates, before the next step samples
        self._queue_count_check(used)
        return used

    def _view_chain(self, k, vb, v, cam, sampled, prefix_n, vs, done=None):
        """Projection, binning, forward and loss of the step's k-th view on
        stream ``vs`` (the current stream).  With ``done`` (views side by
        side) the event is recorded after the loss and the error maps'
        update follows on ``vs`` itself: a wait queued on the side stream
        would hold up whatever view stream shares its hardware queue.  A
        generator: it yields after each stage, with the stream set by the
        caller around every resumption."""
        st = self._stage
        with st("project"):
            vb.project(self.params, cam, self.rp)
        yield
        if sampled[k] is not None and vb.bin_sort_needs_samples():
            vs.wait_event(sampled[k])   # binning keeps the sampled tiles only
        with st("bin_sort"):
            if prefix_n is not None:
                # the nearest Gaussians only; the first step of a slot waits to size its arrays
                vb.bin_sort_prefix(prefix_n, None, self.rp.alpha_min, wait=not vb.sized)
            elif vb.sized:
                vb.bin_sort_async(None, self.rp.alpha_min)   # no host wait
            else:
                vb.bin_sort(None, self.rp.alpha_min)         # sizes the pair arrays once per slot
        yield
        if sampled[k] is not None:
            vs.wait_event(sampled[k])   # the forward renders this view's samples
        if vb.two_part:
            # prefix forward, the marked tiles' continuation lists, their forward
            with st("render_fwd"):
                vb.render_fwd_prefix(self.rp, self.counters)
            yield
            with st("bin_sort"):
                vb.continue_lists(self.rp.alpha_min, wait=not vb.sized)
            yield
            with st("render_fwd"):
                vb.render_fwd_cont(self.rp, self.counters)
            vb.sized = True
        else:
            with st("render_fwd"):
                vb.render_fwd(self.rp, self.counters)
        yield
        # the loss normalises by the step's total sample count
        for ev in sampled:
            if ev is not None:
                vs.wait_event(ev)
        with st("loss"):
            vb.loss(self.gts[v], self.totals, self.lp)
        if done is not None:
            done.record(vs)
        if not vb.dense and done is not None and self.tiles is None:
            with st("ema_age"):
                vb.ema_age(self.E[v], self.A[v], self.cfg.beta)
        elif not vb.dense:
            while len(self._lossed) <= k:
                self._lossed.append(torch.cuda.Event())
            self._lossed[k].record(vs)
            self.side.wait_event(self._lossed[k])
            with torch.cuda.stream(self.side):
                with st("ema_age"):
                    vb.ema_age(self.E[v], self.A[v], self.cfg.beta)
                if self.tiles is not None:
                    self.tiles.learn(k, v, self.E[v], self.A[v], vb, cam)

    def _view_stream(self, k: int):
        """Stream of the k-th view's sampler and chain when views run side
        by side (default priority; view_streams of them, reused round-robin)."""
        while len(self._view_streams) < min(k + 1, self.cfg.view_streams):
            self._view_streams.append(torch.cuda.Stream(device=self.dev))
        return self._view_streams[k % self.cfg.view_streams]

    def _sample_stream(self, k: int):
        """Stream of the k-th view's sampler (default priority; a few reused
        round-robin)."""
        while len(self._sample_streams) < min(k + 1, self.SAMPLE_STREAMS):
            self._sample_streams.append(torch.cuda.Stream(device=self.dev))
        return self._sample_streams[k % self.SAMPLE_STREAMS]

    # ---- pair-capacity watch: the asynchronous bin/sort reports its counts on
    # the device; they are copied to pinned host memory after each step and
    # read two steps later (by then the device has finished that step), so
    # the step loop never waits for them.  A view whose lists needed more
    # than 85% of its capacity gets larger pair arrays before its next step;
    # one that overflowed (its lists came out empty) raises.
    _COUNT_LAG = 2

    def _queue_count_check(self, used):
        if not used:
            return
        host = torch.zeros((len(used), 5), dtype=torch.int64, pin_memory=True)
        for k, vb in enumerate(used):
            host[k, :3].copy_(vb.counts, non_blocking=True)
            if vb.two_part:
                host[k, 3:].copy_(vb.counts2, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        self._pending.append((ev, host, [(vb, vb.capacity, vb.capacity2, vb.two_part) for vb in used]))

    def check_counts(self, wait_all: bool = False):
        """Reads the pending pair counts that are due (all of them with
        ``wait_all``), growing capacities and raising on an overflow."""
        while self._pending and (wait_all or len(self._pending) > self._COUNT_LAG or self._pending[0][0].query()):
            ev, host, entries = self._pending.pop(0)
            ev.synchronize()
            for (vb, cap, cap2, two), (valid, need, whole, valid2, need2) in zip(entries, host.tolist()):
                if need > cap or (two and need2 > cap2):
                    raise B.CapacityError(f"a step's pair lists needed {need} (continuation {need2}) entries but "
                                          f"had {cap} ({cap2}): that step rendered empty lists and must be redone "
                                          f"with a larger capacity", max(need, need2))
                if not two:
                    if vb.capacity == cap and need > 0.85 * cap:
                        vb._alloc_pairs(int(1.5 * need) + 1024)
                    continue
                if vb.capacity == cap and need > 0.7 * cap:
                    vb._alloc_pairs(int(vb.PREFIX_MARGIN * need) + 1024)
                want2 = max(int(1.5 * need2), int(vb.CONT_MIN_SHARE * whole)) + 1024
                if vb.capacity2 == cap2 and (need2 > 0.7 * cap2 or cap2 < vb.CONT_MIN_SHARE * whole):
                    vb._alloc_cont(want2)

    def reset_density(self):
        """Clears the density-control sums (the start of an accumulation window)."""
        self.dstats.zero_()
        self.gstats.zero_()

    def grad_screen_mean(self):
        """Mean 2D centre gradient norm per view in which each Gaussian was projected."""
        out = torch.empty(self.n, dtype=torch.float32, device=self.dev)
        B.tgs_grad_screen_mean(self.gstats, self.n, out)
        return out

    def density_scores(self, lambda_base: float, rho: float, eps: float = 1e-8):
        """Eq. gauss_score over the sums accumulated since the last reset:
        (e, d, s) per Gaussian."""
        e, d, sc = (torch.empty(self.n, dtype=torch.float32, device=self.dev) for _ in range(3))
        B.tgs_density_score(self.dstats, self.n, lambda_base, rho, eps, e, d, sc)
        return e, d, sc

    def density_select(self, lambda_base: float, rho: float, eta_topk: float, eta_final: float,
                       eps: float = 1e-8, tau_grad: float | None = None, tau_grad_abs: float | None = None,
                       prune: bool = True):
        """The selections of one density step over the current sums: the
        percentile thresholds of the score (densify where s_i reaches the
        k-th largest, k = max(1, ceil((1 - eta_topk) n)); keep where it
        reaches the k-th largest with k = max(1, ceil(eta_final n)); ties are
        selected), densification gated by the gradient thresholds (skipped
        when tau_grad is None), and keep = 1 everywhere when ``prune`` is
        off.  rho is the training progress of Eq. gauss_score.  Returns
        (densify, keep) uint8 masks, the two thresholds and the scores."""
        e, d, sc = self.density_scores(lambda_base, rho, eps)
        if self._select_ws is None:
            self._select_ws = torch.empty(B.tgs_select_workspace_size(), dtype=torch.uint8, device=self.dev)
        thr = torch.empty(2, dtype=torch.float32, device=self.dev)
        masks = torch.empty((2, self.n), dtype=torch.uint8, device=self.dev)
        for j, frac in enumerate((1.0 - eta_topk, eta_final)):
            k = max(1, math.ceil(frac * self.n - 1e-9))
            B.tgs_select_kth_largest(sc, self.n, k, thr[j:j + 1], self._select_ws)
        if tau_grad is None:
            # ungated: the two percentile masks alone
            B.tgs_threshold_mask(sc, self.n, thr[0:1], masks[0])
            if prune:
                B.tgs_threshold_mask(sc, self.n, thr[1:2], masks[1])
            else:
                masks[1].fill_(1)
        else:
            B.tgs_density_masks(sc, self.gstats, self.dstats, self.n, thr, tau_grad,
                                float("inf") if tau_grad_abs is None else tau_grad_abs, prune, masks[0], masks[1])
        return masks[0], masks[1], thr, (e, d, sc)

    def densify_and_prune(self, densify, keep, z, log_split: float):
        """Applies the selections (tgs_density_topology_*): the Gaussians,
        their moments and every per-Gaussian buffer move to the new count;
        the density sums restart.  z: [n, 3] standard normal draws for the
        splits.  Returns the new count."""
        ws = torch.empty(B.tgs_density_topology_workspace_size(self.n), dtype=torch.uint8, device=self.dev)
        n_keep, n_new = B.tgs_density_topology_count(keep, densify, self.n, ws)
        n_out = n_keep + n_new
        p_out = torch.empty((self.params.shape[0], n_out), dtype=torch.float32, device=self.dev)
        m_out, v_out = (torch.empty((n_out, B.MOMENT_STRIDE), dtype=torch.float32, device=self.dev)
                        for _ in range(2))
        B.tgs_density_topology_apply(self.params, self.m, self.v, self.n, z.contiguous(), log_split, ws,
                                     p_out, m_out, v_out, n_out)
        self.params, self.m, self.v, self.n = p_out, m_out, v_out, n_out
        self.grad = torch.zeros_like(self.params)
        self.touched = torch.zeros(self.n, dtype=torch.uint8, device=self.dev)
        self.fused_ws = torch.empty(B.tgs_project_bwd_optimizer_workspace_size(self.n), dtype=torch.uint8,
                                    device=self.dev)
        if self.dstats is not None:
            self.dstats = torch.zeros((self.n, 4), dtype=torch.float32, device=self.dev)
            self.gstats = torch.zeros((self.n, 4), dtype=torch.float32, device=self.dev)
        self._bufs = {}   # per-view buffers are sized by the Gaussian count
        return n_out

    def moments(self):
        """The Adam moments m, v in the parameter layout, [59][n] views of
        the Gaussian-major arrays."""
        return self.m[:, :B.PARAM_ROWS].T, self.v[:, :B.PARAM_ROWS].T

    def loss_value(self, used) -> float:
        return float(sum(vb.tile_loss[: vb.n_st].sum() for vb in used))
