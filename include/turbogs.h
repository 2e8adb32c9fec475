/*
 * turbogs.h - C ABI of the MI355X (gfx950) sparse-pixel Gaussian rasterizer.
 *
 * The library implements the per-iteration hot path of error-guided sparse
 * pixel training of 3D Gaussian Splatting (TurboGS, arXiv 2606.15924):
 * projection with SH colour, tile x depth binning and sort, tile-wise
 * error/age pixel sampling (Sec. 3.5), compositing of only the sampled
 * pixels (Sec. 3.6), the sparse Charbonnier + tile NCC loss (Sec. 3.7),
 * the error/age map update (Sec. 3.3), the adjoint backward, and the hybrid
 * moment-damped LM / Adam update (Sec. 3.9).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a device pointer owned by the caller unless
 *     stated otherwise.  The library never allocates device
 *     memory; scratch space comes from a caller workspace sized by the
 *     matching *_workspace_size function.  Struct arguments (camera and
 *     parameter records) are host pointers read during the call.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     null stream).  Only tgs_bin_sort synchronises (it returns the pair
 *     count; tgs_bin_sort_async writes it to device memory instead), and the
 *     density-control count call that returns sizes.
 *   - Return value: TGS_OK, or a negative error (TGS_ERR_INVALID for a null
 *     pointer or a bad size, TGS_ERR_HIP for a failed launch/runtime call) or
 *     TGS_ERR_CAPACITY (an output is too small; the required count is written
 *     to the named host out-parameter).  tgs_last_error() returns a message
 *     describing the last failure of the calling thread.
 *   - Gaussian parameters live in one float array params[59][n] (row r of
 *     Gaussian i at params[r * n + i]):
 *       rows 0-2 mean xyz; 3-5 log-scale; 6-9 quaternion (w, x, y, z),
 *       unnormalised; 10 opacity logit; 11 + 3k + c SH coefficient k
 *       (k = 0..15, order l then m = -l..l) of colour channel c.
 *     Gradients use the same layout.  The optimizer's moments m, v are
 *     Gaussian-major, m[n][TGS_MOMENT_STRIDE] (the moment of row r of
 *     Gaussian i at m[i * TGS_MOMENT_STRIDE + r]; entries 59-63 are padding
 *     that no update reads or writes): an update touches a few percent of the
 *     Gaussians, and each one's moments then sit in two cache lines.
 *   - Images are tiled in 16 x 16 tiles; tiles_x = ceil(W/16),
 *     tiles_y = ceil(H/16); tile id = ty * tiles_x + tx; a pixel's local
 *     index inside its tile is ly * 16 + lx.
 *   - A sample set (one view) is valid_tiles[n_st] (ascending tile ids),
 *     tile_off[n_st + 1] (prefix offsets) and pix[P] (uint8 local indices,
 *     ascending within a tile).  Per-sample outputs are indexed by sample.
 *     Passing valid_tiles = NULL selects the dense mode: every tile, every
 *     in-image pixel, outputs indexed row-major by y * W + x.
 */
#ifndef TURBOGS_H
#define TURBOGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TGS_ABI_VERSION 12u
#define TGS_TILE 16
#define TGS_SPLAT_FLOATS 12  /* floats per projected splat record */
#define TGS_G2D_FLOATS 9     /* floats per screen-space gradient record */
#define TGS_PARAM_ROWS 59
#define TGS_MOMENT_STRIDE 64 /* floats per Gaussian in the moment arrays m, v */
#define TGS_COUNTER_SLOTS 64 /* slots per counter of tgs_render_fwd */
#define TGS_RENDER_CHUNKS 8     /* backward workgroups per tile when the forward keeps state */
#define TGS_RENDER_CHUNK_LEN 32 /* list positions per backward chunk (the last takes the rest) */

enum {
  TGS_OK = 0,
  TGS_ERR_CAPACITY = 1,
  TGS_ERR_INVALID = -1,
  TGS_ERR_HIP = -2
};

/* OpenCV pinhole camera: x right, y down, z forward.  R (row-major) and t
 * map a world point X to camera space R X + t. */
typedef struct tgs_camera {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
} tgs_camera;

/* Rasterizer constants the paper leaves to the 3DGS conventions. */
typedef struct tgs_raster_params {
  int32_t sh_degree;  /* 0..3 */
  float z_near;       /* cull t_z <= z_near */
  float dilation;     /* added to the 2D covariance diagonal, px^2 */
  float alpha_min;    /* skip alpha < alpha_min */
  float alpha_max;    /* alpha = min(alpha_max, o * G) */
  float T_min;        /* stop before T would fall below T_min */
  float bg[3];        /* background colour */
} tgs_raster_params;

/* Pixel sampling of one view (Sec. 3.5). */
typedef struct tgs_sample_params {
  int32_t n_pix;            /* N_pix per full tile, 1..256 */
  int32_t hard_permille;    /* r_hard in 1/1000 */
  int32_t stable_permille;  /* r_stable in 1/1000 */
  int32_t n_tiles_sel;      /* tiles drawn in proportion to error; < 0: all */
  uint64_t seed;
  uint64_t step;
  int32_t view;
  int32_t reserved;
} tgs_sample_params;

/* Tile structure term of the sparse loss: S-NCC (Sec. 3.7), or a sparse
 * SSIM over the tile's samples (the S-SSIM ablation of Tab. ablation_main). */
#define TGS_STRUCTURE_NCC 0
#define TGS_STRUCTURE_SSIM 1

typedef struct tgs_loss_params {
  float eps_charb;   /* Charbonnier epsilon */
  float eps_ncc;     /* added to V_x V_y under the NCC square root */
  float eps_lambda;  /* denominator guard of the balance weight */
  int32_t structure; /* TGS_STRUCTURE_NCC or TGS_STRUCTURE_SSIM */
} tgs_loss_params;

typedef struct tgs_optim_params {
  double lr_mean, lr_scale, lr_quat, lr_opacity, lr_sh_dc, lr_sh_rest;
  double beta1, beta2, eps_adam, eps_lm;
  int32_t lm_mode;  /* 0: J^T J = g g^T, 1: diag(g^2), 2: Adam for every row */
  int32_t reserved;
} tgs_optim_params;

uint32_t tgs_version(void);
const char* tgs_last_error(void);

/* Debug check of any float array the path reads or writes (parameters,
 * gradients, rendered colours): *count (one device int64) is set to the
 * number of entries of x[n] that are NaN or infinite.  Asynchronous, like
 * every other call; x must be 16-byte aligned, count 8-byte aligned.
 * The hot path itself never checks for non-finite values. */
int32_t tgs_check_finite(const float* x, int64_t n, int64_t* count, void* stream);

/* N_pix = max(1, floor(r * 256)) with r = rate_permille / 1000 (Sec. 3.5). */
int32_t tgs_pixels_per_tile(int32_t rate_permille);

/* Number of sampled tiles tgs_sample produces for this view and parameters
 * (host-side; sizes the per-tile outputs). */
int32_t tgs_sample_tile_count(int32_t height, int32_t width, const tgs_sample_params* sp);

/* EWA projection and SH colour (Sec. 3.1: each Gaussian is projected to a 2D
 * splat whose footprint and opacity give alpha; colour from SH coefficients).
 *   params   [59][n] float, read
 *   splat    [n][12] float, written: floor(px), floor(py), px - floor(px),
 *            py - floor(py), conic Q = [[a, b], [b, c]] in its LDL^T form
 *            a, beta = b / a, delta = det Q / a (so d^T Q d =
 *            a (dx + beta dy)^2 + delta dy^2, two non-negative terms, which
 *            an FP32 evaluation takes without cancellation), opacity,
 *            r, g, b, depth.  The centre is in pixel-index space (pixel
 *            (i, j) sits at offset (i, j) - centre).
 *   depth    [n] float (camera-space z, FP32)
 *   radius   [n] int32 (0 = culled)
 *   rect     [n][4] int32 tile rectangle xmin, ymin, xmax, ymax (exclusive)
 *   clamp    [n] uint8, bit c set when colour channel c was clamped at 0
 *   g2d_clear  nullable [n][9] float, set to zero (the screen-space gradient
 *            accumulator that tgs_render_bwd adds to, cleared in the same
 *            pass over the Gaussians)
 * The projection is computed in FP64; depth bits, centre and rectangle
 * follow a fixed operation order. */
int32_t tgs_project(const float* params, int64_t n, const tgs_camera* cam,
                    const tgs_raster_params* rp, float* splat, float* depth,
                    int32_t* radius, int32_t* rect, uint8_t* clamp, float* g2d_clear,
                    void* stream);

/* Tile-wise error/age pixel sampling (Sec. 3.5, Eq. pix_prob_err and
 * Eq. pix_topk_age, plus the mixed remainder of the hyper-parameter table).
 *   E, A        [H][W] uint16: half-precision error bits, age (read)
 *   tile_pred   nullable [tiles_x * tiles_y] float: predicted mean tile
 *               errors (tgs_tile_mlp_fwd); when given, the tile pass draws
 *               in proportion to floor(clamp(p, 0, 65504) * in-image pixels
 *               * 2^24) instead of the error-map sums (same units)
 *   valid_tiles [n_st] int32, tile_off [n_st + 1] int32 (written)
 *   pix         [n_st * n_pix] uint8 capacity (written up to tile_off[n_st])
 *   tile_slot   [tiles_x * tiles_y] int32: slot of each tile or -1 (written)
 *   totals      [2] int64 device counters: += P and += n_st of this view
 *               (the caller zeroes them once per training step)
 *   ws          workspace of tgs_sample_workspace_size(H, W) bytes (8 per
 *               tile: the race keys)
 * With 0 <= n_tiles_sel < tiles, the tile pass draws that many tiles without
 * replacement in proportion to weight (uniform over the rest once the weight
 * runs out) as an exponential race (Efraimidis and Spirakis 2006): the tiles
 * of the smallest keys L / w win, L the tile's -log2 uniform to 47 fractional
 * bits, computed exactly in integer and IEEE double arithmetic.
 * Deterministic: counter-based SplitMix64 draws keyed by (seed, step, view,
 * tile, slot). */
size_t tgs_sample_workspace_size(int32_t height, int32_t width);
int32_t tgs_sample(const uint16_t* E, const uint16_t* A, int32_t height, int32_t width,
                   const tgs_sample_params* sp, const float* tile_pred, int32_t* valid_tiles,
                   int32_t* tile_off, uint8_t* pix, int32_t* tile_slot, int64_t* totals, void* ws,
                   size_t ws_bytes, void* stream);

/* tgs_sample for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same sampling, outputs and errors, with the workspace taken from a
 * static device array of the library (8 bytes per tile for at most
 * TGS_SAMPLE_NOALLOC_MAX_TILES tiles, 512 KiB, held on each GPU the library
 * runs on until the process ends) instead of a caller buffer.  Calls no
 * allocating routine.  Images of more tiles are rejected with
 * TGS_ERR_INVALID before anything is queued.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (several streams or host
 * threads) race and must be ordered by the caller. */
#define TGS_SAMPLE_NOALLOC_MAX_TILES 65536 /* e.g. 4096 x 4096 pixels */
int32_t tgs_sample_noalloc(const uint16_t* E, const uint16_t* A, int32_t height, int32_t width,
                           const tgs_sample_params* sp, const float* tile_pred, int32_t* valid_tiles,
                           int32_t* tile_off, uint8_t* pix, int32_t* tile_slot, int64_t* totals, void* stream);

/* Tile x depth binning, sort and per-tile ranges (the depth-ordered
 * per-tile Gaussian lists of Eq. alpha_comp, in the tile order of Sec. 3.6).
 * A (Gaussian, tile) pair is listed when the tile lies in the Gaussian's
 * tile rectangle and its pixel-centre rectangle meets the ellipse
 * q(d) <= t of the splat's centre and conic (d measured from the centre,
 * q = a dx^2 + 2 b dx dy + c dy^2; t = 2 ln(o/alpha_min) + 0.004 for the
 * splat's opacity o, rounded up to a multiple of 1/64 and at most
 * tau = 2 ln(1/alpha_min) x 1.001 rounded likewise): alpha = o exp(-q/2)
 * stays below alpha_min (by 0.2 %) outside it, so no dropped pair can reach
 * alpha_min at any pixel of its tile and the lists composite exactly like
 * the rectangle lists.  The kept tiles of a tile row are one interval of columns, found
 * in FP64 from the ellipse's x-extent over the row's pixel-centre strip.
 *   rect, splat, depth  projection outputs of n Gaussians
 *   tile_slot    nullable: only tiles with tile_slot >= 0 receive pairs
 *   alpha_min    the compositing threshold (as in tgs_raster_params)
 *   keys         nullable [capacity] uint64: (tile << 32) | bits(depth) of
 *                each sorted pair
 *   vals         [capacity] uint32: Gaussian ids ordered by (tile, depth
 *                bits, id)
 *   ranges       [tiles_x * tiles_y][2] uint32 [start, end), [0, 0) if empty
 *   touched      nullable [n] uint8: set to 1 for Gaussians with a pair;
 *                other entries are left as they are, so one array
 *                cleared once collects the Gaussians of several views
 *                (tgs_render_bwd marks the narrower set of Gaussians
 *                composited at a sample)
 *   n_pairs      host out: number of pairs in valid tiles
 * capacity must hold the pairs in valid tiles (only those are listed);
 * when it does not, the lists come out empty (every range [0, 0); vals and
 * keys untouched) and the call returns TGS_ERR_CAPACITY with that count in
 * *n_pairs.  Every kernel's grid is
 * sized by the capacity and reads the pair count on the device, so the
 * work is queued without waiting; this call then waits for the stream once
 * (a copy of the two counts into host memory) to return them.  The library
 * keeps no host or device memory of its own for it. */
size_t tgs_bin_sort_workspace_size(int64_t n, int64_t capacity, int32_t n_tiles);
int32_t tgs_bin_sort(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                     const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y, float alpha_min,
                     uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* ranges,
                     uint8_t* touched, int64_t* n_pairs, void* ws, size_t ws_bytes,
                     void* stream);

/* tgs_bin_sort without any host synchronisation: the same lists, with the
 * counts written to device memory instead of returned.
 *   counts  [2] int64, device, 8-byte aligned: counts[0] = pairs in valid
 *           tiles (the lists' length), counts[1] = the capacity the call
 *           needs (the same number: only valid tiles are listed).  When
 *           counts[1] > capacity the lists are empty, as above; the caller
 *           finds out when it next reads counts (after its own
 *           synchronisation), and a step rendered from such lists must be
 *           redone with a larger capacity.
 * Argument errors are still reported before anything is queued. */
int32_t tgs_bin_sort_async(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                           const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y, float alpha_min,
                           uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* ranges,
                           uint8_t* touched, int64_t* counts, void* ws, size_t ws_bytes, void* stream);

/* Depth-prefix lists (an exact shortcut for the forward walk's early
 * stop): the lists of tgs_bin_sort_async restricted to the first `prefix`
 * Gaussians in (depth, id) order (Gaussians with a non-empty rectangle,
 * the others after them), i.e. the first part of every tile's list; only
 * those are counted.  A pixel whose walk stops (T_min) within its prefix composites as
 * with the whole list; tgs_render_fwd_prefix marks the tiles where one does
 * not, tgs_bin_sort_continue_async lists the rest of those tiles' Gaussians
 * and tgs_render_fwd_cont redoes them over both parts, so the images,
 * counts and gradients equal those of the whole lists.  Arguments as
 * tgs_bin_sort_async except touched (only the prefix's Gaussians with a
 * pair are flagged) and counts: [3] int64 device, counts[0] = the lists'
 * length, counts[1] = the pairs the prefix emits (the capacity it needs),
 * counts[2] = an estimate of the whole lists' pairs for sizing a
 * continuation: the prefix's pairs per Gaussian times the Gaussians with a
 * rectangle (exact when the prefix holds them all; the nearest Gaussians
 * cover the most tiles, so it tends to exceed the true count).  The
 * workspace keeps the depth order for the continuation call; prefix >= n
 * gives the whole lists. */
int32_t tgs_bin_sort_prefix_async(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                                  const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y, float alpha_min,
                                  int64_t prefix, uint64_t* keys, uint32_t* vals, int64_t capacity,
                                  uint32_t* ranges, uint8_t* touched, int64_t* counts, void* ws, size_t ws_bytes,
                                  void* stream);

/* The continuation of depth-prefix lists: for every tile with
 * flag_slot[tile] >= 0, the pairs of the Gaussians from depth rank `prefix`
 * on (same culling), each tile's list in (depth, id) order.
 *   flag_slot  [tiles_x * tiles_y] int32 (tgs_render_fwd_prefix's cont_slot)
 *   n_flagged  nullable [1] uint32 device: the number of flagged tiles
 *              (cont_count); when it is 0 the kernels return at once
 *   capacity, ws, ws_bytes  the prefix call's (its depth order is read)
 *   vals2, capacity2, ranges2  the continuation lists, as vals/ranges
 *   counts2    [2] int64 device: both = the continuation pairs; above
 *              capacity2 the lists come out empty, as in tgs_bin_sort_async
 *   ws2        tgs_bin_sort_workspace_size(n, capacity2, n_tiles) bytes */
int32_t tgs_bin_sort_continue_async(const float* splat, int64_t n, const int32_t* flag_slot,
                                    const uint32_t* n_flagged, int32_t tiles_x, int32_t tiles_y, float alpha_min,
                                    int64_t prefix, int64_t capacity,
                                    const void* ws, size_t ws_bytes, uint32_t* vals2, int64_t capacity2,
                                    uint32_t* ranges2, int64_t* counts2, void* ws2, size_t ws2_bytes, void* stream);

/* Front-to-back compositing of the sampled pixels of the sampled tiles
 * (Eq. alpha_comp; Sec. 3.6 tile-parallel forward with prefix-sum pixel
 * offsets).  valid_tiles = NULL: dense mode (n_st ignored).
 *   max_per_tile  largest per-tile sample count (sizes the workgroup)
 *   out       [P][4] float: r, g, b (including T_final * bg), T_final
 *   ncontrib  [P] uint32: range position of the last composited Gaussian + 1
 *   counters  nullable [2][TGS_COUNTER_SLOTS] uint64: evaluations are added
 *             to row 0 and blends to row 1, spread over the slots (a
 *             workgroup adds to slot blockIdx mod TGS_COUNTER_SLOTS, which
 *             keeps same-address atomics rare); the totals are the row sums
 *   state     nullable, tgs_render_state_size(n_slots, max_per_tile) bytes
 *             (n_slots = n_st, or tiles_x * tiles_y in dense mode with
 *             max_per_tile 256), 16-byte aligned: each pixel's transmittance
 *             and accumulated colour (float4 T, r, g, b) at list positions
 *             c * TGS_RENDER_CHUNK_LEN, c = 1 .. TGS_RENDER_CHUNKS - 1, where
 *             the walk reaches them; lets tgs_render_bwd split each tile's
 *             replay into chunks */
size_t tgs_render_state_size(int32_t n_slots, int32_t max_per_tile);
int32_t tgs_render_fwd(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                       int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                       const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                       int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                       float* out, uint32_t* ncontrib, uint64_t* counters, float* state,
                       void* stream);

/* tgs_render_fwd over depth-prefix lists that also marks the tiles with a
 * pixel whose walk ran off the end of its list without the T_min stop:
 *   cont_slot   [tiles_x * tiles_y] int32, written: the tile's slot (its
 *               index in valid_tiles, or the tile in dense mode) when
 *               marked, else -1
 *   cont_list   [n_st, or tiles_x * tiles_y in dense mode] uint32: the
 *               marked slots, in no particular order
 *   cont_count  [1] uint32 device: their number
 * counters count only the pixels that stopped (tgs_render_fwd_cont counts
 * the others). */
int32_t tgs_render_fwd_prefix(const float* splat, const uint32_t* vals, const uint32_t* ranges, int32_t tiles_x,
                              int32_t tiles_y, int32_t width, int32_t height, const int32_t* valid_tiles,
                              const int32_t* tile_off, const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                              const tgs_raster_params* rp, float* out, uint32_t* ncontrib, uint64_t* counters,
                              float* state, int32_t* cont_slot, uint32_t* cont_list, uint32_t* cont_count,
                              void* stream);

/* tgs_render_fwd for the slots cont_list[0 .. *cont_count) over two-part
 * lists (each tile's list is vals[ranges[t]] followed by vals2[ranges2[t]];
 * list positions, ncontrib and the state record count across both parts):
 * rewrites those slots' outputs and state; counters count the pixels that
 * had not stopped within the first part. */
int32_t tgs_render_fwd_cont(const float* splat, const uint32_t* vals, const uint32_t* ranges, const uint32_t* vals2,
                            const uint32_t* ranges2, int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                            const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix, int32_t n_st,
                            int32_t max_per_tile, const tgs_raster_params* rp, const uint32_t* cont_list,
                            const uint32_t* cont_count, float* out, uint32_t* ncontrib, uint64_t* counters,
                            float* state, void* stream);

/* Exact adjoint of tgs_render_fwd for the same samples (Sec. 3.6 backward
 * over sampled pixels only).  Per-pixel state is recomputed front to back
 * from the tile ranges and the forward outputs; nothing per Gaussian is
 * saved.
 *   dL_dout  [P][4] float (channel 3 ignored)
 *   g2d      [n][9] float, accumulated (+=): dL/d(centre x, y; conic a, b, c;
 *            opacity; r, g, b)
 *   state    nullable: the forward's state record for the same call
 *            arguments.  Given, each tile's replay runs as TGS_RENDER_CHUNKS
 *            workgroups, chunk c starting at list position
 *            c * TGS_RENDER_CHUNK_LEN from the recorded state (the last chunk
 *            takes the rest of the list); the per-pixel arithmetic is the
 *            same as the single-workgroup replay, only the order of the
 *            gradient atomics differs.
 *   touched  nullable [n] uint8: set to 1 for every Gaussian composited at
 *            one of the samples (the Gaussians the step's gradient reaches:
 *            the set the sparse update of Sec. 3.9 moves); other entries are
 *            left as they are, so one array cleared once collects the
 *            Gaussians of several views. */
int32_t tgs_render_bwd(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                       int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                       const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                       int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                       const float* out, const uint32_t* ncontrib, const float* dL_dout,
                       float* g2d, const float* state, uint8_t* touched, void* stream);

/* tgs_render_bwd (and, with stats, tgs_render_bwd_density) over two-part
 * lists as in tgs_render_fwd_cont: the adjoint of the forward those lists
 * gave.  err, n and stats as tgs_render_bwd_density; stats NULL: no
 * density sums. */
int32_t tgs_render_bwd2(const float* splat, const uint32_t* vals, const uint32_t* ranges, const uint32_t* vals2,
                        const uint32_t* ranges2, int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                        const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix, int32_t n_st,
                        int32_t max_per_tile, const tgs_raster_params* rp, const float* out,
                        const uint32_t* ncontrib, const float* dL_dout, float* g2d, const float* state,
                        uint8_t* touched, const float* err, int64_t n, float* stats, void* stream);

/* tgs_render_bwd with bitwise-reproducible gradients: the same adjoint and
 * the same per-Gaussian wave sums, but each wave stores its nine sums of
 * a pair into a per-(pair, wave) record of the workspace instead of adding
 * them to g2d with float atomics (whose order varies run to run); a second
 * pass adds, per Gaussian, the records of its pairs in a fixed order (the
 * tiles of its rectangle row by row, then the waves) and adds the total to
 * g2d.  Same inputs give the same bits on every run.  touched as in
 * tgs_render_bwd.
 *   depth, rect  the tgs_project outputs the lists were built from
 *   n            Gaussians; n_pairs the pair count tgs_bin_sort returned
 *   ws           tgs_render_bwd_det_workspace_size(n_pairs, max_per_tile,
 *                dense) bytes, 16-byte aligned (cleared by the call):
 *                36 bytes per pair and wave of a tile's workgroup (one wave
 *                up to 64 samples per tile, two up to 128, four above and
 *                in dense mode)
 * The density-control variant keeps its atomics (tgs_render_bwd_density). */
size_t tgs_render_bwd_det_workspace_size(int64_t n_pairs, int32_t max_per_tile, int32_t dense);
int32_t tgs_render_bwd_deterministic(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                     int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                     const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                                     int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                                     const float* out, const uint32_t* ncontrib, const float* dL_dout,
                                     float* g2d, const float* state, uint8_t* touched, const float* depth,
                                     const int32_t* rect, int64_t n, int64_t n_pairs, void* ws,
                                     size_t ws_bytes, void* stream);

/* Sparse supervision of one view (Sec. 3.7: Charbonnier L1 per pixel plus
 * tile NCC with the gradient-balanced weight of Eq. ncc_weight_auto, summed
 * as Eq. full_loss).  With lp->structure = TGS_STRUCTURE_SSIM the tile term
 * is 1 - SSIM instead, SSIM = (2 mu_x mu_y + C1)(2 C_xy + C2) /
 * ((mu_x^2 + mu_y^2 + C1)(V_x + V_y + C2)) per channel over the tile's
 * samples (1/n moments, C1 = 0.01^2, C2 = 0.03^2), with the same balance
 * weight built from its gradient; tile_loss then holds 1 - mean SSIM in
 * place of 1 - mean NCC.
 *   out        [P][4] rendered colours; gt [3][H][W] float target image
 *   totals     [2] int64 device: sampled pixels and sampled tiles of the step
 *   dL_dout    [P][4] written (channel 3 = 0); err [P] = |I_hat - I|_1
 *   lambda     [n_st] balance weights; tile_loss [n_st][2] = (L1 part, NCC
 *              part) of this tile's contribution to L */
int32_t tgs_loss(const float* out, const float* gt, int32_t height, int32_t width,
                 const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                 int32_t n_st, const int64_t* totals, const tgs_loss_params* lp,
                 float* dL_dout, float* err, float* lambda, float* tile_loss, void* stream);

/* Error-map EMA at sampled pixels (Eq. ema_err) and age update (Eq.
 * age_update) of one selected view.  E is half bits, blended in FP32 as
 * fl(fl(fl(1 - beta) E) + fl(beta e)) and rounded to nearest even; A is
 * reset to 0 at samples and incremented (saturating) elsewhere.  When the
 * width is a multiple of 8, A must be 16-byte aligned (it moves in 16-byte
 * accesses). */
int32_t tgs_ema_age_update(uint16_t* E, uint16_t* A, int32_t height, int32_t width,
                           const int32_t* tile_slot, const int32_t* tile_off,
                           const uint8_t* pix, const float* err, float beta, void* stream);

/* Dense error-map initialisation (Sec. 3.3: E_v from the dense L1 error of
 * the initial Gaussians): E = half(|dr| + |dg| + |db|) from a dense
 * tgs_render_fwd output. */
int32_t tgs_error_init(const float* out_dense, const float* gt, int32_t height, int32_t width,
                       uint16_t* E, void* stream);

/* Error-driven density control, back-projection (Sec. 3.8, Eq.
 * gauss_err_accum): replays the tgs_render_fwd walk of the same samples
 * (same alpha decisions, bounded by the forward's ncontrib) and adds, for
 * every composited Gaussian i at a rendered pixel p with weight
 * w = T alpha,
 *   stats[i][0] += e(p) w      (E_i)
 *   stats[i][1] += w           (W_i)
 *   stats[i][2] += D_i(p) w    (D_i), D_i(p) = sqrt(d^T Q d), the
 *                              Mahalanobis distance of p from the centre
 *                              under the conic Q.
 * Arguments up to rp are those of the tgs_render_fwd call that produced
 * ncontrib.
 *   ncontrib  [P] uint32 from that call (sparse: P samples; dense: H*W)
 *   err       [P] float per-pixel error e(p), indexed like ncontrib (the
 *             tgs_loss err output in sparse mode)
 *   state     nullable: that call's state record; given, each tile's walk
 *             runs as TGS_RENDER_CHUNKS workgroups as in tgs_render_bwd
 *             (same per-pixel arithmetic, another order of the atomics)
 *   n         number of Gaussians (ids in vals must be below n)
 *   stats     [n][4] float, 16-byte aligned, accumulated (+=); entry 3 of
 *             each slot is not touched (the three sums of a Gaussian share
 *             a cache line).  The caller clears it, then calls once per
 *             view and step over which the sums run.
 * Float atomics: the summation order is unspecified. */
int32_t tgs_density_accumulate(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                               int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                               const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                               int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                               const uint32_t* ncontrib, const float* err, const float* state, int64_t n,
                               float* stats, void* stream);

/* tgs_density_accumulate over two-part lists (see tgs_render_fwd_cont). */
int32_t tgs_density_accumulate2(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                const uint32_t* vals2, const uint32_t* ranges2, int32_t tiles_x, int32_t tiles_y,
                                int32_t width, int32_t height, const int32_t* valid_tiles, const int32_t* tile_off,
                                const uint8_t* pix, int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                                const uint32_t* ncontrib, const float* err, const float* state, int64_t n,
                                float* stats, void* stream);

/* tgs_render_bwd that also adds the density-control sums of
 * tgs_density_accumulate (Sec. 3.8) for the same samples: the backward's
 * replay already forms each composited Gaussian's weight w = T alpha, and
 * the three sums join the gradient's wave reduction.  It also adds, in
 * stats[i][3], the absolute-gradient statistic of densification (the
 * threshold tau_grad^abs of the hyper-parameter table): the sum over the
 * rendered pixels of the norm of each pixel's own centre gradient in NDC
 * units, |(W/2 dL_p/dx, H/2 dL_p/dy)|.  g2d and touched get what
 * tgs_render_bwd gives (same arithmetic; float atomics in another order);
 * err, n and stats are as in tgs_density_accumulate (n > 0). */
int32_t tgs_render_bwd_density(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                               int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                               const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                               int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                               const float* out, const uint32_t* ncontrib, const float* dL_dout,
                               float* g2d, const float* state, uint8_t* touched, const float* err, int64_t n,
                               float* stats, void* stream);

/* Difficulty score (Sec. 3.8, Eq. gauss_score) from tgs_density_accumulate's
 * sums, in FP32: e_i = E_i / (W_i + eps), d_i = D_i / (W_i + eps),
 * s_i = e_i + lambda_eff d_i with lambda_eff = lambda_base (1 - rho), rho in
 * [0, 1] the training progress.  A Gaussian never composited scores 0.
 *   stats  [n][4] float (16-byte aligned); e_out, d_out nullable [n]; s_out [n]
 * Errors: eps <= 0 or rho outside [0, 1]. */
int32_t tgs_density_score(const float* stats, int64_t n, float lambda_base, float rho, float eps,
                          float* e_out, float* d_out, float* s_out, void* stream);

/* Percentile threshold of the density control (Sec. 3.8: densification and
 * pruning by percentile thresholds of the scores): the k-th largest
 * (1 <= k <= n) of values[n] in the total order of the IEEE bit patterns
 * (-0 below +0, NaN above +inf), written to out (one device float) by an
 * exact MSB-first radix select that stays on the device (nine small
 * launches, no host synchronisation).
 *   ws  tgs_select_workspace_size() bytes, 16-byte aligned, device memory
 *       (fully rewritten by every call; calls that share it must not overlap)
 * Errors: n < 1, k outside [1, n], a short workspace. */
size_t tgs_select_workspace_size(void);
int32_t tgs_select_kth_largest(const float* values, int64_t n, int64_t k, float* out, void* ws,
                               size_t ws_bytes, void* stream);

/* mask[i] = 1 when values[i] >= *thr in the order above (thr is a device
 * pointer, e.g. the tgs_select_kth_largest output), else 0. */
int32_t tgs_threshold_mask(const float* values, int64_t n, const float* thr, uint8_t* mask, void* stream);

/* Densify and prune on the selections (Alg. 1 step 11, second line), in
 * two calls.  tgs_density_topology_count scans the masks (keep[n],
 * densify[n] uint8, nonzero = set) into ws and returns, after waiting for
 * the stream, n_keep = #keep and n_new = #(keep and densify).
 * tgs_density_topology_apply then writes the new arrays, n_out = n_keep +
 * n_new Gaussians, from the same ws (same n; the masks are not read again):
 *   - Gaussians with keep = 0 are dropped; the kept ones stay in order,
 *     then one new Gaussian per kept and densified one, in order;
 *   - a densified Gaussian whose largest log-scale (rows 3-5) exceeds
 *     log_split is split: o = R(q/|q|) diag(exp(s)) z[i] (z: [n][3] standard
 *     normal draws supplied by the caller), the kept slot at mean + o, the
 *     new one at mean - o, both with log-scales lowered by ln 1.6;
 *     otherwise the new Gaussian is a copy;
 *   - m and v are copied, except for split and new Gaussians (zeros).
 *   params [59][n], m, v [n][TGS_MOMENT_STRIDE] float, read
 *   params_out [59][n_out], m_out, v_out [n_out][TGS_MOMENT_STRIDE] float,
 *   written (moment records move whole, padding included; the four moment
 *   arrays 16-byte aligned)
 * Errors: n outside [1, 2^31), n_out outside [0, 2n], a short workspace. */
size_t tgs_density_topology_workspace_size(int64_t n);
int32_t tgs_density_topology_count(const uint8_t* keep, const uint8_t* densify, int64_t n, int64_t* n_keep,
                                   int64_t* n_new, void* ws, size_t ws_bytes, void* stream);
int32_t tgs_density_topology_apply(const float* params, const float* m, const float* v, int64_t n,
                                   const float* z, float log_split, const void* ws, size_t ws_bytes,
                                   float* params_out, float* m_out, float* v_out, int64_t n_out,
                                   void* stream);

/* Screen-space statistics of densification (Alg. 1 step 8, second line;
 * the gradient threshold tau_grad of the hyper-parameter table), per view
 * after its backward: for every Gaussian projected in the view
 * (radius > 0), acc[i][0] += |(W/2 g2d[i][0], H/2 g2d[i][1])| (the 2D centre
 * gradient in NDC units, the units the table's thresholds are stated in),
 * acc[i][1] += 1, acc[i][2] = max(acc[i][2], radius); acc[i][3] is not
 * touched.
 *   g2d [n][9] (tgs_render_bwd output), radius [n] (tgs_project output),
 *   width, height  the view's image size (W, H above),
 *   acc [n][4] float, 16-byte aligned; the caller clears it.
 * tgs_grad_screen_mean: out[i] = acc[i][0] / acc[i][1], 0 where never
 * projected. */
int32_t tgs_grad_screen_accumulate(const float* g2d, const int32_t* radius, int64_t n, int32_t width,
                                   int32_t height, float* acc, void* stream);

/* Both selections of one density step (Sec. 3.8: percentile thresholds of
 * the score; the gradient thresholds tau_grad and tau_grad^abs of the
 * hyper-parameter table gate densification), in one pass:
 *   keep[i]    = prune ? scores[i] >= thr[1] : 1
 *   densify[i] = keep[i] and scores[i] >= thr[0] and
 *                (gmean_i >= tau_grad or amean_i >= tau_grad_abs)
 * with gmean_i = gstats[i][0] / gstats[i][1] (tgs_grad_screen_accumulate
 * sums) and amean_i = dstats[i][3] / gstats[i][1] (the absolute statistic of
 * tgs_render_bwd_density), both FP32; a Gaussian never projected
 * (gstats[i][1] = 0) is not densified.  Scores compare in the total order of
 * tgs_threshold_mask.
 *   scores  [n]; thr  device [2] (densify threshold, keep threshold, e.g.
 *           from tgs_select_kth_largest)
 *   gstats, dstats  [n][4], 16-byte aligned; dstats nullable (then only
 *           tau_grad gates)
 *   prune   nonzero on a final-pruning step
 *   densify, keep  [n] uint8, written. */
int32_t tgs_density_masks(const float* scores, const float* gstats, const float* dstats, int64_t n,
                          const float* thr, float tau_grad, float tau_grad_abs, int32_t prune,
                          uint8_t* densify, uint8_t* keep, void* stream);
int32_t tgs_grad_screen_mean(const float* acc, int64_t n, float* out, void* stream);

/* Per-view error sums for the anchor view (Sec. 3.4, Eq. anchor_view):
 * sums[v] = the exact sum over the image of E_v(p) * 2^24 (every finite
 * non-negative half is then an integer; negative, infinite and NaN values
 * count 0, as in the sampler), so E_bar_v = sums[v] / (2^24 * pixels).
 *   E     [n_views][pixels] half bits, contiguous
 *   sums  [n_views] uint64, written (cleared first) */
int32_t tgs_view_error_sums(const uint16_t* E, int32_t n_views, int64_t pixels, uint64_t* sums, void* stream);

/* Chain rule from g2d to the Gaussian parameters (backward of tgs_project).
 *   accumulate  1: grad[59][n] += gradient; Gaussians whose gradient is
 *               zero (culled, radius 0, or all nine g2d entries zero) are
 *               left untouched.  0: grad = gradient, every entry written
 *               (zeros for them), so grad needs no clearing.
 *   clamp       the tgs_project output. */
int32_t tgs_project_bwd(const float* params, int64_t n, const tgs_camera* cam,
                        const tgs_raster_params* rp, const int32_t* radius,
                        const uint8_t* clamp, const float* g2d, float* grad, int32_t accumulate,
                        void* stream);

/* ---- FP64 instantiation, for gradient checks (torch.autograd.gradcheck of
 * the rasterizer as a function of the Gaussian parameters).  The same
 * definitions as the FP32 path (projection of Sec. 3.1 with SH colour,
 * Eq. alpha_comp with its thresholds, its exact adjoint, the chain rule),
 * evaluated in doubles; not tuned for speed.
 * tgs_project_f64: params[59][n] double; rec64[n][12] double written
 *   (centre x, y; conic a, b, c; opacity; r, g, b; depth; 0; 0); splat,
 *   depth, radius, rect, clamp written as by tgs_project (rounded to FP32),
 *   so tgs_bin_sort builds the lists from them.
 * tgs_render_fwd_f64 / tgs_render_bwd_f64: as tgs_render_fwd and
 *   tgs_render_bwd (same sample layout, NULL valid_tiles = dense) over
 *   rec64; out [P][4] double (colour, T), ncontrib [P]; the backward reads
 *   dL [P][4] double and adds to g2d[n][9] double (the caller clears it).
 * tgs_project_bwd_f64: as tgs_project_bwd over doubles. */
int32_t tgs_project_f64(const double* params, int64_t n, const tgs_camera* cam,
                        const tgs_raster_params* rp, double* rec64, float* splat, float* depth,
                        int32_t* radius, int32_t* rect, uint8_t* clamp, void* stream);
int32_t tgs_render_fwd_f64(const double* rec64, const uint32_t* vals, const uint32_t* ranges,
                           int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                           const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                           int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                           double* out, uint32_t* ncontrib, void* stream);
int32_t tgs_render_bwd_f64(const double* rec64, const uint32_t* vals, const uint32_t* ranges,
                           int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                           const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                           int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                           const double* out, const uint32_t* ncontrib, const double* dL,
                           double* g2d, void* stream);
int32_t tgs_project_bwd_f64(const double* params, int64_t n, const tgs_camera* cam,
                            const tgs_raster_params* rp, const int32_t* radius, const uint8_t* clamp,
                            const double* g2d, double* grad, int32_t accumulate, void* stream);

/* tgs_project_bwd followed by tgs_optimizer_step in one pass, for the last
 * view of a training step (Sec. 3.9 update applied to the gradient of
 * Sec. 3.6's backward): each parameter row's gradient stays in registers
 * and the row is updated at once.  Results equal the two calls bit for bit.
 *   grad_prev  nullable [59][n]: gradient accumulated from the step's
 *              earlier views (read only); NULL when this is the only view
 *   ws         workspace of tgs_project_bwd_optimizer_workspace_size(n)
 *              bytes (8-byte aligned)
 *   other arguments as in tgs_project_bwd and tgs_optimizer_step */
size_t tgs_project_bwd_optimizer_workspace_size(int64_t n);
int32_t tgs_project_bwd_optimizer_step(float* params, int64_t n, const tgs_camera* cam,
                                       const tgs_raster_params* rp, const int32_t* radius,
                                       const uint8_t* clamp, const float* g2d,
                                       const float* grad_prev, float* m, float* v,
                                       const uint8_t* touched, const tgs_optim_params* op,
                                       int64_t step, void* ws, size_t ws_bytes, void* stream);

/* The projection backward of every view of a training step fused with the
 * update (Sec. 3.9 update applied to the sum over the step's views of
 * Sec. 3.6's backward), in place of tgs_project_bwd for each view and
 * tgs_project_bwd_optimizer_step for the last: each Gaussian's chain rule
 * is evaluated for every view in registers and the rows are updated in the
 * same pass; no gradient array is written or read.  SH rows of degree >= 1
 * sum each view's float-rounded gradient in view order (as the per-view
 * path's gradient array does); rows 0-13 sum the views in FP64, the
 * covariance, opacity and colour gradients before the linear maps to the
 * scale, quaternion, opacity and DC rows, so they agree with the per-view
 * path to rounding, not bit for bit.
 *   n_views  1..16
 *   cams     [n_views] host array of the views' cameras
 *   radius, clamp, g2d  host arrays of n_views device pointers: each view's
 *            projection outputs and its backward's screen-space gradient
 *   ws       tgs_project_bwd_optimizer_views_workspace_size(n, n_views)
 *            bytes (8-byte aligned): per Gaussian the mean's gradient
 *            through the SH rows' view directions (3 doubles)
 *   other arguments as in tgs_project_bwd_optimizer_step */
size_t tgs_project_bwd_optimizer_views_workspace_size(int64_t n, int32_t n_views);
int32_t tgs_project_bwd_optimizer_step_views(float* params, int64_t n, int32_t n_views, const tgs_camera* cams,
                                             const tgs_raster_params* rp, const int32_t* const* radius,
                                             const uint8_t* const* clamp, const float* const* g2d, float* m,
                                             float* v, const uint8_t* touched, const tgs_optim_params* op,
                                             int64_t step, void* ws, size_t ws_bytes, void* stream);

/* Hybrid moment-damped LM / Adam update (Sec. 3.9, Eq. moment_damped_lm, and
 * the appendix optimizer details): per touched Gaussian, Adam moments for all
 * rows; geometry (rows 0-9) and base appearance (SH DC, opacity) solve
 * (J^T J + diag(sqrt(v) + eps)) Delta = -m and move by lr * Delta; with
 * J^T J = g g^T (lm_mode 0) the system is diagonal plus rank one and is
 * solved in closed form by the Sherman-Morrison identity, with
 * J^T J = diag(g^2) (lm_mode 1) elementwise (lm_mode 2: Adam for every
 * row); the other SH rows take a bias-corrected Adam step.  touched
 * nullable (all).  params, grad [59][n]; m, v [n][TGS_MOMENT_STRIDE].
 * step >= 1.  Internally FP64. */
int32_t tgs_optimizer_step(float* params, const float* grad, float* m, float* v, int64_t n,
                           const uint8_t* touched, const tgs_optim_params* op, int64_t step,
                           void* stream);

/* ---- Learned tile priority.  Not in the paper: a small network that
 * predicts the tile error the error-map sampler (Sec. 3.3) would measure,
 * from cheap per-(view, tile) features, trained online on the tile errors
 * the method measures; the error-map ranking stays the reference.
 * Parameter vector (float32, TGS_TILE_MLP_PARAMS): W1[32][64] at 0, b1 at
 * 2048, W2[64][64] at 2112, b2 at 6208, w3[64] at 6272, b3 at 6336;
 * y = x_19 + w3 . gelu(W2^T gelu(W1^T x + b1) + b2) + b3 (GELU in its erf
 * form; x_19, the tile's mean error when its map was written, makes the
 * network predict the change since then).
 * The two 64-wide layers run as bfloat16 MFMA products (x, W1, the first
 * activation and W2 rounded to nearest even) with float32 sums. */
#define TGS_TILE_MLP_FEATURES 32
#define TGS_TILE_MLP_PARAMS 6337

/* Features of every tile of one view, X [tiles_x * tiles_y][32] float
 * (16-byte aligned), row-major tile order: tile centre x / W, y / H; 16 pose
 * features of the camera centre c = -R^T t (c / |c|, |c| / 3, then sin and
 * cos of pi c_j / |c| and of 2 pi c_j / |c| for j = 0, 1, 2); log(1 + pairs
 * in ranges); the mean of E and log(1 + the mean of A) over the tile's
 * in-image pixels; zeros.  ranges: tgs_bin_sort output; E, A: [H][W] half
 * error and uint16 age maps. */
int32_t tgs_tile_features(const uint32_t* ranges, const uint16_t* E, const uint16_t* A,
                          int32_t height, int32_t width, const tgs_camera* cam, float* X,
                          void* stream);

/* Predictions y [n] for feature rows X [n][32] (16-byte aligned).  act:
 * nullable [n][128] float, 16-byte aligned: the pre-activations of the two
 * hidden layers, which tgs_tile_mlp_train_step needs. */
int32_t tgs_tile_mlp_fwd(const float* params, const float* X, int64_t n, float* y, float* act,
                         void* stream);

/* One online training step: the gradient of mean_i (y_i - target_i)^2 over
 * the n rows of the last tgs_tile_mlp_fwd (X, act, y), with each bfloat16
 * rounding taken as the identity, then a bias-corrected Adam step (0.9,
 * 0.999, 1e-8, learning rate lr) on params with moments m, v [6337] float.
 * grad: nullable [6337] float, receives the gradient.  ws: workspace of
 * tgs_tile_mlp_workspace_size(n) bytes.  step >= 1. */
size_t tgs_tile_mlp_workspace_size(int64_t n);
int32_t tgs_tile_mlp_train_step(float* params, float* m, float* v, const float* X,
                                const float* act, const float* y, const float* target, int64_t n,
                                int64_t step, float lr, float* grad, void* ws, size_t ws_bytes,
                                void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TURBOGS_H */
