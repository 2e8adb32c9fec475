// FP64 instantiation of the compositing and its adjoint, for gradient
// checks: the same definitions as the FP32 kernels (Eq. alpha_comp with the
// alpha_min / alpha_max / T_min rules, the same per-tile depth-sorted
// lists), evaluated in doubles with one thread per pixel walking its tile's
// list.  Speed is not the point of this path: it has no LDS staging and
// sums the screen-space gradients with double atomics.
//
// Splat record rec64[n][12] (tgs_project_f64): centre x, y; conic a, b, c
// (power = -(a dx^2 + c dy^2) / 2 - b dx dy, d = pixel - centre); opacity;
// r, g, b; depth; two zeros.
#include "common.h"

namespace tgs {

struct Raster64 {
  const double* rec;
  const uint32_t* vals;
  const uint2* ranges;
  const int32_t* valid_tiles;
  const int32_t* tile_off;
  const uint8_t* pix;
  int tiles_x, width, height;
  double amin, amax, tmin, bg[3];
};

// Pixel of thread tid of workgroup slot: image coordinates, the tile and
// the output index; false when the slot has no such pixel.
__device__ __forceinline__ bool pixel64(const Raster64& a, int slot, int tid, int& x, int& y, int& tile,
                                        int64_t& o) {
  if (a.valid_tiles == nullptr) {
    tile = slot;
    x = (tile % a.tiles_x) * kTile + (tid & 15);
    y = (tile / a.tiles_x) * kTile + (tid >> 4);
    o = (int64_t)y * a.width + x;
    return x < a.width && y < a.height;
  }
  tile = a.valid_tiles[slot];
  const int p0 = a.tile_off[slot];
  if (tid >= a.tile_off[slot + 1] - p0) return false;
  const int loc = a.pix[p0 + tid];
  x = (tile % a.tiles_x) * kTile + (loc & 15);
  y = (tile / a.tiles_x) * kTile + (loc >> 4);
  o = p0 + tid;
  return true;
}

struct Eval64 {
  double dx, dy, power, G, alpha, a, b, c, o;
  bool ok, unclamped;
};

__device__ __forceinline__ Eval64 eval64(const double* r, int x, int y, double amin, double amax) {
#pragma clang fp contract(off)
  Eval64 e;
  e.dx = (double)x - r[0];
  e.dy = (double)y - r[1];
  e.a = r[2];
  e.b = r[3];
  e.c = r[4];
  e.o = r[5];
  e.power = -0.5 * (e.a * e.dx * e.dx + e.c * e.dy * e.dy) - e.b * e.dx * e.dy;
  e.G = exp(e.power);
  const double araw = e.o * e.G;
  e.alpha = fmin(amax, araw);
  e.unclamped = araw < amax;
  e.ok = e.power <= 0.0 && e.alpha >= amin;
  return e;
}

__global__ void __launch_bounds__(256) render_fwd64_kernel(Raster64 a, double* __restrict__ out,
                                                           uint32_t* __restrict__ ncontrib) {
#pragma clang fp contract(off)
  int x, y, tile;
  int64_t o;
  if (!pixel64(a, blockIdx.x, threadIdx.x, x, y, tile, o)) return;
  const uint2 rg = a.ranges[tile];
  double T = 1.0, C[3] = {0.0, 0.0, 0.0};
  uint32_t last = 0;
  for (uint32_t k = rg.x; k < rg.y; ++k) {
    const double* r = a.rec + 12 * (int64_t)a.vals[k];
    const Eval64 e = eval64(r, x, y, a.amin, a.amax);
    if (!e.ok) continue;
    const double tn = T * (1.0 - e.alpha);
    if (tn < a.tmin) break;
    const double w = T * e.alpha;
    for (int ch = 0; ch < 3; ++ch) C[ch] += w * r[6 + ch];
    T = tn;
    last = k - rg.x + 1;
  }
  for (int ch = 0; ch < 3; ++ch) out[4 * o + ch] = C[ch] + T * a.bg[ch];
  out[4 * o + 3] = T;
  ncontrib[o] = last;
}

// With B_k = C - sum_{j<=k} T_j alpha_j c_j (C the output, background
// included): dC/dc_k = T_k alpha_k, dC/dalpha_k = T_k c_k - B_k / (1 - alpha_k);
// alpha = o G is differentiated only below the clamp.
__global__ void __launch_bounds__(256) render_bwd64_kernel(Raster64 a, const double* __restrict__ out,
                                                           const uint32_t* __restrict__ ncontrib,
                                                           const double* __restrict__ dL,
                                                           double* __restrict__ g2d) {
#pragma clang fp contract(off)
  int x, y, tile;
  int64_t o;
  if (!pixel64(a, blockIdx.x, threadIdx.x, x, y, tile, o)) return;
  const uint2 rg = a.ranges[tile];
  const uint32_t end = rg.x + ncontrib[o];
  const double g[3] = {dL[4 * o], dL[4 * o + 1], dL[4 * o + 2]};
  const double Cf[3] = {out[4 * o], out[4 * o + 1], out[4 * o + 2]};
  double T = 1.0, acc[3] = {0.0, 0.0, 0.0};
  for (uint32_t k = rg.x; k < end; ++k) {
    const uint32_t gid = a.vals[k];
    const double* r = a.rec + 12 * (int64_t)gid;
    const Eval64 e = eval64(r, x, y, a.amin, a.amax);
    if (!e.ok) continue;
    const double w = T * e.alpha;
    double dLda = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      acc[ch] += w * r[6 + ch];
      dLda += g[ch] * (T * r[6 + ch] - (Cf[ch] - acc[ch]) / (1.0 - e.alpha));
    }
    const double dpow = e.unclamped ? e.o * e.G * dLda : 0.0;
    double* dst = g2d + 9 * (int64_t)gid;
    atomicAdd(dst + 0, (e.a * e.dx + e.b * e.dy) * dpow);
    atomicAdd(dst + 1, (e.b * e.dx + e.c * e.dy) * dpow);
    atomicAdd(dst + 2, -0.5 * e.dx * e.dx * dpow);
    atomicAdd(dst + 3, -e.dx * e.dy * dpow);
    atomicAdd(dst + 4, -0.5 * e.dy * e.dy * dpow);
    atomicAdd(dst + 5, e.unclamped ? e.G * dLda : 0.0);
    for (int ch = 0; ch < 3; ++ch) atomicAdd(dst + 6 + ch, w * g[ch]);
    T *= 1.0 - e.alpha;
  }
}

static int32_t make_raster64(Raster64& a, const double* rec, const uint32_t* vals, const uint32_t* ranges,
                             int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                             const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix, int32_t n_st,
                             int32_t max_per_tile, const tgs_raster_params* rp, const char* who) {
  TGS_REQUIRE(rp != nullptr, "%s: null raster params", who);
  TGS_REQUIRE(width > 0 && height > 0 && tiles_x == (int32_t)ceil_div(width, kTile) &&
                  tiles_y == (int32_t)ceil_div(height, kTile),
              "%s: tile grid does not match the image", who);
  TGS_REQUIRE(rec && vals && ranges, "%s: null pointer", who);
  TGS_REQUIRE(valid_tiles == nullptr || (tile_off && pix && n_st >= 0 && max_per_tile >= 1 &&
                                         max_per_tile <= kTilePixels),
              "%s: bad sample set", who);
  a.rec = rec;
  a.vals = vals;
  a.ranges = (const uint2*)ranges;
  a.valid_tiles = valid_tiles;
  a.tile_off = tile_off;
  a.pix = pix;
  a.tiles_x = tiles_x;
  a.width = width;
  a.height = height;
  a.amin = rp->alpha_min;
  a.amax = rp->alpha_max;
  a.tmin = rp->T_min;
  for (int c = 0; c < 3; ++c) a.bg[c] = rp->bg[c];
  return TGS_OK;
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_render_fwd_f64(const double* rec64, const uint32_t* vals, const uint32_t* ranges,
                                      int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                      const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                                      int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                                      double* out, uint32_t* ncontrib, void* stream) {
  Raster64 a;
  if (int32_t e = make_raster64(a, rec64, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off,
                                pix, n_st, max_per_tile, rp, "tgs_render_fwd_f64"))
    return e;
  TGS_REQUIRE(out && ncontrib, "tgs_render_fwd_f64: null output");
  const int blocks = valid_tiles == nullptr ? tiles_x * tiles_y : n_st;
  if (blocks > 0)
    hipLaunchKernelGGL(render_fwd64_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), a, out,
                       ncontrib);
  return hip_status("tgs_render_fwd_f64");
}

extern "C" int32_t tgs_render_bwd_f64(const double* rec64, const uint32_t* vals, const uint32_t* ranges,
                                      int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                      const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                                      int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                                      const double* out, const uint32_t* ncontrib, const double* dL,
                                      double* g2d, void* stream) {
  Raster64 a;
  if (int32_t e = make_raster64(a, rec64, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off,
                                pix, n_st, max_per_tile, rp, "tgs_render_bwd_f64"))
    return e;
  TGS_REQUIRE(out && ncontrib && dL && g2d, "tgs_render_bwd_f64: null pointer");
  const int blocks = valid_tiles == nullptr ? tiles_x * tiles_y : n_st;
  if (blocks > 0)
    hipLaunchKernelGGL(render_bwd64_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), a, out,
                       ncontrib, dL, g2d);
  return hip_status("tgs_render_bwd_f64");
}
