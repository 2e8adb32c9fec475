// Front-to-back compositing of the sampled pixels (forward) and its adjoint.
//
// One workgroup per sampled tile; a lane owns one sampled pixel of the tile
// (sparse mode: the tile's explicit sample list from the prefix offsets;
// dense mode: all 256 pixels).  The tile's depth-sorted Gaussian range is
// walked in batches of one Gaussian per thread, staged into LDS as a
// tile-local centre, the conic, the opacity and the colour, so every lane
// evaluates the batch from LDS broadcasts.  The walk stops when every lane's
// transmittance has terminated (workgroup vote per batch, wave exit inside).
//
// The backward replays the same walk front to back, recomputing T and the
// accumulated colour from the forward outputs (final colour and the number
// of contributors), so nothing per Gaussian or per (pixel, Gaussian) is
// stored.  Per Gaussian, each lane's contribution to the nine screen-space
// gradients is summed across the wave with DPP, and nine lanes of the wave
// issue one float atomic each.
#include "common.h"

namespace tgs {

struct RasterArgs {
  const float4* splat;
  const uint32_t* vals;
  const uint2* ranges;
  const int32_t* valid_tiles;
  const int32_t* tile_off;
  const uint8_t* pix;
  int tiles_x, tiles_y, width, height;
  float alpha_min, alpha_max, T_min;
  float bg0, bg1, bg2;
};

// The alpha decisions must come out bit-identical in the forward and the
// replay, so they are written with explicit fused operations and no
// contraction left to the compiler.
__device__ __forceinline__ float splat_power(float dx, float dy, float ca, float cb, float cc) {
#pragma clang fp contract(off)
  const float xx = dx * dx, yy = dy * dy, xy = dx * dy;
  const float q = __builtin_fmaf(ca, xx, cc * yy);
  return __builtin_fmaf(-0.5f, q, -(cb * xy));
}

__device__ __forceinline__ float one_minus_times(float T, float alpha) {
#pragma clang fp contract(off)
  return T * (1.0f - alpha);
}

struct PixelSlot {
  int loc;      // local index in the tile, -1 if none
  bool inside;  // pixel exists and lies in the image
  int64_t out;  // output index
};

template <int kBlock, bool kDense>
__device__ __forceinline__ PixelSlot pixel_of(const RasterArgs& a, int slot, int tile, int tid) {
  PixelSlot p;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  if (kDense) {
    p.loc = tid;
    const int x = tx * kTile + (tid & 15), y = ty * kTile + (tid >> 4);
    p.inside = x < a.width && y < a.height;
    p.out = (int64_t)y * a.width + x;
  } else {
    const int p0 = a.tile_off[slot], np = a.tile_off[slot + 1] - p0;
    p.loc = tid < np ? (int)a.pix[p0 + tid] : -1;
    p.inside = p.loc >= 0;
    p.out = p0 + tid;
  }
  return p;
}

template <int kBlock, bool kDense>
__global__ void __launch_bounds__(kBlock) render_fwd_kernel(RasterArgs a, float4* __restrict__ out,
                                                            uint32_t* __restrict__ ncontrib,
                                                            unsigned long long* __restrict__ counters) {
  __shared__ float4 s_geo[kBlock];  // tile-local centre x, y; conic a, b
  __shared__ float4 s_app[kBlock];  // conic c, opacity, r, g
  __shared__ float s_blue[kBlock];
  const int slot = blockIdx.x, tid = threadIdx.x;
  const int tile = kDense ? slot : a.valid_tiles[slot];
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const PixelSlot px = pixel_of<kBlock, kDense>(a, slot, tile, tid);
  const float lx = (float)(px.loc & 15), ly = (float)(px.loc >> 4);
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const uint2 range = a.ranges[tile];

  float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  uint32_t last = 0, n_eval = 0, n_blend = 0;
  bool done = !px.inside;
  for (uint32_t start = range.x; start < range.y; start += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const uint32_t idx = start + tid;
    if (idx < range.y) {
      const uint32_t g = a.vals[idx];
      const float4 p0 = a.splat[3 * g], p1 = a.splat[3 * g + 1], p2 = a.splat[3 * g + 2];
      s_geo[tid] = make_float4((p0.x - x0) + p0.z, (p0.y - y0) + p0.w, p1.x, p1.y);
      s_app[tid] = make_float4(p1.z, p1.w, p2.x, p2.y);
      s_blue[tid] = p2.z;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBlock, range.y - start);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 ge = s_geo[j];
        const float4 ap = s_app[j];
        const float power = splat_power(lx - ge.x, ly - ge.y, ge.z, ge.w, ap.x);
        ++n_eval;
        if (power > 0.f) continue;
        const float alpha = fminf(a.alpha_max, ap.y * __expf(power));
        if (alpha < a.alpha_min) continue;
        const float t_next = one_minus_times(T, alpha);
        if (t_next < a.T_min) {
          done = true;
          break;
        }
        const float w = alpha * T;
        c0 += w * ap.z;
        c1 += w * ap.w;
        c2 += w * s_blue[j];
        T = t_next;
        last = start - range.x + (uint32_t)j + 1u;
        ++n_blend;
      }
    }
  }
  if (px.inside) {
    out[px.out] = make_float4(c0 + T * a.bg0, c1 + T * a.bg1, c2 + T * a.bg2, T);
    ncontrib[px.out] = last;
  }
  if (counters != nullptr) {
    const int se = wave_sum_i((int)n_eval), sb = wave_sum_i((int)n_blend);
    if (lane_id() == 0) {
      atomicAdd(&counters[0], (unsigned long long)se);
      atomicAdd(&counters[1], (unsigned long long)sb);
    }
  }
}

template <int kBlock, bool kDense>
__global__ void __launch_bounds__(kBlock) render_bwd_kernel(RasterArgs a,
                                                            const float4* __restrict__ out,
                                                            const uint32_t* __restrict__ ncontrib,
                                                            const float4* __restrict__ dL,
                                                            float* __restrict__ g2d) {
  __shared__ float4 s_geo[kBlock];
  __shared__ float4 s_app[kBlock];
  __shared__ float s_blue[kBlock];
  __shared__ uint32_t s_gid[kBlock];
  const int slot = blockIdx.x, tid = threadIdx.x;
  const int tile = kDense ? slot : a.valid_tiles[slot];
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const PixelSlot px = pixel_of<kBlock, kDense>(a, slot, tile, tid);
  const float lx = (float)(px.loc & 15), ly = (float)(px.loc >> 4);
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const uint2 range = a.ranges[tile];

  float Cout0 = 0.f, Cout1 = 0.f, Cout2 = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  uint32_t last = 0;
  if (px.inside) {
    const float4 o = out[px.out];
    const float4 d = dL[px.out];
    Cout0 = o.x; Cout1 = o.y; Cout2 = o.z;
    g0 = d.x; g1 = d.y; g2 = d.z;
    last = ncontrib[px.out];
  }
  bool done = last == 0;
  float T = 1.f, acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  const int lane = lane_id();
  for (uint32_t start = range.x; start < range.y; start += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const uint32_t idx = start + tid;
    if (idx < range.y) {
      const uint32_t g = a.vals[idx];
      const float4 p0 = a.splat[3 * g], p1 = a.splat[3 * g + 1], p2 = a.splat[3 * g + 2];
      s_geo[tid] = make_float4((p0.x - x0) + p0.z, (p0.y - y0) + p0.w, p1.x, p1.y);
      s_app[tid] = make_float4(p1.z, p1.w, p2.x, p2.y);
      s_blue[tid] = p2.z;
      s_gid[tid] = g;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBlock, range.y - start);
    for (int j = 0; j < cnt; ++j) {
      if (__ballot(!done) == 0ull) break;  // the whole wave has finished
      const uint32_t pos = start - range.x + (uint32_t)j;
      const float4 ge = s_geo[j];
      const float4 ap = s_app[j];
      float v[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      bool contrib = false;
      if (!done) {
        const float dx = lx - ge.x, dy = ly - ge.y;
        const float power = splat_power(dx, dy, ge.z, ge.w, ap.x);
        if (power <= 0.f) {
          const float G = __expf(power);
          const float araw = ap.y * G;
          const float alpha = fminf(a.alpha_max, araw);
          if (alpha >= a.alpha_min) {
            contrib = true;
            const float blue = s_blue[j];
            const float w = alpha * T;
            acc0 += w * ap.z;
            acc1 += w * ap.w;
            acc2 += w * blue;
            const float inv = 1.f / (1.f - alpha);
            const float dalpha = g0 * (T * ap.z - (Cout0 - acc0) * inv) +
                                 g1 * (T * ap.w - (Cout1 - acc1) * inv) +
                                 g2 * (T * blue - (Cout2 - acc2) * inv);
            v[6] = w * g0;
            v[7] = w * g1;
            v[8] = w * g2;
            if (araw < a.alpha_max) {
              v[5] = G * dalpha;
              const float dpow = ap.y * G * dalpha;
              v[0] = (ge.z * dx + ge.w * dy) * dpow;
              v[1] = (ge.w * dx + ap.x * dy) * dpow;
              v[2] = -0.5f * dx * dx * dpow;
              v[3] = -dx * dy * dpow;
              v[4] = -0.5f * dy * dy * dpow;
            }
            T = one_minus_times(T, alpha);
          }
        }
        if (pos + 1u >= last) done = true;
      }
      if (__ballot(contrib) != 0ull) {
        float mine = 0.f;
#pragma unroll
        for (int f = 0; f < 9; ++f) {
          const float s = wave_sum(v[f]);
          if (lane == f) mine = s;
        }
        if (lane < 9 && mine != 0.f) unsafeAtomicAdd(&g2d[(int64_t)s_gid[j] * 9 + lane], mine);
      }
    }
  }
}

template <int kBlock, bool kDense>
static void launch_fwd(const RasterArgs& a, int grid, float* out, uint32_t* ncontrib,
                       uint64_t* counters, hipStream_t s) {
  hipLaunchKernelGGL((render_fwd_kernel<kBlock, kDense>), dim3(grid), dim3(kBlock), 0, s, a,
                     (float4*)out, ncontrib, (unsigned long long*)counters);
}

template <int kBlock, bool kDense>
static void launch_bwd(const RasterArgs& a, int grid, const float* out, const uint32_t* ncontrib,
                       const float* dL, float* g2d, hipStream_t s) {
  hipLaunchKernelGGL((render_bwd_kernel<kBlock, kDense>), dim3(grid), dim3(kBlock), 0, s, a,
                     (const float4*)out, ncontrib, (const float4*)dL, g2d);
}

static int32_t make_args(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                         int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                         const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                         int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                         const char* who, RasterArgs& a) {
  TGS_REQUIRE(rp != nullptr, "%s: null raster params", who);
  TGS_REQUIRE(width > 0 && height > 0 && tiles_x == (int32_t)ceil_div(width, kTile) &&
                  tiles_y == (int32_t)ceil_div(height, kTile),
              "%s: tile grid %d x %d does not match image %d x %d", who, tiles_x, tiles_y, width,
              height);
  TGS_REQUIRE(splat && vals && ranges, "%s: null splat/vals/ranges", who);
  TGS_REQUIRE(((uintptr_t)splat & 15) == 0, "%s: splat must be 16-byte aligned", who);
  if (valid_tiles != nullptr) {
    TGS_REQUIRE(tile_off && pix, "%s: null tile_off/pix", who);
    TGS_REQUIRE(n_st >= 0 && (int64_t)n_st <= (int64_t)tiles_x * tiles_y, "%s: bad n_st %d", who, n_st);
    TGS_REQUIRE(max_per_tile >= 0 && max_per_tile <= kTilePixels, "%s: bad max_per_tile %d", who,
                max_per_tile);
  }
  a.splat = (const float4*)splat;
  a.vals = vals;
  a.ranges = (const uint2*)ranges;
  a.valid_tiles = valid_tiles;
  a.tile_off = tile_off;
  a.pix = pix;
  a.tiles_x = tiles_x;
  a.tiles_y = tiles_y;
  a.width = width;
  a.height = height;
  a.alpha_min = rp->alpha_min;
  a.alpha_max = rp->alpha_max;
  a.T_min = rp->T_min;
  a.bg0 = rp->bg[0];
  a.bg1 = rp->bg[1];
  a.bg2 = rp->bg[2];
  return TGS_OK;
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_render_fwd(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                  int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                  const int32_t* valid_tiles, const int32_t* tile_off,
                                  const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                  const tgs_raster_params* rp, float* out, uint32_t* ncontrib,
                                  uint64_t* counters, void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_render_fwd", a))
    return e;
  TGS_REQUIRE(out && ncontrib, "tgs_render_fwd: null output");
  TGS_REQUIRE(((uintptr_t)out & 15) == 0, "tgs_render_fwd: out must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  if (valid_tiles == nullptr) {
    launch_fwd<256, true>(a, tiles_x * tiles_y, out, ncontrib, counters, s);
  } else if (n_st > 0) {
    if (max_per_tile <= 64) launch_fwd<64, false>(a, n_st, out, ncontrib, counters, s);
    else if (max_per_tile <= 128) launch_fwd<128, false>(a, n_st, out, ncontrib, counters, s);
    else launch_fwd<256, false>(a, n_st, out, ncontrib, counters, s);
  }
  return hip_status("tgs_render_fwd");
}

extern "C" int32_t tgs_render_bwd(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                  int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                  const int32_t* valid_tiles, const int32_t* tile_off,
                                  const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                  const tgs_raster_params* rp, const float* out,
                                  const uint32_t* ncontrib, const float* dL_dout, float* g2d,
                                  void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_render_bwd", a))
    return e;
  TGS_REQUIRE(out && ncontrib && dL_dout && g2d, "tgs_render_bwd: null pointer");
  TGS_REQUIRE(((uintptr_t)out & 15) == 0 && ((uintptr_t)dL_dout & 15) == 0,
              "tgs_render_bwd: out and dL_dout must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  if (valid_tiles == nullptr) {
    launch_bwd<256, true>(a, tiles_x * tiles_y, out, ncontrib, dL_dout, g2d, s);
  } else if (n_st > 0) {
    if (max_per_tile <= 64) launch_bwd<64, false>(a, n_st, out, ncontrib, dL_dout, g2d, s);
    else if (max_per_tile <= 128) launch_bwd<128, false>(a, n_st, out, ncontrib, dL_dout, g2d, s);
    else launch_bwd<256, false>(a, n_st, out, ncontrib, dL_dout, g2d, s);
  }
  return hip_status("tgs_render_bwd");
}
