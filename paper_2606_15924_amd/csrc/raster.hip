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
// stored.  Optionally the forward records each pixel's (T, accumulated
// colour) every TGS_RENDER_CHUNK_LEN list positions; the backward then runs
// one workgroup per (tile, chunk of TGS_RENDER_CHUNK_LEN positions, the last
// of TGS_RENDER_CHUNKS chunks taking the rest) that starts from the
// recorded state.  The replay performs the same operations in the same
// order, so every per-lane value equals the unchunked one; at 64 samples
// per tile this turns one wave per tile into several, which the SIMDs need
// to hide latency.  Per Gaussian, each lane's contribution to the nine screen-space
// gradients is summed across the wave (lane-half swaps, then DPP within rows
// of 16), and nine lanes of the wave issue one float atomic each.
//
// Both walks keep the next batch's loads in flight while the current batch
// is evaluated: at 64 samples per tile a tile is one wave, so there are few
// waves per SIMD to hide memory latency otherwise.
#include <algorithm>

#include "common.h"

namespace tgs {

struct RasterArgs {
  const float4* splat;
  const uint32_t* vals;
  const uint2* ranges;
  // optional second segment of every tile's list (depth-prefix lists and
  // their continuation): the tile's list is vals[ranges[t]] followed by
  // vals2[ranges2[t]]
  const uint32_t* vals2;
  const uint2* ranges2;
  const int32_t* valid_tiles;
  const int32_t* tile_off;
  const uint8_t* pix;
  int tiles_x, tiles_y, width, height;
  float alpha_min, alpha_max, T_min;
  float bg0, bg1, bg2;
  // forward only: 0 plain; 1 depth-prefix pass (marks the tiles with a
  // pixel that ran off its list without the T_min stop, counts the other
  // pixels); 2 continuation pass over the slots cont_list[0 .. *cont_count)
  // (counts only the pixels the prefix pass left open)
  int mode;
  int32_t* cont_slot;     // [n_tiles] -1, or the slot of a marked tile (mode 1)
  uint32_t* cont_list;    // marked slots (written in mode 1, read in mode 2)
  uint32_t* cont_count;   // their number
};

// One tile's list: n1 entries from vals at b1, then len - n1 from vals2 at
// b2.  Positions are list-relative (0 .. len).
struct TileList {
  uint32_t b1, n1, b2, len;
};

__device__ __forceinline__ TileList tile_list(const RasterArgs& a, int tile) {
  const uint2 r = a.ranges[tile];
  TileList L{r.x, r.y - r.x, 0u, r.y - r.x};
  if (a.ranges2 != nullptr) {
    const uint2 q = a.ranges2[tile];
    L.b2 = q.x;
    L.len += q.y - q.x;
  }
  return L;
}

__device__ __forceinline__ uint32_t list_id(const RasterArgs& a, const TileList& L, uint32_t pos) {
  return pos < L.n1 ? a.vals[L.b1 + pos] : a.vals2[L.b2 + (pos - L.n1)];
}

// The alpha decisions must come out bit-identical in the forward and the
// replay, so both evaluate alpha through these functions, written with
// explicit fused operations and no contraction left to the compiler.
//
// The splat record holds the conic Q = [[a, b], [b, c]] in its LDL^T form
// (a, beta = b/a, delta = det Q / a), so that
// d^T Q d = a (dx + beta dy)^2 + delta dy^2: a sum of two non-negative
// terms.  (Summing a dx^2 + 2 b dx dy + c dy^2 cancels far along a thin
// splat, where the terms are many thousand times the result; the FP32
// alpha there would carry percent-level errors.)  Staged: A = -a/2 log2(e),
// beta, D = -delta/2 log2(e), so p2 = A w^2 + D dy^2 with w = dx + beta dy is
// log2(e) * power and G = exp(power) = 2^p2.
constexpr float kLog2e = 1.4426950408889634f;
constexpr int kUnroll = 8;   // forward: alphas evaluated per group
constexpr int kUnrollB = 2;  // backward

__device__ __forceinline__ float splat_exponent(float dx, float dy, float A, float beta, float D) {
#pragma clang fp contract(off)
  const float w = __builtin_fmaf(beta, dy, dx);
  const float ww = w * w, yy = dy * dy;
  return __builtin_fmaf(A, ww, D * yy);
}

// The same exponent (same operations, bit-identical), also returning the
// products dx^2, dx dy, dy^2 for the conic gradient.
__device__ __forceinline__ float splat_exponent_p(float dx, float dy, float A, float beta, float D, float& xx,
                                                  float& xy, float& yy) {
#pragma clang fp contract(off)
  xx = dx * dx;
  yy = dy * dy;
  xy = dx * dy;
  const float w = __builtin_fmaf(beta, dy, dx);
  const float ww = w * w;
  return __builtin_fmaf(A, ww, D * yy);
}

// alpha = min(alpha_max, o G); ok = exponent <= 0 and alpha >= alpha_min.
__device__ __forceinline__ float splat_alpha(float p2, float opacity, float amax, float& G) {
  G = __builtin_amdgcn_exp2f(p2);
  return __builtin_amdgcn_fmed3f(opacity * G, 0.f, amax);  // o G >= 0
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

// Staging of one batch: every thread holds one Gaussian of the batch in
// registers; the next batch's loads are issued before the current batch is
// evaluated, so their latency overlaps the compute.
struct Staged {
  float4 geo;  // tile-local centre x, y; staged A, beta
  float4 app;  // staged D, opacity, r, g
  float4 con;  // conic a, b, c in natural units, blue (backward only)
  float blue;
  uint32_t gid;
};

__device__ __forceinline__ Staged stage_load(const RasterArgs& a, uint32_t gid, float x0, float y0) {
#pragma clang fp contract(off)
  const float4 p0 = a.splat[3 * gid], p1 = a.splat[3 * gid + 1], p2 = a.splat[3 * gid + 2];
  Staged st;
  // exact integer difference first, then the fraction: the tile-local centre
  // keeps full FP32 precision relative to the pixel offsets
  st.geo = make_float4((p0.x - x0) + p0.z, (p0.y - y0) + p0.w, p1.x * (-0.5f * kLog2e), p1.y);
  st.app = make_float4(p1.z * (-0.5f * kLog2e), p1.w, p2.x, p2.y);
  const float b = p1.y * p1.x;  // b = beta a, c = delta + beta b
  st.con = make_float4(p1.x, b, __builtin_fmaf(p1.y, b, p1.z), p2.z);
  st.blue = p2.z;
  st.gid = gid;
  return st;
}

template <int kBlock, bool kDense>
__global__ void __launch_bounds__(kBlock) render_fwd_kernel(RasterArgs a, float4* __restrict__ out,
                                                            uint32_t* __restrict__ ncontrib,
                                                            unsigned long long* __restrict__ counters,
                                                            float4* __restrict__ state) {
  __shared__ float4 s_geo[kBlock];
  __shared__ float4 s_app[kBlock];
  __shared__ float s_blue[kBlock];
  if (a.mode == 2 && blockIdx.x >= *a.cont_count) return;  // workgroup-uniform
  const int slot = a.mode == 2 ? (int)a.cont_list[blockIdx.x] : (int)blockIdx.x, tid = threadIdx.x;
  const int tile = kDense ? slot : a.valid_tiles[slot];
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const PixelSlot px = pixel_of<kBlock, kDense>(a, slot, tile, tid);
  const float lx = (float)(px.loc & 15), ly = (float)(px.loc >> 4);
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const TileList L = tile_list(a, tile);
  const uint2 range = make_uint2(0u, L.len);
  const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.T_min;

  float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  uint32_t last = 0;
  uint32_t n_eval = 0, n_blend = 0;  // this lane's evaluations and blends (summed over the wave at the end)
  bool done = !px.inside, stopped = false;
  uint32_t stop_at = 0;  // list position of the T_min stop

  // prologue: records of batch 0 and ids of batch 1 in flight
  Staged nxt = {};
  uint32_t g_after = 0;
  if (range.x + tid < range.y) nxt = stage_load(a, list_id(a, L, range.x + tid), x0, y0);
  if (range.x + kBlock + tid < range.y) g_after = list_id(a, L, range.x + kBlock + tid);

  for (uint32_t start = range.x; start < range.y; start += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const bool live = start + tid < range.y;  // past the range: a zero-opacity record
    s_geo[tid] = live ? nxt.geo : make_float4(0.f, 0.f, 0.f, 0.f);
    s_app[tid] = live ? nxt.app : make_float4(0.f, 0.f, 0.f, 0.f);
    s_blue[tid] = live ? nxt.blue : 0.f;
    __syncthreads();
    const uint32_t i1 = start + kBlock + tid, i2 = start + 2 * kBlock + tid;
    if (i1 < range.y) nxt = stage_load(a, g_after, x0, y0);
    if (i2 < range.y) g_after = list_id(a, L, i2);
    const int cnt = (int)min((uint32_t)kBlock, range.y - start);
    const uint32_t pos0 = start - range.x;
    // groups of kUnroll Gaussians: their alphas are independent and are
    // evaluated first, then composited in order (entries past cnt hold a
    // zero-opacity record and never composite)
    for (int j = 0; j < cnt; j += kUnroll) {
      if (__ballot(!done) == 0ull) break;  // the whole wave has terminated
      const uint32_t pos = pos0 + (uint32_t)j;  // uniform; chunk starts are multiples of kUnroll
      if (state != nullptr && pos % TGS_RENDER_CHUNK_LEN == 0 && pos > 0 &&
          pos < (uint32_t)(TGS_RENDER_CHUNKS * TGS_RENDER_CHUNK_LEN))
        state[((int64_t)slot * (TGS_RENDER_CHUNKS - 1) + pos / TGS_RENDER_CHUNK_LEN - 1) * kBlock + tid] =
            make_float4(T, c0, c1, c2);
      float al[kUnroll], pw[kUnroll], cr[kUnroll], cg[kUnroll], cb[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const float4 ge = s_geo[j + u];
        const float4 ap = s_app[j + u];
        pw[u] = splat_exponent(lx - ge.x, ly - ge.y, ge.z, ge.w, ap.x);
        float G;
        al[u] = splat_alpha(pw[u], ap.y, amax, G);
        cr[u] = ap.z;
        cg[u] = ap.w;
        cb[u] = s_blue[j + u];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const float t_next = one_minus_times(T, al[u]);
        bool ok = !done && pw[u] <= 0.f && al[u] >= amin;
        n_eval += (j + u < cnt && !done) ? 1u : 0u;
        const bool stop = ok && t_next < tmin;
        stop_at = stop ? pos0 + (uint32_t)(j + u) : stop_at;
        stopped = stopped || stop;
        done = done || stop;
        ok = ok && !stop;
        const float w = ok ? al[u] * T : 0.f;
        c0 = __builtin_fmaf(w, cr[u], c0);
        c1 = __builtin_fmaf(w, cg[u], c1);
        c2 = __builtin_fmaf(w, cb[u], c2);
        T = ok ? t_next : T;
        last = ok ? pos0 + (uint32_t)(j + u) + 1u : last;
        n_blend += ok ? 1u : 0u;
      }
    }
  }
  if (px.inside) {
    out[px.out] = make_float4(c0 + T * a.bg0, c1 + T * a.bg1, c2 + T * a.bg2, T);
    ncontrib[px.out] = last;
  }
  if (a.mode == 1) {
    // a pixel that ran off its list without stopping needs the continuation;
    // its counts come from the continuation pass
    const bool open = px.inside && !stopped;
    if (open) n_eval = n_blend = 0u;
    if (__ballot(open) != 0ull && lane_id() == 0 &&
        atomicCAS(&a.cont_slot[tile], -1, slot) == -1)  // the tile's first marking wave lists it
      a.cont_list[atomicAdd(a.cont_count, 1u)] = (uint32_t)slot;
  } else if (a.mode == 2 && stopped && stop_at < L.n1) {
    n_eval = n_blend = 0u;  // stopped within the prefix: counted by the prefix pass
  }
  if (counters != nullptr) {
    n_eval = (uint32_t)wave_sum_i((int)n_eval);
    n_blend = (uint32_t)wave_sum_i((int)n_blend);
  }
  if (counters != nullptr && lane_id() == 0) {  // wave totals
    const int cs = blockIdx.x & (TGS_COUNTER_SLOTS - 1);
    atomicAdd(&counters[cs], (unsigned long long)n_eval);
    atomicAdd(&counters[TGS_COUNTER_SLOTS + cs], (unsigned long long)n_blend);
  }
}

__device__ __forceinline__ float swap_sum32(float x, float y) {
  // after the swap x = [x_lo | y_lo], y = [x_hi | y_hi]: the sum folds both
  // values to 32 lanes, x in lanes 0-31 and y in lanes 32-63
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap_sum16(float x, float y) {
  // rows of 16 lanes: x = [x0 y0 x2 y2], y = [x1 y1 x3 y3] after the swap
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float row_sum16(float v) {
  v += dpp_f<kDppQuadPerm1032>(0.f, v);
  v += dpp_f<kDppQuadPerm2301>(0.f, v);
  v += dpp_f<kDppRowHalfMirror>(0.f, v);
  v += dpp_f<kDppRowMirror>(0.f, v);
  return v;  // every lane of a row holds the row's sum
}

// Which of the nine sums a lane holds after the reduction below, and
// whether it issues that sum's atomic: row r of register R_k (rows of 16
// lanes) holds one field, lanes 0 and 1 of every row issue r0's and r1's
// field, lane 2 of row 0 issues field 8.  With the density sums (thirteen
// fields) lane 2 of every row issues one of fields 8-11 and lane 3 of row 0
// field 12.  Fixed per lane, so computed once.
struct Sum9Lane {
  int field;   // 0..12, or -1 when the lane issues no atomic
  int which;   // 0: r0, 1: r1, 2: r2, 3: r3
};

__device__ __forceinline__ Sum9Lane sum9_lane(bool thirteen = false) {
  const int lane = lane_id(), k = lane & 15, row = lane >> 4;
  Sum9Lane s;
  s.which = k < 4 ? k : 0;
  const int f = k * 4 + ((row & 1) << 1) + (row >> 1);
  if (k < 2) s.field = f;
  else if (k == 2) s.field = (thirteen || row == 0) ? f : -1;
  else s.field = (thirteen && k == 3 && row == 0) ? f : -1;
  return s;
}

// Sums each of v[0..8] over the wave and adds the nine sums to dst[0..8]
// with one atomic instruction.  Halves of the wave are folded pairwise with
// the lane swaps (64 -> 32 -> 16 lanes per value), then each row of 16 is
// reduced with DPP; row r of register R_k then holds the sum of one field.
// dst is wave-uniform (a scalar address).
__device__ __forceinline__ void wave_sum9_atomic(const float (&v)[9], float* __restrict__ dst, const Sum9Lane& sl) {
  const float p01 = swap_sum32(v[0], v[1]);
  const float p23 = swap_sum32(v[2], v[3]);
  const float p45 = swap_sum32(v[4], v[5]);
  const float p67 = swap_sum32(v[6], v[7]);
  const float p8 = swap_sum32(v[8], 0.f);
  // rows of r0: fields 0, 2, 1, 3; rows of r1: 4, 6, 5, 7; row 0 of r2: 8
  const float r0 = row_sum16(swap_sum16(p01, p23));
  const float r1 = row_sum16(swap_sum16(p45, p67));
  const float r2 = row_sum16(swap_sum16(p8, 0.f));
  float val = sl.which == 0 ? r0 : (sl.which == 1 ? r1 : r2);
  // every lane takes its sum here, with the whole wave active, so the last
  // DPP step stays one fused add instead of a move out of the branch below
  asm volatile("" : "+v"(val));
  if (sl.field >= 0 && val != 0.f) unsafeAtomicAdd(&dst[sl.field], val);
}

// The same nine wave sums, stored (not added) to dst[0..8]: the
// deterministic backward's per-(pair, wave) partial record, which no other
// wave writes.  Zero sums are stored too (the record is not cleared).
__device__ __forceinline__ void wave_sum9_store(const float (&v)[9], float* __restrict__ dst, const Sum9Lane& sl) {
  const float p01 = swap_sum32(v[0], v[1]);
  const float p23 = swap_sum32(v[2], v[3]);
  const float p45 = swap_sum32(v[4], v[5]);
  const float p67 = swap_sum32(v[6], v[7]);
  const float p8 = swap_sum32(v[8], 0.f);
  const float r0 = row_sum16(swap_sum16(p01, p23));
  const float r1 = row_sum16(swap_sum16(p45, p67));
  const float r2 = row_sum16(swap_sum16(p8, 0.f));
  float val = sl.which == 0 ? r0 : (sl.which == 1 ? r1 : r2);
  asm volatile("" : "+v"(val));  // as in wave_sum9_atomic
  if (sl.field >= 0) dst[sl.field] = val;
}

// The nine gradient sums plus the four density-control sums (e w, w, D w
// and the per-pixel centre-gradient norm) of the same Gaussian: the same
// folding with fields 9-11 in the rows of r2 that the nine-value form leaves
// empty (row 2: field 9, row 1: 10, row 3: 11) and field 12 in row 0 of r3;
// they go to stats[gid][field - 9], one 16-byte slot.
__device__ __forceinline__ void wave_sum13_atomic(const float (&v)[13], float* __restrict__ dst,
                                                  float* __restrict__ stats, uint32_t gid, int64_t n,
                                                  const Sum9Lane& sl) {
  const float p01 = swap_sum32(v[0], v[1]);
  const float p23 = swap_sum32(v[2], v[3]);
  const float p45 = swap_sum32(v[4], v[5]);
  const float p67 = swap_sum32(v[6], v[7]);
  const float p89 = swap_sum32(v[8], v[9]);
  const float pab = swap_sum32(v[10], v[11]);
  const float pc = swap_sum32(v[12], 0.f);
  const float r0 = row_sum16(swap_sum16(p01, p23));
  const float r1 = row_sum16(swap_sum16(p45, p67));
  const float r2 = row_sum16(swap_sum16(p89, pab));
  const float r3 = row_sum16(swap_sum16(pc, 0.f));
  float val = sl.which == 0 ? r0 : (sl.which == 1 ? r1 : (sl.which == 2 ? r2 : r3));
  asm volatile("" : "+v"(val));  // as in wave_sum9_atomic
  if (sl.field >= 0 && val != 0.f) {
    if (sl.field < 9) unsafeAtomicAdd(&dst[sl.field], val);
    else if (gid < (uint32_t)n) unsafeAtomicAdd(&stats[(int64_t)gid * 4 + (sl.field - 9)], val);
  }
}

// Optional density-control sums in the backward (Sec. 3.8): the replay
// already has each composited Gaussian's weight w = T alpha and each lane's
// own centre gradient.
struct DensityArgs {
  const float* err;  // [P] per-pixel error e(p), indexed like out
  float* stats;      // [n][4] E, W, D, sum of per-pixel NDC centre-gradient norms (+=)
  int64_t n;
};

// kDet: the deterministic variant.  Instead of adding each wave's nine sums
// to g2d[gid] with atomics, it stores them to g2d[(pos * kWaves + wave) * 9]
// (g2d is then the partial buffer, pos the pair's index in the sorted list);
// det_reduce_kernel adds them up per Gaussian in a fixed order.
template <int kBlock, bool kDense, bool kDensity = false, bool kDet = false>
__global__ void __launch_bounds__(kBlock) render_bwd_kernel(RasterArgs a,
                                                            const float4* __restrict__ out,
                                                            const uint32_t* __restrict__ ncontrib,
                                                            const float4* __restrict__ dL,
                                                            float* __restrict__ g2d,
                                                            const float4* __restrict__ state,
                                                            uint8_t* __restrict__ touched,
                                                            DensityArgs dens = {}) {
  __shared__ float4 s_geo[kBlock];
  __shared__ float4 s_app[kBlock];
  __shared__ float4 s_con[kBlock];  // conic a, b, c (natural units), blue
  __shared__ uint32_t s_gid[kBlock];
  // the last chunk (the rest of the list, the longest walks) is dispatched
  // first, so its workgroups run beside the fixed-length chunks
  const int slot = blockIdx.x, chunk = (int)gridDim.y - 1 - (int)blockIdx.y, tid = threadIdx.x;
  const int tile = kDense ? slot : a.valid_tiles[slot];
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const TileList L = tile_list(a, tile);
  const uint2 range = make_uint2(0u, L.len);
  // list positions [begin, end) of this chunk (one chunk without a state record)
  const uint32_t begin = range.x + (uint32_t)(chunk * TGS_RENDER_CHUNK_LEN);
  if (begin >= range.y && chunk > 0) return;  // workgroup-uniform
  const uint32_t end =
      chunk + 1 == (int)gridDim.y ? range.y : min(range.y, begin + (uint32_t)TGS_RENDER_CHUNK_LEN);
  const PixelSlot px = pixel_of<kBlock, kDense>(a, slot, tile, tid);
  const float lx = (float)(px.loc & 15), ly = (float)(px.loc >> 4);
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const float amin = a.alpha_min, amax = a.alpha_max;
  const Sum9Lane sl = sum9_lane(kDensity);
  const float hw = 0.5f * (float)a.width, hh = 0.5f * (float)a.height;  // pixel -> NDC units

  float Cout0 = 0.f, Cout1 = 0.f, Cout2 = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  uint32_t last = 0;
  float e_pix = 0.f;
  if (px.inside) last = ncontrib[px.out];
  bool done = last <= begin - range.x;  // nothing composited from this chunk on
  // a chunk past every pixel's last composited position has nothing to do:
  // it leaves before reading the pixels' outputs, gradients and state
  if (__syncthreads_count(done) == kBlock) return;
  if (px.inside) {
    const float4 o = out[px.out];
    const float4 d = dL[px.out];
    Cout0 = o.x; Cout1 = o.y; Cout2 = o.z;
    g0 = d.x; g1 = d.y; g2 = d.z;
    if (kDensity) e_pix = dens.err[px.out];
  }
  // T and S = sum_c g_c (C_c - acc_c): the loss-weighted colour behind the
  // current Gaussian (final colour minus what is composited in front of
  // and at it), updated as S -= w * sum_c g_c colour_c
  float T = 1.f, acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  if (chunk > 0 && !done) {
    const float4 st = state[((int64_t)slot * (TGS_RENDER_CHUNKS - 1) + chunk - 1) * kBlock + tid];
    T = st.x;
    acc0 = st.y;
    acc1 = st.z;
    acc2 = st.w;
  }
  float S = g0 * (Cout0 - acc0) + g1 * (Cout1 - acc1) + g2 * (Cout2 - acc2);

  Staged nxt = {};
  uint32_t g_after = 0;
  if (begin + tid < end) nxt = stage_load(a, list_id(a, L, begin + tid), x0, y0);
  if (begin + kBlock + tid < end) g_after = list_id(a, L, begin + kBlock + tid);

  for (uint32_t start = begin; start < end; start += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const bool live = start + tid < end;
    s_geo[tid] = live ? nxt.geo : make_float4(0.f, 0.f, 0.f, 0.f);
    s_app[tid] = live ? nxt.app : make_float4(0.f, 0.f, 0.f, 0.f);
    s_con[tid] = live ? nxt.con : make_float4(0.f, 0.f, 0.f, 0.f);
    s_gid[tid] = nxt.gid;
    __syncthreads();
    const uint32_t i1 = start + kBlock + tid, i2 = start + 2 * kBlock + tid;
    if (i1 < end) nxt = stage_load(a, g_after, x0, y0);
    if (i2 < end) g_after = list_id(a, L, i2);
    const int cnt = (int)min((uint32_t)kBlock, end - start);
    const uint32_t pos0 = start - range.x;
    for (int j = 0; j < cnt; j += kUnrollB) {
      if (__ballot(!done) == 0ull) break;  // the whole wave has finished
      float al[kUnrollB], Gv[kUnrollB], pw[kUnrollB], dxv[kUnrollB], dyv[kUnrollB];
      float pxx[kUnrollB], pxy[kUnrollB], pyy[kUnrollB];
#pragma unroll
      for (int u = 0; u < kUnrollB; ++u) {
        const float4 ge = s_geo[j + u];
        const float4 ap = s_app[j + u];
        dxv[u] = lx - ge.x;
        dyv[u] = ly - ge.y;
        pw[u] = splat_exponent_p(dxv[u], dyv[u], ge.z, ge.w, ap.x, pxx[u], pxy[u], pyy[u]);
        al[u] = splat_alpha(pw[u], ap.y, amax, Gv[u]);
      }
#pragma unroll
      for (int u = 0; u < kUnrollB; ++u) {
        if (j + u >= cnt) break;  // uniform
        const float4 ap = s_app[j + u];
        const float4 cn = s_con[j + u];
        const float alpha = al[u];
        const bool ok = !done && pw[u] <= 0.f && alpha >= amin;
        const float w = ok ? alpha * T : 0.f;
        // loss-weighted colour of this Gaussian: sum_c g_c colour_c
        const float gc = __builtin_fmaf(g2, cn.w, __builtin_fmaf(g1, ap.w, g0 * ap.z));
        const float T_before = T;
        T = ok ? one_minus_times(T, alpha) : T;
        S = __builtin_fmaf(-w, gc, S);
        done = done || (pos0 + (uint32_t)(j + u) + 1u >= last);
        if (__ballot(ok) != 0ull) {  // the gradient terms only where some lane composited
          const float G = Gv[u], dx = dxv[u], dy = dyv[u];
          const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
          // dL/dalpha = T_before sum_c g_c colour_c - S / (1 - alpha)
          const float dalpha = __builtin_fmaf(T_before, gc, -S * inv);
          const bool unclamped = ok && ap.y * G < amax;
          const float dop = unclamped ? G * dalpha : 0.f;
          const float dpow = ap.y * dop;
          const float hdp = -0.5f * dpow;
          float v[9];
          v[0] = (cn.x * dx + cn.y * dy) * dpow;
          v[1] = (cn.y * dx + cn.z * dy) * dpow;
          v[2] = pxx[u] * hdp;
          v[3] = pxy[u] * (2.f * hdp);
          v[4] = pyy[u] * hdp;
          v[5] = dop;
          v[6] = w * g0;
          v[7] = w * g1;
          v[8] = w * g2;
          const uint32_t gid = __builtin_amdgcn_readfirstlane(s_gid[j + u]);  // uniform
          if (touched != nullptr && lane_id() == 0) touched[gid] = 1u;  // composited at a sample
          if constexpr (kDet) {
            // the pair's index in vals (the deterministic backward takes single-segment lists)
            const size_t rec = (size_t)(L.b1 + start + (uint32_t)(j + u)) * (kBlock / kWave) + (size_t)(tid / kWave);
            wave_sum9_store(v, g2d + rec * 9, sl);
          } else if constexpr (kDensity) {
            constexpr float kTwoLn2 = 1.3862943611198906f;
            const float dist = __builtin_sqrtf(fmaxf(-kTwoLn2 * pw[u], 0.f));
            const float nx = hw * v[0], ny = hh * v[1];
            const float v13[13] = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8],
                                   e_pix * w, w, dist * w, __builtin_sqrtf(nx * nx + ny * ny)};
            wave_sum13_atomic(v13, g2d + (size_t)gid * 9, dens.stats, gid, dens.n, sl);
          } else {
            wave_sum9_atomic(v, g2d + (size_t)gid * 9, sl);
          }
        }
      }
    }
  }
}

// Back-projection of per-pixel statistics onto the Gaussians (Sec. 3.8,
// Eq. gauss_err_accum): the forward walk is replayed with the same alpha
// decisions, bounded by the forward's contributor count, and every
// composited Gaussian collects e(p) w, w and D(p) w with w = T alpha and
// D(p) = sqrt(d^T Q d) = sqrt(-2 ln2 p2) (p2 is the staged exponent, log2(e)
// times the power).  Per Gaussian the three values are summed across the
// wave (lane-half swaps, then DPP within rows of 16) and three lanes issue
// one float atomic each into stats[gid][0 | 1 | 2] (one 16-byte slot, so the
// three atomics touch one cache line).  With the forward's
// state record the walk is split into chunks exactly as the backward's.
template <int kBlock, bool kDense>
__global__ void __launch_bounds__(kBlock) render_accum_kernel(RasterArgs a, const uint32_t* __restrict__ ncontrib,
                                                              const float* __restrict__ err, int64_t n,
                                                              float* __restrict__ stats,
                                                              const float4* __restrict__ state) {
  __shared__ float4 s_geo[kBlock];
  __shared__ float s_opa[kBlock];
  __shared__ float s_cc[kBlock];
  __shared__ uint32_t s_gid[kBlock];
  // the last chunk (the rest of the list, the longest walks) is dispatched
  // first, so its workgroups run beside the fixed-length chunks
  const int slot = blockIdx.x, chunk = (int)gridDim.y - 1 - (int)blockIdx.y, tid = threadIdx.x;
  const int tile = kDense ? slot : a.valid_tiles[slot];
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const TileList L = tile_list(a, tile);
  const uint2 range = make_uint2(0u, L.len);
  const uint32_t begin = range.x + (uint32_t)(chunk * TGS_RENDER_CHUNK_LEN);
  if (begin >= range.y && chunk > 0) return;  // workgroup-uniform
  const uint32_t end =
      chunk + 1 == (int)gridDim.y ? range.y : min(range.y, begin + (uint32_t)TGS_RENDER_CHUNK_LEN);
  const PixelSlot px = pixel_of<kBlock, kDense>(a, slot, tile, tid);
  const float lx = (float)(px.loc & 15), ly = (float)(px.loc >> 4);
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const float amin = a.alpha_min, amax = a.alpha_max;
  constexpr float kTwoLn2 = 1.3862943611198906f;
  // lane 0 of row 0 sums field 0, lane 0 of row 2 field 1, lane 0 of row 1 field 2
  const int lane = lane_id();
  const int field = (lane & 15) != 0 ? -1 : (lane == 0 ? 0 : (lane == 32 ? 1 : (lane == 16 ? 2 : -1)));

  float e = 0.f;
  uint32_t last = 0;
  if (px.inside) {
    e = err[px.out];
    last = ncontrib[px.out];
  }
  bool done = last <= begin - range.x;  // nothing composited from this chunk on
  float T = 1.f;
  if (chunk > 0 && !done) T = state[((int64_t)slot * (TGS_RENDER_CHUNKS - 1) + chunk - 1) * kBlock + tid].x;

  Staged nxt = {};
  uint32_t g_after = 0;
  if (begin + tid < end) nxt = stage_load(a, list_id(a, L, begin + tid), x0, y0);
  if (begin + kBlock + tid < end) g_after = list_id(a, L, begin + kBlock + tid);

  for (uint32_t start = begin; start < end; start += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const bool live = start + tid < end;
    s_geo[tid] = live ? nxt.geo : make_float4(0.f, 0.f, 0.f, 0.f);
    s_cc[tid] = live ? nxt.app.x : 0.f;
    s_opa[tid] = live ? nxt.app.y : 0.f;
    s_gid[tid] = nxt.gid;
    __syncthreads();
    const uint32_t i1 = start + kBlock + tid, i2 = start + 2 * kBlock + tid;
    if (i1 < end) nxt = stage_load(a, g_after, x0, y0);
    if (i2 < end) g_after = list_id(a, L, i2);
    const int cnt = (int)min((uint32_t)kBlock, end - start);
    const uint32_t pos0 = start - range.x;
    for (int j = 0; j < cnt; j += kUnrollB) {
      if (__ballot(!done) == 0ull) break;  // the whole wave has finished
      float al[kUnrollB], pw[kUnrollB];
#pragma unroll
      for (int u = 0; u < kUnrollB; ++u) {
        const float4 ge = s_geo[j + u];
        pw[u] = splat_exponent(lx - ge.x, ly - ge.y, ge.z, ge.w, s_cc[j + u]);
        float G;
        al[u] = splat_alpha(pw[u], s_opa[j + u], amax, G);
      }
#pragma unroll
      for (int u = 0; u < kUnrollB; ++u) {
        if (j + u >= cnt) break;  // uniform
        const bool ok = !done && pw[u] <= 0.f && al[u] >= amin;
        const float w = ok ? al[u] * T : 0.f;
        T = ok ? one_minus_times(T, al[u]) : T;
        done = done || (pos0 + (uint32_t)(j + u) + 1u >= last);
        if (__ballot(ok) != 0ull) {
          const float dist = __builtin_sqrtf(fmaxf(-kTwoLn2 * pw[u], 0.f));
          const float p01 = swap_sum32(e * w, w);
          const float p2 = swap_sum32(dist * w, 0.f);
          float r = row_sum16(swap_sum16(p01, p2));
          asm volatile("" : "+v"(r));  // the whole row sum with the whole wave active
          const uint32_t gid = __builtin_amdgcn_readfirstlane(s_gid[j + u]);  // uniform
          if (field >= 0 && r != 0.f && gid < (uint32_t)n) unsafeAtomicAdd(&stats[(int64_t)gid * 4 + field], r);
        }
      }
    }
  }
}

template <int kBlock, bool kDense>
static void launch_fwd(const RasterArgs& a, int grid, float* out, uint32_t* ncontrib,
                       uint64_t* counters, float* state, hipStream_t s) {
  hipLaunchKernelGGL((render_fwd_kernel<kBlock, kDense>), dim3(grid), dim3(kBlock), 0, s, a,
                     (float4*)out, ncontrib, (unsigned long long*)counters, (float4*)state);
}

template <int kBlock, bool kDense>
static void launch_bwd(const RasterArgs& a, int grid, const float* out, const uint32_t* ncontrib,
                       const float* dL, float* g2d, const float* state, uint8_t* touched, hipStream_t s,
                       const DensityArgs* dens = nullptr) {
  const unsigned chunks = state != nullptr ? TGS_RENDER_CHUNKS : 1;
  if (dens != nullptr)
    hipLaunchKernelGGL((render_bwd_kernel<kBlock, kDense, true>), dim3(grid, chunks), dim3(kBlock), 0, s, a,
                       (const float4*)out, ncontrib, (const float4*)dL, g2d, (const float4*)state, touched, *dens);
  else
    hipLaunchKernelGGL((render_bwd_kernel<kBlock, kDense>), dim3(grid, chunks), dim3(kBlock), 0, s, a,
                       (const float4*)out, ncontrib, (const float4*)dL, g2d, (const float4*)state, touched,
                       DensityArgs{});
}

template <int kBlock, bool kDense>
static void launch_bwd_det(const RasterArgs& a, int grid, const float* out, const uint32_t* ncontrib,
                           const float* dL, float* partial, const float* state, uint8_t* touched, hipStream_t s) {
  const unsigned chunks = state != nullptr ? TGS_RENDER_CHUNKS : 1;
  hipLaunchKernelGGL((render_bwd_kernel<kBlock, kDense, false, true>), dim3(grid, chunks), dim3(kBlock), 0, s, a,
                     (const float4*)out, ncontrib, (const float4*)dL, partial, (const float4*)state, touched,
                     DensityArgs{});
}

__global__ void __launch_bounds__(256) zero_f32_kernel(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// Deterministic reduction of the partial records: a thread per Gaussian
// visits the tiles of its rectangle in row-major order, finds its pair in
// the tile's list by binary search on (depth bits, id) (the list's order),
// and adds the pair's wave records in wave order; the total is added to
// g2d once.  Any order would do; a fixed one gives the same bits on every
// run.
__global__ void __launch_bounds__(256) det_reduce_kernel(const int4* __restrict__ rect, const float* __restrict__ depth,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint2* __restrict__ ranges, int64_t n, int tiles_x,
                                                         int tiles_y, int waves, const float* __restrict__ partial,
                                                         float* __restrict__ g2d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int4 r = rect[i];
  r.x = min(max(r.x, 0), tiles_x);
  r.z = min(max(r.z, r.x), tiles_x);
  r.y = min(max(r.y, 0), tiles_y);
  r.w = min(max(r.w, r.y), tiles_y);
  const uint32_t key = __float_as_uint(depth[i]), id = (uint32_t)i;
  float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool any = false;
  for (int ty = r.y; ty < r.w; ++ty)
    for (int tx = r.x; tx < r.z; ++tx) {
      const uint2 rg = ranges[ty * tiles_x + tx];
      uint32_t lo = rg.x, hi = rg.y;
      while (lo < hi) {  // first position not below (key, id)
        const uint32_t mid = lo + (hi - lo) / 2;
        const uint32_t gm = vals[mid], km = __float_as_uint(depth[gm]);
        if (km < key || (km == key && gm < id)) lo = mid + 1;
        else hi = mid;
      }
      if (lo < rg.y && vals[lo] == id) {
        const float* p = partial + (size_t)lo * waves * 9;
        for (int w = 0; w < waves; ++w)
          for (int f = 0; f < 9; ++f) acc[f] += p[w * 9 + f];
        any = true;
      }
    }
  if (any)
    for (int f = 0; f < 9; ++f) g2d[i * 9 + f] += acc[f];
}

// Workgroup size of the raster kernels for a launch.
static int raster_block(bool dense, int32_t max_per_tile) {
  if (dense || max_per_tile > 128) return 256;
  return max_per_tile <= 64 ? 64 : 128;
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
  a.vals2 = nullptr;
  a.ranges2 = nullptr;
  a.mode = 0;
  a.cont_slot = nullptr;
  a.cont_list = nullptr;
  a.cont_count = nullptr;
  return TGS_OK;
}

// The second list segment of the two-segment entry points.
static int32_t set_second(RasterArgs& a, const uint32_t* vals2, const uint32_t* ranges2, const char* who) {
  TGS_REQUIRE(vals2 && ranges2, "%s: null vals2/ranges2", who);
  a.vals2 = vals2;
  a.ranges2 = (const uint2*)ranges2;
  return TGS_OK;
}

__global__ void __launch_bounds__(256) fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v,
                                                       uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
  if (i == 0 && count != nullptr) *count = 0u;
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_render_state_size(int32_t n_slots, int32_t max_per_tile) {
  if (n_slots < 0 || max_per_tile < 0 || max_per_tile > kTilePixels) return 0;
  return (size_t)n_slots * (TGS_RENDER_CHUNKS - 1) * (size_t)raster_block(false, max_per_tile) * sizeof(float4);
}

static int32_t render_fwd_launch(const RasterArgs& a, bool dense, int32_t n_st, int32_t max_per_tile, float* out,
                                 uint32_t* ncontrib, uint64_t* counters, float* state, hipStream_t s,
                                 const char* who) {
  TGS_REQUIRE(out && ncontrib, "%s: null output", who);
  TGS_REQUIRE(((uintptr_t)out & 15) == 0 && ((uintptr_t)state & 15) == 0, "%s: out and state must be 16-byte aligned",
              who);
  if (dense) {
    launch_fwd<256, true>(a, a.tiles_x * a.tiles_y, out, ncontrib, counters, state, s);
  } else if (n_st > 0) {
    if (max_per_tile <= 64) launch_fwd<64, false>(a, n_st, out, ncontrib, counters, state, s);
    else if (max_per_tile <= 128) launch_fwd<128, false>(a, n_st, out, ncontrib, counters, state, s);
    else launch_fwd<256, false>(a, n_st, out, ncontrib, counters, state, s);
  }
  return hip_status(who);
}

extern "C" int32_t tgs_render_fwd(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                  int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                  const int32_t* valid_tiles, const int32_t* tile_off,
                                  const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                  const tgs_raster_params* rp, float* out, uint32_t* ncontrib,
                                  uint64_t* counters, float* state, void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_render_fwd", a))
    return e;
  return render_fwd_launch(a, valid_tiles == nullptr, n_st, max_per_tile, out, ncontrib, counters, state,
                           as_stream(stream), "tgs_render_fwd");
}

extern "C" int32_t tgs_render_fwd_prefix(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                         int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                         const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                                         int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp, float* out,
                                         uint32_t* ncontrib, uint64_t* counters, float* state, int32_t* cont_slot,
                                         uint32_t* cont_list, uint32_t* cont_count, void* stream) {
  const char* who = "tgs_render_fwd_prefix";
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix, n_st,
                            max_per_tile, rp, who, a))
    return e;
  TGS_REQUIRE(cont_slot && cont_list && cont_count, "%s: null continuation outputs", who);
  a.mode = 1;
  a.cont_slot = cont_slot;
  a.cont_list = cont_list;
  a.cont_count = cont_count;
  hipStream_t s = as_stream(stream);
  const int64_t n_t = (int64_t)tiles_x * tiles_y;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)ceil_div(n_t, 256)), dim3(256), 0, s, cont_slot, n_t, -1,
                     cont_count);
  return render_fwd_launch(a, valid_tiles == nullptr, n_st, max_per_tile, out, ncontrib, counters, state, s, who);
}

extern "C" int32_t tgs_render_fwd_cont(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                       const uint32_t* vals2, const uint32_t* ranges2, int32_t tiles_x,
                                       int32_t tiles_y, int32_t width, int32_t height, const int32_t* valid_tiles,
                                       const int32_t* tile_off, const uint8_t* pix, int32_t n_st,
                                       int32_t max_per_tile, const tgs_raster_params* rp, const uint32_t* cont_list,
                                       const uint32_t* cont_count, float* out, uint32_t* ncontrib,
                                       uint64_t* counters, float* state, void* stream) {
  const char* who = "tgs_render_fwd_cont";
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix, n_st,
                            max_per_tile, rp, who, a))
    return e;
  if (int32_t e = set_second(a, vals2, ranges2, who)) return e;
  TGS_REQUIRE(cont_list && cont_count, "%s: null continuation list", who);
  a.mode = 2;
  a.cont_list = (uint32_t*)cont_list;
  a.cont_count = (uint32_t*)cont_count;
  return render_fwd_launch(a, valid_tiles == nullptr, n_st, max_per_tile, out, ncontrib, counters, state,
                           as_stream(stream), who);
}

static int32_t render_bwd_launch(const RasterArgs& a, bool dense, int32_t n_st, int32_t max_per_tile,
                                 const float* out, const uint32_t* ncontrib, const float* dL_dout, float* g2d,
                                 const float* state, uint8_t* touched, const DensityArgs* dens, hipStream_t s,
                                 const char* who) {
  TGS_REQUIRE(out && ncontrib && dL_dout && g2d, "%s: null pointer", who);
  TGS_REQUIRE(((uintptr_t)out & 15) == 0 && ((uintptr_t)dL_dout & 15) == 0 && ((uintptr_t)state & 15) == 0,
              "%s: out, dL_dout and state must be 16-byte aligned", who);
  if (dense) {
    launch_bwd<256, true>(a, a.tiles_x * a.tiles_y, out, ncontrib, dL_dout, g2d, state, touched, s, dens);
  } else if (n_st > 0) {
    if (max_per_tile <= 64) launch_bwd<64, false>(a, n_st, out, ncontrib, dL_dout, g2d, state, touched, s, dens);
    else if (max_per_tile <= 128)
      launch_bwd<128, false>(a, n_st, out, ncontrib, dL_dout, g2d, state, touched, s, dens);
    else launch_bwd<256, false>(a, n_st, out, ncontrib, dL_dout, g2d, state, touched, s, dens);
  }
  return hip_status(who);
}

extern "C" int32_t tgs_render_bwd(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                  int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                  const int32_t* valid_tiles, const int32_t* tile_off,
                                  const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                  const tgs_raster_params* rp, const float* out,
                                  const uint32_t* ncontrib, const float* dL_dout, float* g2d,
                                  const float* state, uint8_t* touched, void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_render_bwd", a))
    return e;
  return render_bwd_launch(a, valid_tiles == nullptr, n_st, max_per_tile, out, ncontrib, dL_dout, g2d, state,
                           touched, nullptr, as_stream(stream), "tgs_render_bwd");
}

extern "C" int32_t tgs_render_bwd2(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                   const uint32_t* vals2, const uint32_t* ranges2, int32_t tiles_x, int32_t tiles_y,
                                   int32_t width, int32_t height, const int32_t* valid_tiles,
                                   const int32_t* tile_off, const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                   const tgs_raster_params* rp, const float* out, const uint32_t* ncontrib,
                                   const float* dL_dout, float* g2d, const float* state, uint8_t* touched,
                                   const float* err, int64_t n, float* stats, void* stream) {
  const char* who = "tgs_render_bwd2";
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles, tile_off, pix, n_st,
                            max_per_tile, rp, who, a))
    return e;
  if (int32_t e = set_second(a, vals2, ranges2, who)) return e;
  DensityArgs d{err, stats, n};
  if (stats != nullptr) {
    TGS_REQUIRE(err != nullptr && n > 0 && n < (1ll << 31), "%s: density sums need err and n", who);
    TGS_REQUIRE(((uintptr_t)stats & 15) == 0, "%s: stats must be 16-byte aligned", who);
  }
  return render_bwd_launch(a, valid_tiles == nullptr, n_st, max_per_tile, out, ncontrib, dL_dout, g2d, state,
                           touched, stats != nullptr ? &d : nullptr, as_stream(stream), who);
}

extern "C" size_t tgs_render_bwd_det_workspace_size(int64_t n_pairs, int32_t max_per_tile, int32_t dense) {
  if (n_pairs < 0 || max_per_tile < 0 || max_per_tile > kTilePixels) return 0;
  const int waves = raster_block(dense != 0, max_per_tile) / kWave;
  return (size_t)std::max<int64_t>(n_pairs, 1) * (size_t)waves * 9 * sizeof(float);
}

extern "C" int32_t tgs_render_bwd_deterministic(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                                int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                                const int32_t* valid_tiles, const int32_t* tile_off,
                                                const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                                const tgs_raster_params* rp, const float* out,
                                                const uint32_t* ncontrib, const float* dL_dout, float* g2d,
                                                const float* state, uint8_t* touched, const float* depth,
                                                const int32_t* rect, int64_t n, int64_t n_pairs, void* ws,
                                                size_t ws_bytes, void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_render_bwd_deterministic", a))
    return e;
  TGS_REQUIRE(out && ncontrib && dL_dout && g2d && depth && rect && ws, "tgs_render_bwd_deterministic: null pointer");
  TGS_REQUIRE(n >= 0 && n < (1ll << 31) && n_pairs >= 0 && n_pairs < (1ll << 32),
              "tgs_render_bwd_deterministic: n or n_pairs out of range");
  TGS_REQUIRE(((uintptr_t)out & 15) == 0 && ((uintptr_t)dL_dout & 15) == 0 && ((uintptr_t)state & 15) == 0 &&
                  ((uintptr_t)rect & 15) == 0 && ((uintptr_t)ws & 15) == 0,
              "tgs_render_bwd_deterministic: out, dL_dout, state, rect and ws must be 16-byte aligned");
  const bool dense = valid_tiles == nullptr;
  const size_t need = tgs_render_bwd_det_workspace_size(n_pairs, max_per_tile, dense);
  TGS_REQUIRE(ws_bytes >= need, "tgs_render_bwd_deterministic: workspace %zu bytes < %zu", ws_bytes, need);
  hipStream_t s = as_stream(stream);
  float* partial = (float*)ws;
  const int waves = raster_block(dense, max_per_tile) / kWave;
  const int64_t words = std::max<int64_t>(n_pairs, 1) * waves * 9;
  hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(words, 256), 8192)), dim3(256), 0,
                     s, partial, words);
  if (dense) {
    launch_bwd_det<256, true>(a, tiles_x * tiles_y, out, ncontrib, dL_dout, partial, state, touched, s);
  } else if (n_st > 0) {
    if (max_per_tile <= 64) launch_bwd_det<64, false>(a, n_st, out, ncontrib, dL_dout, partial, state, touched, s);
    else if (max_per_tile <= 128)
      launch_bwd_det<128, false>(a, n_st, out, ncontrib, dL_dout, partial, state, touched, s);
    else launch_bwd_det<256, false>(a, n_st, out, ncontrib, dL_dout, partial, state, touched, s);
  }
  if (n > 0)
    hipLaunchKernelGGL(det_reduce_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, (const int4*)rect,
                       depth, vals, (const uint2*)ranges, n, tiles_x, tiles_y, waves, partial, g2d);
  return hip_status("tgs_render_bwd_deterministic");
}

extern "C" int32_t tgs_render_bwd_density(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                          int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                          const int32_t* valid_tiles, const int32_t* tile_off,
                                          const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                          const tgs_raster_params* rp, const float* out,
                                          const uint32_t* ncontrib, const float* dL_dout, float* g2d,
                                          const float* state, uint8_t* touched, const float* err, int64_t n,
                                          float* stats, void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_render_bwd_density", a))
    return e;
  TGS_REQUIRE(out && ncontrib && dL_dout && g2d && err && stats, "tgs_render_bwd_density: null pointer");
  TGS_REQUIRE(n > 0 && n < (1ll << 31), "tgs_render_bwd_density: n out of range");
  TGS_REQUIRE(((uintptr_t)stats & 15) == 0, "tgs_render_bwd_density: stats must be 16-byte aligned");
  TGS_REQUIRE(((uintptr_t)out & 15) == 0 && ((uintptr_t)dL_dout & 15) == 0 && ((uintptr_t)state & 15) == 0,
              "tgs_render_bwd_density: out, dL_dout and state must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  const DensityArgs d{err, stats, n};
  if (valid_tiles == nullptr) {
    launch_bwd<256, true>(a, tiles_x * tiles_y, out, ncontrib, dL_dout, g2d, state, touched, s, &d);
  } else if (n_st > 0) {
    if (max_per_tile <= 64) launch_bwd<64, false>(a, n_st, out, ncontrib, dL_dout, g2d, state, touched, s, &d);
    else if (max_per_tile <= 128)
      launch_bwd<128, false>(a, n_st, out, ncontrib, dL_dout, g2d, state, touched, s, &d);
    else launch_bwd<256, false>(a, n_st, out, ncontrib, dL_dout, g2d, state, touched, s, &d);
  }
  return hip_status("tgs_render_bwd_density");
}

static int32_t density_accumulate_launch(const RasterArgs& a, const int32_t* valid_tiles, int32_t n_st,
                                         int32_t max_per_tile, const uint32_t* ncontrib, const float* err,
                                         const float* state, int64_t n, float* stats, void* stream);

extern "C" int32_t tgs_density_accumulate(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                          int32_t tiles_x, int32_t tiles_y, int32_t width, int32_t height,
                                          const int32_t* valid_tiles, const int32_t* tile_off,
                                          const uint8_t* pix, int32_t n_st, int32_t max_per_tile,
                                          const tgs_raster_params* rp, const uint32_t* ncontrib,
                                          const float* err, const float* state, int64_t n, float* stats,
                                          void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_density_accumulate", a))
    return e;
  return density_accumulate_launch(a, valid_tiles, n_st, max_per_tile, ncontrib, err, state, n, stats, stream);
}

extern "C" int32_t tgs_density_accumulate2(const float* splat, const uint32_t* vals, const uint32_t* ranges,
                                           const uint32_t* vals2, const uint32_t* ranges2, int32_t tiles_x,
                                           int32_t tiles_y, int32_t width, int32_t height,
                                           const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                                           int32_t n_st, int32_t max_per_tile, const tgs_raster_params* rp,
                                           const uint32_t* ncontrib, const float* err, const float* state,
                                           int64_t n, float* stats, void* stream) {
  RasterArgs a;
  if (int32_t e = make_args(splat, vals, ranges, tiles_x, tiles_y, width, height, valid_tiles,
                            tile_off, pix, n_st, max_per_tile, rp, "tgs_density_accumulate2", a))
    return e;
  if (int32_t e = set_second(a, vals2, ranges2, "tgs_density_accumulate2")) return e;
  return density_accumulate_launch(a, valid_tiles, n_st, max_per_tile, ncontrib, err, state, n, stats, stream);
}

static int32_t density_accumulate_launch(const RasterArgs& a, const int32_t* valid_tiles, int32_t n_st,
                                         int32_t max_per_tile, const uint32_t* ncontrib, const float* err,
                                         const float* state, int64_t n, float* stats, void* stream) {
  const int tiles_x = a.tiles_x, tiles_y = a.tiles_y;
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_density_accumulate: n out of range");
  TGS_REQUIRE(ncontrib && err && stats, "tgs_density_accumulate: null pointer");
  TGS_REQUIRE(((uintptr_t)stats & 15) == 0, "tgs_density_accumulate: stats must be 16-byte aligned");
  TGS_REQUIRE(((uintptr_t)state & 15) == 0, "tgs_density_accumulate: state must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  if (n == 0) return hip_status("tgs_density_accumulate");
  const unsigned chunks = state != nullptr ? TGS_RENDER_CHUNKS : 1;
  const float4* st = (const float4*)state;
#define TGS_ACCUM(BLK, DENSE, GRID) \
  hipLaunchKernelGGL((render_accum_kernel<BLK, DENSE>), dim3(GRID, chunks), dim3(BLK), 0, s, a, ncontrib, err, n, \
                     stats, st)
  if (valid_tiles == nullptr) {
    TGS_ACCUM(256, true, tiles_x * tiles_y);
  } else if (n_st > 0) {
    if (max_per_tile <= 64) TGS_ACCUM(64, false, n_st);
    else if (max_per_tile <= 128) TGS_ACCUM(128, false, n_st);
    else TGS_ACCUM(256, false, n_st);
  }
#undef TGS_ACCUM
  return hip_status("tgs_density_accumulate");
}
