// Tile x depth binning, sort and per-tile ranges.
//
// The per-tile Gaussian lists must follow (tile, FP32 depth bits, Gaussian
// id) and hold only the (Gaussian, tile) pairs whose tile can composite: the
// tile lies in the Gaussian's 3-sigma rectangle and its pixel-centre
// rectangle meets the ellipse q(d) <= tau of the stored centre and conic.
// Row by row that is an interval of columns (row_span, FP64 with a fixed
// operation order).  Rather than radix-sorting a 64-bit (tile, depth) key
// with an id for every pair, the Gaussians are put in (depth, id) order once
// (a 32-bit sort of n keys) and the pairs are emitted in that order; a
// stable sort on the tile bits alone then yields the full order.  The pair
// key is (tile << id_bits) | Gaussian id, usually 32 bits: the id bits only
// ride along, since a stable sort never compares them.
//
//   count     a thread per Gaussian over its rectangle rows: kept pairs in
//             valid tiles, depth key (Gaussians without a kept valid tile
//             get a key above every depth), touched flag
//   sort      LSD radix sort of (depth key, id) over n, one kernel per pass:
//             stable, so ties keep id order; Gaussians with pairs come
//             first; the last pass gathers rectangles and pair counts into
//             depth order
//   scan      exclusive scan of the counts -> pair offsets; the totals are
//             read back once
//   emit      a wave per 32 depth-ordered Gaussians walks their rows; each
//             row's span (its valid columns, with a tile subset) is keyed
//             and written contiguously after the rows before it
//   sort      LSD radix sort of the pair keys on the tile bits only; the
//             last pass writes the ids, the sorted keys and (if asked) the
//             64-bit keys
//   ranges    tile boundaries of the sorted keys -> [start, end) per tile
//
// A radix pass is a stable counting sort over blocks of 256 x kItems keys:
// per-block digit histograms, one scan of the digit-major histogram table,
// and a scatter that ranks the block's keys (peer lanes of a digit found by
// a ballot match; each wave owns a contiguous quarter of the block),
// reorders them by digit in LDS and writes runs of equal digits to
// consecutive addresses.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <utility>

#include "scan.h"

namespace tgs {

// Zeroes two arrays in one launch: [0, n0) of p0, then [0, n1) of p1.
__global__ void __launch_bounds__(256) zero2_u32_kernel(uint32_t* __restrict__ p0, int64_t n0,
                                                        uint32_t* __restrict__ p1, int64_t n1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n0) p0[i] = 0u;
  else if (i - n0 < n1) p1[i - n0] = 0u;
}

__global__ void __launch_bounds__(64) copy_counts_kernel(const unsigned long long* __restrict__ src,
                                                         unsigned long long* __restrict__ dst) {
  if (threadIdx.x < 2) dst[threadIdx.x] = src[threadIdx.x];
}

// Sums the count kernel's partial totals (one wave): counts[0] = pairs in
// valid tiles, counts[1] = all pairs, and the number of pairs the pair sort
// takes: all of them when they fit the capacity, else none.
__global__ void __launch_bounds__(64) totals_kernel(const unsigned long long* __restrict__ slots, int64_t capacity,
                                                    unsigned long long* __restrict__ counts,
                                                    uint32_t* __restrict__ eff_total) {
  const int i = threadIdx.x;
  unsigned long long v = 0, a = 0;
  for (int q = i; q < TGS_COUNTER_SLOTS; q += 64) {
    v += slots[q];
    a += slots[TGS_COUNTER_SLOTS + q];
  }
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_down(v, o, 64);
    a += __shfl_down(a, o, 64);
  }
  if (i == 0) {
    counts[0] = v;
    counts[1] = a;
    counts[3] = a;  // kept when a depth-prefix call replaces counts[1]
    *eff_total = a <= (unsigned long long)capacity ? (uint32_t)a : 0u;
  }
}

// The prefix call's three counts: lists' length, pairs emitted, whole-list pairs.
__global__ void __launch_bounds__(64) copy_counts3_kernel(const unsigned long long* __restrict__ src,
                                                          unsigned long long* __restrict__ dst) {
  if (threadIdx.x < 3) dst[threadIdx.x] = src[threadIdx.x == 2 ? 3 : threadIdx.x];
}

// ------------------------------------------------------------------ scans
template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const T* __restrict__ in, int64_t n,
                                                                  T* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  __shared__ T lds[kScanThreads / kWave];
  T total;
  block_exclusive_scan<kScanThreads, T>(s, lds, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Down-sweep of a block: its prefix is the sum of the earlier blocks' sums
// (each block adds them up itself, so the scan takes two launches).
template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const T* __restrict__ in, int64_t n,
                                                                const T* __restrict__ part,
                                                                T* __restrict__ out) {
  __shared__ T lds[kScanThreads / kWave];
  T before = 0;
  for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kScanThreads) before += part[b];
  T block_pre;
  (void)block_exclusive_scan<kScanThreads, T>(before, lds, &block_pre);
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  T total;
  T run = block_pre + block_exclusive_scan<kScanThreads, T>(s, lds, &total);
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) out[n] = run;
}

template <typename T>
__global__ void __launch_bounds__(64) set_kernel(T* __restrict__ p, T v) {
  if (threadIdx.x == 0) *p = v;
}

// out[0..n] = exclusive prefix of in[0..n) and the total.
template <typename T>
static void exclusive_scan(const T* in, T* out, int64_t n, T* partials, hipStream_t s) {
  const int64_t nb = scan_partials(n);
  if (nb == 0) {
    hipLaunchKernelGGL(set_kernel<T>, dim3(1), dim3(64), 0, s, out, (T)0);
    return;
  }
  hipLaunchKernelGGL(scan_reduce_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials);
  hipLaunchKernelGGL(scan_down_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials, out);
}

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials, hipStream_t s) {
  exclusive_scan<uint32_t>(in, out, n, partials, s);
}



// ------------------------------------------------------------------ row spans
// Depth key of a Gaussian without pairs: above every finite positive depth bit pattern.
constexpr uint32_t kCulledKey = 0xffffffffu;

// Rectangles are clamped to the tile grid (projection already does so; the
// clamp keeps every index of the binning in bounds for any input).
__device__ __forceinline__ int4 clamp_rect(int4 r, int tiles_x, int tiles_y) {
  r.x = min(max(r.x, 0), tiles_x);
  r.z = min(max(r.z, r.x), tiles_x);
  r.y = min(max(r.y, 0), tiles_y);
  r.w = min(max(r.w, r.y), tiles_y);
  return r;
}

// What the row test needs of one Gaussian: the stored centre (integer part
// and fraction) and conic widened to FP64 (exact), and per-Gaussian terms of
// the ellipse q(d) = A dx^2 + 2 B dx dy + C dy^2 <= t: det = AC - B^2,
// its half-height ym = sqrt(t A / det), ys = B sqrt(t / (C det)) (the
// rightmost point of the ellipse sits at dy = -ys, the leftmost at +ys) and
// tA = t A.  pd = 0 for a conic that is not positive definite.
//
// The bound t is the Gaussian's own: alpha = o exp(-q/2) reaches alpha_min
// only where q <= 2 ln(o / alpha_min), so t = that plus 0.004 (alpha below
// alpha_min by 0.2 % past it, far above the FP32 error of the renderer's
// alpha), rounded up to a multiple of 1/64, and at most tau (the bound for
// o = 1).  A Gaussian with t <= 0 keeps no tile (ym < 0 empties every row).
// lia = ln(1 / alpha_min).
struct RowEllipse {
  double xi, xf, yi, yf, A, B, det, ym, ys, tA;
  int pd;
};

__device__ __forceinline__ RowEllipse load_row_ellipse(const float4* __restrict__ splat, int64_t i, double tau,
                                                       double lia) {
#pragma clang fp contract(off)
  const float4 p0 = splat[3 * i], p1 = splat[3 * i + 1];
  RowEllipse e;
  const double o = (double)p1.w;
  const double t = o > 0.0 ? fmin(tau, ceil(64.0 * (2.0 * (log(o) + lia) + 0.004)) * (1.0 / 64.0)) : -1.0;
  e.xi = p0.x;
  e.yi = p0.y;
  e.xf = p0.z;
  e.yf = p0.w;
  // the record's conic is (a, beta, delta) with b = beta a, c = delta + beta b,
  // det = a c - b^2 = a delta
  e.A = p1.x;
  e.B = (double)p1.y * e.A;
  const double C = (double)p1.z + (double)p1.y * e.B;
  e.det = e.A * (double)p1.z;
  e.pd = e.A > 0.0 && e.det > 0.0;
  e.ym = !e.pd ? 0.0 : (t > 0.0 ? sqrt((t * e.A) / e.det) : -1.0);
  e.ys = e.pd && t > 0.0 ? e.B * sqrt(t / (C * e.det)) : 0.0;
  e.tA = t * e.A;
  return e;
}

// Kept columns [lo, hi] of tile row ty inside the rectangle columns
// [rx0, rx1) (lo > hi when none): the tiles whose pixel-centre column range
// meets the x-extent of the ellipse cut by the row's pixel-centre strip.
// The right boundary of the ellipse, x(dy) = (sqrt(tA - det dy^2) - B dy)/A,
// is concave, so the strip's rightmost point is at the ellipse's rightmost
// dy clamped to the strip (the leftmost likewise).  FP64, IEEE operations
// in a fixed order and no contraction: the decision is reproducible bit for
// bit by any implementation of the same order.
__device__ __forceinline__ void row_span(const RowEllipse& e, int ty, int rx0, int rx1, int& lo, int& hi) {
#pragma clang fp contract(off)
  if (!e.pd) {  // keeps the whole rectangle row
    lo = rx0;
    hi = rx1 - 1;
    return;
  }
  const double Y0 = ((double)(kTile * ty) - e.yi) - e.yf;
  const double Y1 = ((double)(kTile * ty + kTile - 1) - e.yi) - e.yf;
  const double ylo = fmax(Y0, -e.ym), yhi = fmin(Y1, e.ym);
  if (!(ylo <= yhi)) {
    lo = rx0;
    hi = rx0 - 1;
    return;
  }
  const double yr = fmin(fmax(-e.ys, ylo), yhi);
  const double yl = fmin(fmax(e.ys, ylo), yhi);
  const double sr = sqrt(fmax(0.0, e.tA - e.det * (yr * yr)));
  const double sl = sqrt(fmax(0.0, e.tA - e.det * (yl * yl)));
  const double xmax = (sr - e.B * yr) / e.A;
  const double xmin = (-sl - e.B * yl) / e.A;
  const double PL = (xmin + e.xf) + e.xi, PR = (xmax + e.xf) + e.xi;  // image pixel coordinates
  const double l = ceil((PL - (double)(kTile - 1)) * (1.0 / kTile));
  const double h = floor(PR * (1.0 / kTile));
  lo = (int)fmin(fmax(l, (double)rx0), (double)rx1);
  hi = (int)fmin(fmax(h, (double)(rx0 - 1)), (double)(rx1 - 1));
}

// Inclusive max-scan over the wave (identity -1): DPP shifts inside rows of
// 16, then the row broadcasts.
__device__ __forceinline__ int wave_max_scan(int v) {
  v = max(v, dpp_i<0x111>(-1, v));  // row_shr:1
  v = max(v, dpp_i<0x112>(-1, v));  // row_shr:2
  v = max(v, dpp_i<0x114>(-1, v));  // row_shr:4
  v = max(v, dpp_i<0x118>(-1, v));  // row_shr:8
  v = max(v, dpp_i<kDppRowBcast15, 0xa>(-1, v));
  v = max(v, dpp_i<kDppRowBcast31, 0xc>(-1, v));
  return v;
}

// ------------------------------------------------------------------ count
// Depth sort blocks (see depth_pass_kernel): 256 threads x 8 keys, 256 digits.
constexpr int kDepthItems = 8;
constexpr int kDepthBlockKeys = 256 * kDepthItems;
constexpr int kDepthDigits = 256;

// One wave per 64 Gaussians (in index order).  Their rectangle rows are
// flattened Gaussian by Gaussian and handed out 64 per round, so every lane
// evaluates a row span whatever the rectangles' heights; a Gaussian whose
// first row falls in the round marks its slot and an inclusive max-scan
// carries each owner to the following slots.  Per Gaussian: kept pairs in
// valid tiles (every kept pair when there is no tile subset), summed by LDS
// atomics; then the depth key (Gaussians without a kept valid tile get a key
// above every depth), pair count and touched flag.
constexpr int kCountBatch = kWave;  // Gaussians per wave (32 measured slower)

struct CountBatch {
  int4 rect[kWave];
  uint32_t row0[kWave];  // exclusive prefix of the row counts in the batch
  RowEllipse ell[kWave];
  int mark[kWave];
  uint32_t valid[kWave];
};

// ids == nullptr: Gaussian i of the index order (rect, depth by index),
// writing the depth keys.  ids != nullptr: position i of the depth order
// (rect is then the sorted rectangles, ids the Gaussians), writing only the
// counts by position (emit_cnt) and the touched flags.
__global__ void __launch_bounds__(kWave) count_kernel(
    const int4* __restrict__ rect, const uint32_t* __restrict__ ids, const float4* __restrict__ splat,
    const float* __restrict__ depth, int64_t n, const int32_t* __restrict__ tile_slot, int tiles_x, int tiles_y,
    double tau, double lia, uint32_t* __restrict__ dkeys, uint32_t* __restrict__ dvals,
    uint32_t* __restrict__ emit_cnt, uint8_t* __restrict__ touched, unsigned long long* __restrict__ totals) {
  __shared__ CountBatch cb;
  __shared__ uint64_t s_red[1];
  const int lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * kCountBatch + lane;
  const bool mine = lane < kCountBatch && i < n;
  int4 r = make_int4(0, 0, 0, 0);
  uint32_t g = (uint32_t)i;
  if (mine) {
    r = clamp_rect(rect[i], tiles_x, tiles_y);
    if (ids != nullptr) g = ids[i];
  }
  const uint32_t rows = r.z > r.x ? (uint32_t)(r.w - r.y) : 0u;
  const uint32_t incl = wave_inclusive_scan_u32(rows);
  const uint32_t my_row0 = incl - rows;
  const uint32_t n_rows = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  cb.rect[lane] = r;
  cb.row0[lane] = my_row0;
  cb.valid[lane] = 0u;
  if (rows > 0) cb.ell[lane] = load_row_ellipse(splat, g, tau, lia);
  int carry = -1;
  for (uint32_t f0 = 0; f0 < n_rows; f0 += kWave) {
    cb.mark[lane] = -1;
    __syncthreads();
    if (rows > 0 && my_row0 >= f0 && my_row0 - f0 < (uint32_t)kWave) cb.mark[my_row0 - f0] = lane;
    __syncthreads();
    const int jl = max(wave_max_scan(cb.mark[lane]), carry);
    carry = __builtin_amdgcn_readlane(jl, kWave - 1);
    const uint32_t f = f0 + (uint32_t)lane;
    // jl >= 0 whenever f < n_rows: the first Gaussian with rows starts at row 0
    if (f < n_rows && jl >= 0) {
      const int4 rj = cb.rect[jl];
      const int ty = rj.y + (int)(f - cb.row0[jl]);
      int lo, hi;
      row_span(cb.ell[jl], ty, rj.x, rj.z, lo, hi);
      uint32_t cv = (uint32_t)max(hi - lo + 1, 0);
      if (tile_slot != nullptr) {
        cv = 0u;
        const int32_t* trow = tile_slot + (int64_t)ty * tiles_x;
        for (int tx = lo; tx <= hi; ++tx) cv += trow[tx] >= 0 ? 1u : 0u;
      }
      if (cv > 0) atomicAdd(&cb.valid[jl], cv);
    }
    __syncthreads();  // the round's reads and sums before the next round's writes
  }
  __syncthreads();
  const uint32_t valid = cb.valid[lane];
  if (mine) {
    if (ids == nullptr) {
      dkeys[i] = valid > 0 ? __float_as_uint(depth[i]) : kCulledKey;
      dvals[i] = (uint32_t)i;
    }
    emit_cnt[i] = valid;  // only the valid tiles are listed
    if (touched != nullptr && valid > 0) touched[g] = 1;
  }
  // 64-bit totals, spread over slots: [0] pairs in valid tiles, [1] pairs
  // listed (the same count: the lists hold the valid tiles only)
  const uint64_t v2[2] = {valid, valid};
  for (int k = 0; k < 2; ++k) {
    uint64_t tot;
    block_exclusive_scan<kWave, uint64_t>(v2[k], s_red, &tot);
    if (lane == 0 && tot > 0)
      atomicAdd(&totals[k * TGS_COUNTER_SLOTS + (blockIdx.x & (TGS_COUNTER_SLOTS - 1))], (unsigned long long)tot);
  }
}

// Depth keys of the depth-prefix call, before any count: a Gaussian with a
// non-empty rectangle is keyed by its depth, the others sort last; the
// number of keyed Gaussians goes to the 64-bit slots of row 2.
__global__ void __launch_bounds__(256) key_kernel(const int4* __restrict__ rect, const float* __restrict__ depth,
                                                  int64_t n, int tiles_x, int tiles_y, uint32_t* __restrict__ dkeys,
                                                  uint32_t* __restrict__ dvals,
                                                  unsigned long long* __restrict__ totals) {
  __shared__ uint64_t s_red[1];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool keyed = false;
  if (i < n) {
    const int4 r = clamp_rect(rect[i], tiles_x, tiles_y);
    keyed = r.z > r.x && r.w > r.y;
    dkeys[i] = keyed ? __float_as_uint(depth[i]) : kCulledKey;
    dvals[i] = (uint32_t)i;
  }
  uint64_t tot;
  block_exclusive_scan<256, uint64_t>(keyed ? 1ull : 0ull, s_red, &tot);
  if (threadIdx.x == 0 && tot > 0)
    atomicAdd(&totals[2 * TGS_COUNTER_SLOTS + (blockIdx.x & (TGS_COUNTER_SLOTS - 1))], (unsigned long long)tot);
}

// The depth-prefix call's counts from the slots: counts[0] = pairs of the
// prefix in valid tiles, counts[1] = its pairs (the capacity it needs; the
// sort takes them when they fit), counts[3] = an estimate of the whole
// lists' pairs for sizing a continuation: the prefix's pairs per Gaussian
// times the keyed Gaussians (exact when the prefix holds them all; the
// nearest Gaussians cover the most tiles, so it tends to exceed the count).
__global__ void __launch_bounds__(64) prefix_totals_kernel(const unsigned long long* __restrict__ slots, int64_t m,
                                                           int64_t capacity, unsigned long long* __restrict__ counts,
                                                           uint32_t* __restrict__ eff_total) {
  const int i = threadIdx.x;
  unsigned long long v = 0, a = 0, k = 0;
  for (int q = i; q < TGS_COUNTER_SLOTS; q += 64) {
    v += slots[q];
    a += slots[TGS_COUNTER_SLOTS + q];
    k += slots[2 * TGS_COUNTER_SLOTS + q];
  }
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_down(v, o, 64);
    a += __shfl_down(a, o, 64);
    k += __shfl_down(k, o, 64);
  }
  if (i == 0) {
    counts[0] = v;
    counts[1] = a;
    const unsigned long long mk = (unsigned long long)(m < (int64_t)k ? m : (int64_t)k);
    counts[3] = mk >= k || mk == 0 ? a : (unsigned long long)ceil((double)a * (double)k / (double)mk);
    *eff_total = a <= (unsigned long long)capacity ? (uint32_t)a : 0u;
  }
}

// Per tile row, the running count of flagged tiles: rowc[y * (tiles_x + 1)
// + x] = flagged tiles among columns < x of row y (a wave per row, 64
// columns per scan).  Nothing to do when no tile is flagged.
__global__ void __launch_bounds__(kWave) flag_rows_kernel(const int32_t* __restrict__ flag_slot, int tiles_x,
                                                          const uint32_t* __restrict__ n_flagged,
                                                          uint32_t* __restrict__ rowc) {
  if (n_flagged != nullptr && *n_flagged == 0u) return;
  const int y = blockIdx.x, lane = lane_id();
  const int64_t W1 = tiles_x + 1;
  uint32_t carry = 0;
  if (lane == 0) rowc[y * W1] = 0u;
  for (int x0 = 0; x0 < tiles_x; x0 += kWave) {
    const int x = x0 + lane;
    const uint32_t f = x < tiles_x && flag_slot[(int64_t)y * tiles_x + x] >= 0 ? 1u : 0u;
    const uint32_t incl = carry + wave_inclusive_scan_u32(f);
    if (x < tiles_x) rowc[y * W1 + x + 1] = incl;
    carry = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  }
}

// The summed-area table of the flagged tiles: sat[y * (tiles_x + 1) + x] =
// flagged tiles in rows < y and columns < x, (tiles_y + 1) x (tiles_x + 1)
// entries built in LDS by one workgroup (row scans by the waves, then a
// column pass per thread).  Nothing to do when no tile is flagged.
constexpr int kSatWords = 12288;  // LDS words: grids up to this many (tiles_x + 1) (tiles_y + 1)

__global__ void __launch_bounds__(1024) flag_sat_kernel(const int32_t* __restrict__ flag_slot, int tiles_x,
                                                        int tiles_y, const uint32_t* __restrict__ n_flagged,
                                                        uint32_t* __restrict__ sat) {
  __shared__ uint32_t t[kSatWords];
  if (n_flagged != nullptr && *n_flagged == 0u) return;  // workgroup-uniform
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int W1 = tiles_x + 1, words = (tiles_y + 1) * W1;
  for (int x = tid; x < W1; x += 1024) t[x] = 0u;
  for (int y = wave; y < tiles_y; y += 1024 / kWave) {
    uint32_t carry = 0;
    if (lane == 0) t[(y + 1) * W1] = 0u;
    for (int x0 = 0; x0 < tiles_x; x0 += kWave) {
      const int x = x0 + lane;
      const uint32_t f = x < tiles_x && flag_slot[(int64_t)y * tiles_x + x] >= 0 ? 1u : 0u;
      const uint32_t incl = carry + wave_inclusive_scan_u32(f);
      if (x < tiles_x) t[(y + 1) * W1 + x + 1] = incl;
      carry = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    }
  }
  __syncthreads();
  // column prefix: a wave scans each of its columns, 64 rows at a time
  for (int x = wave; x < W1; x += 1024 / kWave) {
    uint32_t carry = 0;
    for (int y0 = 0; y0 <= tiles_y; y0 += kWave) {
      const int y = y0 + lane;
      const uint32_t incl = carry + wave_inclusive_scan_u32(y <= tiles_y ? t[y * W1 + x] : 0u);
      if (y <= tiles_y) t[y * W1 + x] = incl;
      carry = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    }
  }
  __syncthreads();
  for (int i = tid; i < words; i += 1024) sat[i] = t[i];
}

// Continuation counts: one wave per 64 Gaussians of the depth order from a
// given rank on (their rectangles, ids and, when known, first-pass pair
// counts in that order).  Per Gaussian: its kept pairs in the flagged tiles (tile map
// entry >= 0), by the same row spans.  Gaussians without pairs in the first
// pass, or whose rectangle holds no flagged tile (four reads of the
// summed-area table, or two reads of the row counts per rectangle row, when
// given), are skipped before their splat is read; the whole call is skipped
// when no tile is flagged (every count 0).
// The sum goes to the 64-bit totals (both slots).
__global__ void __launch_bounds__(kWave) count_cont_kernel(
    const int4* __restrict__ rect_sorted, const uint32_t* __restrict__ ids_sorted,
    const uint32_t* __restrict__ cnt_sorted, int64_t m, const float4* __restrict__ splat,
    const int32_t* __restrict__ flag_slot, const uint32_t* __restrict__ n_flagged,
    const uint32_t* __restrict__ rowc, const uint32_t* __restrict__ sat, int tiles_x, int tiles_y, double tau,
    double lia, uint32_t* __restrict__ cnt, unsigned long long* __restrict__ totals) {
  __shared__ CountBatch cb;
  __shared__ uint64_t s_red[1];
  const int lane = lane_id();
  const int64_t k = (int64_t)blockIdx.x * kCountBatch + lane;
  if (n_flagged != nullptr && *n_flagged == 0u) {  // workgroup-uniform
    if (k < m) cnt[k] = 0u;
    return;
  }
  bool mine = k < m && (cnt_sorted == nullptr || cnt_sorted[k] > 0);
  int4 r = make_int4(0, 0, 0, 0);
  uint32_t g = 0;
  if (mine) {
    r = clamp_rect(rect_sorted[k], tiles_x, tiles_y);
    if (sat != nullptr || rowc != nullptr) {
      const int64_t W1 = tiles_x + 1;
      uint32_t f = 0u;
      if (sat != nullptr)
        f = (sat[r.w * W1 + r.z] - sat[r.y * W1 + r.z]) - (sat[r.w * W1 + r.x] - sat[r.y * W1 + r.x]);
      else
        for (int y = r.y; y < r.w && f == 0u; ++y) f = rowc[y * W1 + r.z] - rowc[y * W1 + r.x];
      if (f == 0u) {
        mine = false;
        r = make_int4(0, 0, 0, 0);
      }
    }
    if (mine) g = ids_sorted[k];
  }
  const uint32_t rows = r.z > r.x ? (uint32_t)(r.w - r.y) : 0u;
  const uint32_t incl = wave_inclusive_scan_u32(rows);
  const uint32_t my_row0 = incl - rows;
  const uint32_t n_rows = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  cb.rect[lane] = r;
  cb.row0[lane] = my_row0;
  cb.valid[lane] = 0u;
  if (rows > 0) cb.ell[lane] = load_row_ellipse(splat, g, tau, lia);
  int carry = -1;
  for (uint32_t f0 = 0; f0 < n_rows; f0 += kWave) {
    cb.mark[lane] = -1;
    __syncthreads();
    if (rows > 0 && my_row0 >= f0 && my_row0 - f0 < (uint32_t)kWave) cb.mark[my_row0 - f0] = lane;
    __syncthreads();
    const int jl = max(wave_max_scan(cb.mark[lane]), carry);
    carry = __builtin_amdgcn_readlane(jl, kWave - 1);
    const uint32_t f = f0 + (uint32_t)lane;
    if (f < n_rows && jl >= 0) {
      const int4 rj = cb.rect[jl];
      const int ty = rj.y + (int)(f - cb.row0[jl]);
      int lo, hi;
      row_span(cb.ell[jl], ty, rj.x, rj.z, lo, hi);
      uint32_t cv = 0u;
      const int32_t* trow = flag_slot + (int64_t)ty * tiles_x;
      for (int tx = lo; tx <= hi; ++tx) cv += trow[tx] >= 0 ? 1u : 0u;
      if (cv > 0) atomicAdd(&cb.valid[jl], cv);
    }
    __syncthreads();
  }
  __syncthreads();
  const uint32_t valid = cb.valid[lane];
  if (k < m) cnt[k] = valid;
  uint64_t tot;
  block_exclusive_scan<kWave, uint64_t>((uint64_t)valid, s_red, &tot);
  if (lane == 0 && tot > 0)
    for (int q = 0; q < 2; ++q)
      atomicAdd(&totals[q * TGS_COUNTER_SLOTS + (blockIdx.x & (TGS_COUNTER_SLOTS - 1))], (unsigned long long)tot);
}

// ------------------------------------------------------------------ ranges
// A workgroup takes 256 x kRangeItems consecutive sorted pairs: their tile
// ids are loaded coalesced into LDS (with the one before the block), then
// each position is compared with its predecessor.  A tile boundary writes
// the start of the new tile and the end of the previous one, the last pair
// the end of its tile (a tile id >= n_t, which no list emits, would write
// nothing); empty tiles keep the [0, 0) of the fill.
constexpr int kRangeItems = 8;
constexpr int kRangeBlock = 256 * kRangeItems;

template <typename K>
__global__ void __launch_bounds__(256) ranges_kernel(const K* __restrict__ keys, uint32_t total_arg,
                                                     const uint32_t* __restrict__ total_dev, int id_bits,
                                                     uint32_t n_t, uint2* __restrict__ ranges) {
  const uint32_t total = total_dev != nullptr ? *total_dev : total_arg;  // the device count when given
  __shared__ uint32_t s_t[kRangeBlock + 1];  // s_t[0]: the pair before the block
  const uint32_t b0 = blockIdx.x * (uint32_t)kRangeBlock;
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kRangeItems; ++k) {
    const uint32_t i = b0 + (uint32_t)(k * 256 + tid);
    s_t[1 + k * 256 + tid] = i < total ? (uint32_t)(keys[i] >> id_bits) : 0xffffffffu;
  }
  if (tid == 0) s_t[0] = b0 > 0 ? (uint32_t)(keys[b0 - 1] >> id_bits) : 0xffffffffu;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRangeItems; ++k) {
    const int l = k * 256 + tid;
    const uint32_t i = b0 + (uint32_t)l;
    if (i >= total) break;
    const uint32_t t = s_t[1 + l], tp = s_t[l];
    if (i == 0 || t != tp) {
      if (t < n_t) ranges[t].x = i;
      if (i > 0 && tp < n_t) ranges[tp].y = i;
    }
    if (i == total - 1 && t < n_t) ranges[t].y = total;
  }
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kPairItems = 16;  // keys per thread of the pair sort

static int64_t sort_blocks(int64_t n, int items) { return ceil_div(n, (int64_t)kSortThreads * items); }

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave holding the same digit (inactive lanes excluded), found
// through LDS: each active lane clears its digit's mask word, ORs in its own
// lane bit and reads the word back.  The three LDS operations of one wave
// execute in order, so every read sees exactly the bits of the lanes that
// share the digit.  s_mask holds one word per digit, private to the wave.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid, uint64_t* s_mask) {
  uint64_t peers = 0ull;
  if (valid) {
    s_mask[d] = 0ull;
    __hip_atomic_fetch_or(&s_mask[d], 1ull << lane_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    peers = __hip_atomic_load(&s_mask[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  return peers;
}

// Per-block histogram: block b covers keys [b * 256 * kItems, ...), wave w
// the contiguous quarter w of it, 64 keys per round.
template <typename K, int kBits, int kItems>
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const K* __restrict__ keys, uint32_t n_arg,
                                                                 const uint32_t* __restrict__ n_dev, int shift,
                                                                 int nblocks, uint32_t* __restrict__ hist) {
  const uint32_t n = n_dev != nullptr ? *n_dev : n_arg;  // the device count when given
  // blocks past the count (a grid sized by the capacity) leave their entries
  // unwritten: the scan and the scatter stop at the last block that holds keys
  if (n_dev != nullptr && (int64_t)blockIdx.x * kSortThreads * kItems >= (int64_t)n) return;
  constexpr int kDigits = 1 << kBits;
  __shared__ uint32_t h[kDigits];
  for (int i = threadIdx.x; i < kDigits; i += kSortThreads) h[i] = 0;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int64_t wbase = (int64_t)blockIdx.x * kSortThreads * kItems + (int64_t)wave * kWave * kItems;
  K key[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = wbase + k * kWave + lane;
    key[k] = i < n ? keys[i] : (K)0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (wbase + k * kWave + lane < n) atomicAdd(&h[(uint32_t)(key[k] >> shift) & (kDigits - 1u)], 1u);
  __syncthreads();
  for (int dg = threadIdx.x; dg < kDigits; dg += kSortThreads)
    hist[(int64_t)dg * nblocks + blockIdx.x] = h[dg];
}

// One workgroup per digit: exclusive prefix of the digit's per-block counts
// (a contiguous row of the digit-major table) and the digit's total.
__global__ void __launch_bounds__(1024) digit_scan_kernel(const uint32_t* __restrict__ hist, int nblocks,
                                                          int stride, uint32_t* __restrict__ hoffs,
                                                          uint32_t* __restrict__ dtot,
                                                          const uint32_t* __restrict__ n_dev, int block_keys) {
  __shared__ uint32_t lds[1024 / kWave];
  // with a device count, only the blocks that hold keys have table entries
  if (n_dev != nullptr) nblocks = (int)min<int64_t>(nblocks, ceil_div((int64_t)*n_dev, (int64_t)block_keys));
  const int64_t row = (int64_t)blockIdx.x * stride;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nblocks; b0 += 1024) {
    const int b = b0 + (int)threadIdx.x;
    const uint32_t v = b < nblocks ? hist[row + b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024, uint32_t>(v, lds, &tot);
    if (b < nblocks) hoffs[row + b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Output of a scatter pass: the keys (and values) for the next pass; in the
// last pass of the pair sort also the Gaussian ids carried in the low key
// bits and optionally the 64-bit (tile << 32) | depth-bits keys.
struct ScatterOut {
  void* keys;
  uint32_t* vals;
  int id_bits;           // final pass: key = (tile << id_bits) | id
  const float* depth;    // final pass, for keys64
  uint64_t* keys64;      // final pass, nullable
};

template <typename K, bool kVals, bool kFinal, int kBits, int kItems>
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t n_arg,
    const uint32_t* __restrict__ n_dev, int shift, int nblocks, const uint32_t* __restrict__ offs,
    const uint32_t* __restrict__ dtot, ScatterOut o) {
  const uint32_t n = n_dev != nullptr ? *n_dev : n_arg;  // the device count when given
  constexpr int kDigits = 1 << kBits;
  constexpr int kBlockKeys = kSortThreads * kItems;
  if ((int64_t)blockIdx.x * kBlockKeys >= (int64_t)n) return;  // past the keys: nothing to place
  __shared__ uint32_t s_cnt[kSortWaves][kDigits];  // per-wave digit counts, then block-local offsets
  __shared__ uint32_t s_gbase[kDigits];            // global position of block-local position 0 of the digit
  __shared__ K s_keys[kBlockKeys];
  __shared__ uint32_t s_vals[kVals ? kBlockKeys : 1];
  __shared__ uint32_t s_red[kSortWaves];
  __shared__ uint64_t s_mask[kSortWaves][kDigits];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int i = tid; i < kSortWaves * kDigits; i += kSortThreads) (&s_cnt[0][0])[i] = 0;
  const int64_t blk0 = (int64_t)blockIdx.x * kBlockKeys;
  const int64_t wbase = blk0 + (int64_t)wave * kWave * kItems;
  K key[kItems];
  uint32_t val[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = wbase + k * kWave + lane;
    key[k] = i < n ? keys_in[i] : (K)0;
    if (kVals) val[k] = i < n ? vals_in[i] : 0u;
  }
  __syncthreads();
  // rank of each key among the wave's keys of the same digit (stable: by
  // round, then lane); the wave's running counts live in s_cnt[wave]
  const uint64_t below = lanes_below();
  uint32_t rank[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const bool valid = wbase + k * kWave + lane < n;
    const uint32_t d = (uint32_t)(key[k] >> shift) & (kDigits - 1u);
    const uint64_t peers = digit_peers(d, valid, s_mask[wave]);
    const uint32_t r = (uint32_t)__popcll(peers & below);
    const uint32_t before = valid ? s_cnt[wave][d] : 0u;
    rank[k] = before + r;
    if (valid && r == 0) s_cnt[wave][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // block-local start of each (digit, wave) and the digit's global base
  uint32_t pre[kSortWaves];
  uint32_t tot = 0;
  if (tid < kDigits)
    for (int w = 0; w < kSortWaves; ++w) {
      pre[w] = tot;
      tot += s_cnt[w][tid];
    }
  uint32_t all;
  const uint32_t lstart = block_exclusive_scan<kSortThreads, uint32_t>(tid < kDigits ? tot : 0u, s_red, &all);
  const uint32_t gstart =
      block_exclusive_scan<kSortThreads, uint32_t>(tid < kDigits ? dtot[tid] : 0u, s_red, &all);
  if (tid < kDigits) {
    for (int w = 0; w < kSortWaves; ++w) s_cnt[w][tid] = lstart + pre[w];
    s_gbase[tid] = gstart + offs[(int64_t)tid * nblocks + blockIdx.x] - lstart;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (wbase + k * kWave + lane < n) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kDigits - 1u);
      const uint32_t lp = s_cnt[wave][d] + rank[k];
      if (lp < (uint32_t)kBlockKeys) {  // always (ranks are a permutation); a safeguard
        s_keys[lp] = key[k];
        if (kVals) s_vals[lp] = val[k];
      }
    }
  }
  __syncthreads();
  // runs of equal digits go to consecutive addresses
  const int count = (int)min((int64_t)kBlockKeys, (int64_t)n - blk0);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int lp = k * kSortThreads + tid;
    if (lp < count) {
      const K kk = s_keys[lp];
      const uint32_t dst = s_gbase[(uint32_t)(kk >> shift) & (kDigits - 1u)] + (uint32_t)lp;
      if (dst >= n) continue;  // never taken for a consistent table; keeps every write in bounds
      ((K*)o.keys)[dst] = kk;
      if (kFinal) {
        // the Gaussian id: the payload, or the low key bits when it rides in the key
        const uint32_t g = kVals ? s_vals[lp] : (uint32_t)(kk & (((K)1 << o.id_bits) - 1));
        o.vals[dst] = g;
        if (o.keys64 != nullptr)
          o.keys64[dst] = ((uint64_t)(kk >> o.id_bits) << 32) | (uint64_t)__float_as_uint(o.depth[g]);
      } else if (kVals) {
        o.vals[dst] = s_vals[lp];
      }
    }
  }
}

// ------------------------------------------------------------------ depth sort
// The depth sort (four 8-bit passes over n keys with ids) takes three
// kernels per pass: the per-block digit counts (the table hist[digit][block],
// row stride hstride), one workgroup per digit scanning its row (each
// block's exclusive offset within the digit, and the digit's total), then
// the scatter.  (Letting every scatter block add up its offsets from the
// raw table instead reads the whole table once per block, which grows with
// the square of the block count: 70-100 us per pass at 1.5M Gaussians.)
// The last pass writes the ids and gathers each Gaussian's rectangle and
// pair count into depth order instead of writing keys.
static_assert(kDepthBlockKeys == kSortThreads * kDepthItems && kDepthDigits == kSortThreads,
              "a depth pass block: one thread per digit");

static int64_t depth_blocks(int64_t n) { return ceil_div(n, (int64_t)kDepthBlockKeys); }
static int64_t depth_hstride(int64_t n) { return ceil_div(std::max<int64_t>(depth_blocks(n), 1), 4) * 4; }

struct DepthPassOut {
  uint32_t* keys;             // not last: keys and ids
  uint32_t* vals;
  uint32_t* ids_sorted;       // last: ids, rectangles and pair counts in depth order
  const int4* rect;
  const uint32_t* emit_cnt;
  int4* rect_sorted;
  uint32_t* cnt_sorted;
  int tiles_x, tiles_y;
};

template <bool kLast>
__global__ void __launch_bounds__(kSortThreads) depth_pass_kernel(const uint32_t* __restrict__ keys_in,
                                                                  const uint32_t* __restrict__ vals_in, uint32_t n,
                                                                  int shift, int hstride,
                                                                  const uint32_t* __restrict__ hoffs,
                                                                  const uint32_t* __restrict__ dtot, DepthPassOut o) {
  constexpr int kItems = kDepthItems, kBlockKeys = kDepthBlockKeys, kDigits = kDepthDigits;
  __shared__ uint32_t s_cnt[kSortWaves][kDigits];  // per-wave digit counts, then block-local offsets
  __shared__ uint32_t s_gbase[kDigits];            // global position of block-local position 0 of the digit
  __shared__ uint32_t s_keys[kBlockKeys];
  __shared__ uint32_t s_vals[kBlockKeys];
  __shared__ uint32_t s_red[kSortWaves];
  __shared__ uint64_t s_mask[kSortWaves][kDigits];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int i = tid; i < kSortWaves * kDigits; i += kSortThreads) (&s_cnt[0][0])[i] = 0;
  // keys of digit tid in the earlier blocks, and in all blocks
  const uint32_t before = hoffs[(int64_t)tid * hstride + blockIdx.x], all_d = dtot[tid];
  const int64_t blk0 = (int64_t)blockIdx.x * kBlockKeys;
  const int64_t wbase = blk0 + (int64_t)wave * kWave * kItems;
  uint32_t key[kItems], val[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = wbase + k * kWave + lane;
    key[k] = i < n ? keys_in[i] : 0u;
    val[k] = i < n ? vals_in[i] : 0u;
  }
  __syncthreads();
  const uint64_t below = lanes_below();
  uint32_t rank[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const bool valid = wbase + k * kWave + lane < n;
    const uint32_t d = (key[k] >> shift) & (kDigits - 1u);
    const uint64_t peers = digit_peers(d, valid, s_mask[wave]);
    const uint32_t r = (uint32_t)__popcll(peers & below);
    const uint32_t prior = valid ? s_cnt[wave][d] : 0u;
    rank[k] = prior + r;
    if (valid && r == 0) s_cnt[wave][d] = prior + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  uint32_t pre[kSortWaves];
  uint32_t tot = 0;
  for (int w = 0; w < kSortWaves; ++w) {
    pre[w] = tot;
    tot += s_cnt[w][tid];
  }
  uint32_t all;
  const uint32_t lstart = block_exclusive_scan<kSortThreads, uint32_t>(tot, s_red, &all);
  const uint32_t dstart = block_exclusive_scan<kSortThreads, uint32_t>(all_d, s_red, &all);
  for (int w = 0; w < kSortWaves; ++w) s_cnt[w][tid] = lstart + pre[w];
  s_gbase[tid] = dstart + before - lstart;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (wbase + k * kWave + lane < n) {
      const uint32_t d = (key[k] >> shift) & (kDigits - 1u);
      const uint32_t lp = s_cnt[wave][d] + rank[k];
      if (lp < (uint32_t)kBlockKeys) {  // always (ranks are a permutation); a safeguard
        s_keys[lp] = key[k];
        s_vals[lp] = val[k];
      }
    }
  }
  __syncthreads();
  const int count = (int)min((int64_t)kBlockKeys, (int64_t)n - blk0);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int lp = k * kSortThreads + tid;
    if (lp < count) {
      const uint32_t kk = s_keys[lp], g = s_vals[lp];
      const uint32_t dst = s_gbase[(kk >> shift) & (kDigits - 1u)] + (uint32_t)lp;
      if (dst >= n || g >= n) continue;  // never taken for a consistent table; keeps every access in bounds
      if (kLast) {
        o.ids_sorted[dst] = g;
        o.rect_sorted[dst] = clamp_rect(o.rect[g], o.tiles_x, o.tiles_y);
        if (o.emit_cnt != nullptr) o.cnt_sorted[dst] = o.emit_cnt[g];
      } else {
        o.keys[dst] = kk;
        o.vals[dst] = g;
      }
    }
  }
}

// One radix pass over n keys on bits [shift, shift + kBits); the histogram
// table is taken here unless the caller already wrote it (hist_ready).
template <typename K, bool kVals, bool kFinal, int kBits, int kItems>
static void radix_pass(const K* keys, const uint32_t* vals, uint32_t n, const uint32_t* n_dev, int shift,
                       uint32_t* hist, uint32_t* hoffs, uint32_t* dtot, const ScatterOut& o, hipStream_t s) {
  // n bounds the keys (the grid); n_dev, when given, holds the actual count on the device
  const int nblocks = (int)sort_blocks(n, kItems);
  hipLaunchKernelGGL((radix_hist_kernel<K, kBits, kItems>), dim3(nblocks), dim3(kSortThreads), 0, s, keys, n, n_dev,
                     shift, nblocks, hist);
  hipLaunchKernelGGL(digit_scan_kernel, dim3(1 << kBits), dim3(1024), 0, s, hist, nblocks, nblocks, hoffs, dtot, n_dev,
                     kSortThreads * kItems);
  hipLaunchKernelGGL((radix_scatter_kernel<K, kVals, kFinal, kBits, kItems>), dim3(nblocks), dim3(kSortThreads),
                     0, s, keys, vals, n, n_dev, shift, nblocks, hoffs, dtot, o);
}

template <typename K, bool kVals, bool kFinal, int kItems>
static void radix_pass_bits(int bits, const K* keys, const uint32_t* vals, uint32_t n, const uint32_t* n_dev,
                            int shift, uint32_t* hist, uint32_t* hoffs, uint32_t* dtot, const ScatterOut& o,
                            hipStream_t s) {
  switch (bits) {
#define TGS_PASS(B) \
  case B: radix_pass<K, kVals, kFinal, B, kItems>(keys, vals, n, n_dev, shift, hist, hoffs, dtot, o, s); break;
    TGS_PASS(1) TGS_PASS(2) TGS_PASS(3) TGS_PASS(4) TGS_PASS(5) TGS_PASS(6) TGS_PASS(7)
    default: radix_pass<K, kVals, kFinal, 8, kItems>(keys, vals, n, n_dev, shift, hist, hoffs, dtot, o, s);
#undef TGS_PASS
  }
}

// Passes of at most 8 bits over [lo, lo + bits), split evenly.
static int pass_count(int bits) { return (bits + 7) / 8; }
static int pass_bits(int bits, int p) {
  const int per = (bits + pass_count(bits) - 1) / pass_count(bits);
  return std::min(per, bits - p * per);
}

// ------------------------------------------------------------------ emit
// Per-wave LDS slice of a batch of up to 64 depth-ordered Gaussians.
struct RowBatch {
  int4 rect[kWave];
  uint32_t row0[kWave];  // exclusive prefix of the row counts in the batch
  RowEllipse ell[kWave];
  uint32_t id[kWave];
  int mark[kWave];
  // a round's row spans: first column, tile id of the row's column 0, id,
  // first output (exclusive prefix of the span lengths)
  int lo[kWave], hi[kWave];
  uint32_t trow[kWave], gid[kWave], ex[kWave];
};

constexpr int kEmitThreads = kWave;  // one wave per workgroup: __syncthreads is a wave barrier
constexpr int kEmitBatch = 32;       // Gaussians per wave: more waves, fewer rounds each (64 measured slower)
// The continuation's emission runs over every Gaussian past the prefix, few
// of which have pairs in the marked tiles: 64 per wave halves the waves
// that only find an empty batch.
// What a row emits: every kept column; its columns with a map entry >= 0,
// compacted by a ballot over the sub-round's outputs (a tile subset, where
// a good share of the columns is valid); or its flagged columns found by a
// walk over the row (the continuation, where few are).
constexpr int kEmitAll = 0, kEmitCompact = 1, kEmitWalk = 2;
template <int kMode>
constexpr int emit_batch() { return kMode == kEmitWalk ? kWave : kEmitBatch; }

// A wave per kEmitBatch depth-ordered Gaussians.  Their rectangle rows are
// flattened Gaussian by Gaussian and handed out 64 per round; a Gaussian
// whose first row falls in the round marks its slot and an inclusive
// max-scan carries each owner to the following slots, so a lane finds its
// Gaussian without a search.  Each lane takes its row's span; a wave scan of
// the span lengths places the row's keys after those of the rows before it,
// starting from the batch's first pair offset (pairs are emitted Gaussian by
// Gaussian, row by row, columns ascending).
//
// kEmitCompact, kEmitWalk: only the tiles whose map entry is >= 0 are
// emitted.  Compact hands out every kept column as above and writes the
// valid ones at the ballot prefix of the sub-round's valid outputs; Walk
// (the continuation lists) counts a row's flagged columns and hands out only
// those, each output lane walking the row's span to its column.
template <typename K, int kMode>
__global__ void __launch_bounds__(kEmitThreads) emit_kernel(
    const int4* __restrict__ rect_sorted, const uint32_t* __restrict__ off, const uint32_t* __restrict__ ids_sorted,
    int64_t n, const float4* __restrict__ splat, const int32_t* __restrict__ tile_slot, int tiles_x, uint32_t n_t,
    int id_bits, double tau, double lia, const uint32_t* __restrict__ total_dev, K* __restrict__ keys,
    uint32_t* __restrict__ pay) {
  const uint32_t total = *total_dev;  // pairs to emit (0 when they exceed the capacity)
  __shared__ RowBatch rb;
  const int lane = lane_id();
  constexpr int kBatch = emit_batch<kMode>();
  const int64_t b0 = (int64_t)blockIdx.x * kBatch;
  const int64_t j = b0 + lane;
  int4 r = make_int4(0, 0, 0, 0);
  uint32_t g = 0, rows = 0;
  if (total == 0) return;  // workgroup-uniform
  if (lane < kBatch && j < n && off[j + 1] > off[j]) {
    r = rect_sorted[j];
    g = ids_sorted[j];
    rows = (uint32_t)(r.w - r.y);
  }
  const uint32_t incl = wave_inclusive_scan_u32(rows);
  const uint32_t my_row0 = incl - rows;
  const uint32_t n_rows = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  if (n_rows == 0) return;  // wave-uniform: no Gaussian of the batch has pairs
  rb.rect[lane] = r;
  rb.row0[lane] = my_row0;
  rb.id[lane] = g;
  if (rows > 0) rb.ell[lane] = load_row_ellipse(splat, g, tau, lia);
  const uint32_t base = off[b0];  // pair offset of the batch's first Gaussian
  uint32_t written = 0;           // wave-uniform
  int carry = -1;
  for (uint32_t f0 = 0; f0 < n_rows; f0 += kWave) {
    rb.mark[lane] = -1;
    __syncthreads();
    if (rows > 0 && my_row0 >= f0 && my_row0 - f0 < (uint32_t)kWave) rb.mark[my_row0 - f0] = lane;
    __syncthreads();
    const int jl = max(wave_max_scan(rb.mark[lane]), carry);
    carry = __builtin_amdgcn_readlane(jl, kWave - 1);
    const uint32_t f = f0 + (uint32_t)lane;
    // jl >= 0 whenever f < n_rows: the first Gaussian with rows starts at row 0
    const bool in = f < n_rows && jl >= 0;
    int lo = 0, hi = -1, ty = 0;
    uint32_t gid = 0;
    if (in) {
      const int4 rj = rb.rect[jl];
      ty = rj.y + (int)(f - rb.row0[jl]);
      gid = rb.id[jl];
      row_span(rb.ell[jl], ty, rj.x, rj.z, lo, hi);
    }
    uint32_t c = (uint32_t)max(hi - lo + 1, 0);
    if (kMode == kEmitWalk && c > 0) {
      const int32_t* tr = tile_slot + (int64_t)ty * tiles_x;
      uint32_t cf = 0u;
      for (int tx = lo; tx <= hi; ++tx) cf += tr[tx] >= 0 ? 1u : 0u;
      c = cf;
    }
    const uint32_t ci = wave_inclusive_scan_u32(c);
    const uint32_t n_out = (uint32_t)__builtin_amdgcn_readlane((int)ci, kWave - 1);
    // the round's rows write n_out consecutive pairs from base + written; they
    // are handed out 64 per sub-round, lane q taking output q, so every store
    // covers consecutive addresses: the row owning an output is found like
    // the rows' owners above (its first output marked, a max-scan carries it)
    rb.lo[lane] = lo;
    rb.hi[lane] = hi;
    rb.trow[lane] = in ? (uint32_t)ty * (uint32_t)tiles_x : 0u;
    rb.gid[lane] = gid;
    rb.ex[lane] = ci - c;
    int ocarry = -1;
    for (uint32_t q0 = 0; q0 < n_out; q0 += kWave) {
      rb.mark[lane] = -1;
      __syncthreads();
      if (c > 0 && ci - c >= q0 && ci - c - q0 < (uint32_t)kWave) rb.mark[ci - c - q0] = lane;
      __syncthreads();
      const int own = max(wave_max_scan(rb.mark[lane]), ocarry);
      ocarry = __builtin_amdgcn_readlane(own, kWave - 1);
      const uint32_t q = q0 + (uint32_t)lane;
      // own >= 0 whenever q < n_out: output 0 belongs to the first row with pairs
      bool out = q < n_out && own >= 0;
      uint32_t tile = 0;
      if (out) {
        if (kMode == kEmitWalk) {  // the (q - ex)-th flagged column of the row (there are c of them)
          int left = (int)(q - rb.ex[own]), tx = rb.lo[own];
          const uint32_t tr = rb.trow[own];
          for (; tx < rb.hi[own]; ++tx) {
            if (tile_slot[tr + (uint32_t)tx] >= 0) {
              if (left == 0) break;
              --left;
            }
          }
          tile = tr + (uint32_t)tx;
        } else {
          tile = rb.trow[own] + (uint32_t)(rb.lo[own] + (int)(q - rb.ex[own]));
        }
      }
      uint32_t pos = base + written + q;
      if (kMode == kEmitCompact) {
        out = out && tile_slot[tile] >= 0;
        const uint64_t vb = __ballot(out);
        pos = base + written +
              __builtin_amdgcn_mbcnt_hi((uint32_t)(vb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)vb, 0u));
        written += (uint32_t)__popcll(vb);  // wave-uniform
      }
      if (out && pos < total) {  // pos < total always holds; the bound is a safeguard
        if (pay != nullptr) {  // the id as a separate payload, the key is the tile alone
          keys[pos] = (K)tile;
          pay[pos] = rb.gid[own];
        } else {
          keys[pos] = ((K)tile << id_bits) | (K)rb.gid[own];
        }
      }
      __syncthreads();  // the sub-round's mark reads before the next one's writes
    }
    if (kMode != kEmitCompact) written += n_out;
    __syncthreads();  // the round's mark reads before the next round's writes
  }
}

// ------------------------------------------------------------------ workspace
struct SortWs {
  unsigned long long* scalars;  // [2][TGS_COUNTER_SLOTS] partial totals: valid pairs, pairs
  uint32_t* dhist[4];           // [256][hstride] per-block digit counts of each depth pass
  uint32_t* dhoffs;             // [256][hstride] their exclusive prefix per digit (the pass being run)
  uint32_t* ddtot;              // [256] digit totals of the pass being run
  uint32_t* zeroed;             // scalars and dhist: one region, cleared at the start
  int64_t zeroed_words;         // its size in 32-bit words
  int hstride;                  // row stride of the depth tables
  uint32_t* emit_cnt;           // [n] pairs each Gaussian emits
  int4* rect_sorted;            // [n] rectangles in depth order
  uint32_t* cnt_sorted;         // [n] pair counts in depth order
  uint32_t* ids_sorted;         // [n] Gaussian ids in depth order
  uint32_t* off;                // [n + 1] exclusive prefix of the counts: pair offsets
  uint32_t* dkeys[2];           // [n] depth keys (ping-pong)
  uint32_t* dvals[2];           // [n] ids
  uint32_t* partials;           // scan block sums, digit totals
  uint32_t* hist;               // [256 * max_blocks]
  uint32_t* hoffs;              // [256 * max_blocks]
  void* pkeys[2];               // [capacity] x 8 bytes each: pair keys (u32), or u16/u32 tile keys then u32 ids
  int64_t cap;                  // pairs each ping-pong buffer holds
  unsigned long long* counts;   // [2] pairs in valid tiles, all pairs (the call's device result)
  uint32_t* eff_total;          // all pairs when they fit the capacity, else 0 (what the pair sort sorts)
  size_t bytes;
};

static SortWs layout(void* ws, int64_t n, int64_t capacity) {
  const int64_t cap = std::max<int64_t>(capacity, 1), nn = std::max<int64_t>(n, 1);
  const int64_t m = std::max(cap, nn);
  // blocks of any sort of up to m keys: 1024-key blocks below 2^20 keys, 4096-key blocks above
  const int64_t max_blocks = std::max<int64_t>(1024, sort_blocks(m, kPairItems)) + 1;
  const int64_t hist_n = 256 * max_blocks;
  const int64_t part_n = std::max<int64_t>(256, scan_partials(nn + 1)) + 1;
  size_t o = 0;
  char* b = (char*)ws;
  auto take = [&](size_t bytes) {
    char* p = b ? b + o : nullptr;
    o += align_up(bytes, 256);
    return (void*)p;
  };
  SortWs w;
  w.hstride = (int)depth_hstride(nn);
  const int64_t table_words = (int64_t)kDepthDigits * w.hstride;
  const int64_t scalar_words = 3 * 2 * TGS_COUNTER_SLOTS;  // three rows of 64-bit slots
  w.zeroed_words = scalar_words + 4 * table_words;
  w.zeroed = (uint32_t*)take(sizeof(uint32_t) * w.zeroed_words);
  w.scalars = (unsigned long long*)w.zeroed;
  for (int k = 0; k < 4; ++k) w.dhist[k] = w.zeroed ? w.zeroed + scalar_words + k * table_words : nullptr;
  w.counts = (unsigned long long*)take(4 * sizeof(unsigned long long));
  w.eff_total = (uint32_t*)(w.counts ? w.counts + 2 : nullptr);
  w.dhoffs = (uint32_t*)take(sizeof(uint32_t) * table_words);
  w.ddtot = (uint32_t*)take(sizeof(uint32_t) * kDepthDigits);
  w.emit_cnt = (uint32_t*)take(sizeof(uint32_t) * nn);
  w.rect_sorted = (int4*)take(sizeof(int4) * nn);
  w.cnt_sorted = (uint32_t*)take(sizeof(uint32_t) * nn);
  w.ids_sorted = (uint32_t*)take(sizeof(uint32_t) * nn);
  w.off = (uint32_t*)take(sizeof(uint32_t) * (nn + 1));
  for (int k = 0; k < 2; ++k) {
    w.dkeys[k] = (uint32_t*)take(sizeof(uint32_t) * nn);
    w.dvals[k] = (uint32_t*)take(sizeof(uint32_t) * nn);
  }
  w.partials = (uint32_t*)take(sizeof(uint32_t) * part_n);
  w.hist = (uint32_t*)take(sizeof(uint32_t) * hist_n);
  w.hoffs = (uint32_t*)take(sizeof(uint32_t) * hist_n);
  w.cap = cap;
  // 8 bytes per pair: a u32 key, or (16-byte aligned halves) a u16/u32 tile key and a u32 id
  for (int k = 0; k < 2; ++k) w.pkeys[k] = take(align_up(sizeof(uint32_t) * cap, 256) + sizeof(uint32_t) * cap);
  w.bytes = o;
  return w;
}

static int bits_for(uint64_t max_value) {  // bits needed to represent 0..max_value
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) ++b;
  return b;
}

// Stable LSD sort of the n depth keys with their ids (the count kernel has
// filled the first pass's table); the last pass writes ids, rectangles and
// pair counts in depth order.
static void sort_depth(const SortWs& w, uint32_t n, const int4* rect, int tiles_x, int tiles_y, hipStream_t s,
                       bool gather_counts = true) {
  const unsigned nb = (unsigned)depth_blocks(n);
  int cur = 0;
  for (int p = 0; p < 4; ++p) {
    // rows of hstride entries (the padding stays zero from the start-of-call fill)
    hipLaunchKernelGGL((radix_hist_kernel<uint32_t, 8, kDepthItems>), dim3(nb), dim3(kSortThreads), 0, s,
                       w.dkeys[cur], n, (const uint32_t*)nullptr, 8 * p, w.hstride, w.dhist[p]);
    hipLaunchKernelGGL(digit_scan_kernel, dim3(kDepthDigits), dim3(1024), 0, s, w.dhist[p], (int)nb, w.hstride,
                       w.dhoffs, w.ddtot, (const uint32_t*)nullptr, kDepthBlockKeys);
    DepthPassOut o{};
    if (p < 3) {
      o.keys = w.dkeys[cur ^ 1];
      o.vals = w.dvals[cur ^ 1];
      hipLaunchKernelGGL(depth_pass_kernel<false>, dim3(nb), dim3(kSortThreads), 0, s, w.dkeys[cur], w.dvals[cur],
                         n, 8 * p, w.hstride, w.dhoffs, w.ddtot, o);
    } else {
      o.ids_sorted = w.ids_sorted;
      o.rect = rect;
      o.emit_cnt = gather_counts ? w.emit_cnt : nullptr;
      o.rect_sorted = w.rect_sorted;
      o.cnt_sorted = w.cnt_sorted;
      o.tiles_x = tiles_x;
      o.tiles_y = tiles_y;
      hipLaunchKernelGGL(depth_pass_kernel<true>, dim3(nb), dim3(kSortThreads), 0, s, w.dkeys[cur], w.dvals[cur],
                         n, 8 * p, w.hstride, w.dhoffs, w.ddtot, o);
    }
    cur ^= 1;
  }
}

// kPay false: the key is (tile << id_bits) | id (32 bits when they fit).
// kPay true: the key is the tile alone (16 bits) and the id travels as a
// 32-bit payload; used when tile and id bits together exceed 32, where a
// 64-bit key would move 16 bytes per pair and pass instead of 12.
// bound: the capacity (host), sizing every grid; the pair count itself is
// read on the device (w.eff_total), so nothing here waits for the host.
template <typename K, bool kPay, int kMode = kEmitAll>
static void sort_pairs(const SortWs& w, const uint32_t* ids, int64_t n, uint32_t bound, const float4* splat,
                       const int32_t* tile_slot, int tiles_x, uint32_t n_t, int id_bits, int tbits, double tau, double lia,
                       const float* depth, uint32_t* vals, uint64_t* keys64, uint32_t* ranges, hipStream_t s) {
  // each ping-pong buffer (8 bytes per pair of capacity) holds the keys and, after them, the payload
  K* kb[2] = {(K*)w.pkeys[0], (K*)w.pkeys[1]};
  uint32_t* pb[2] = {nullptr, nullptr};
  if (kPay)
    for (int k = 0; k < 2; ++k) pb[k] = (uint32_t*)((char*)w.pkeys[k] + align_up(sizeof(K) * (size_t)w.cap, 256));
  const int key_id_bits = kPay ? 0 : id_bits;
  hipLaunchKernelGGL((emit_kernel<K, kMode>), dim3((unsigned)std::max<int64_t>(ceil_div(n, emit_batch<kMode>()), 1)),
                     dim3(kEmitThreads), 0, s,
                     w.rect_sorted, w.off, ids, n, splat, tile_slot, tiles_x, n_t, key_id_bits, tau, lia, w.eff_total,
                     kb[0], pb[0]);
  const int passes = pass_count(tbits);
  int cur = 0, shift = key_id_bits;
  for (int p = 0; p < passes; ++p) {
    const int b = pass_bits(tbits, p);
    // non-final passes carry the payload to the other buffer; the last writes the ids
    const ScatterOut o = {kb[cur ^ 1], p == passes - 1 ? vals : pb[cur ^ 1], key_id_bits, depth, keys64};
    if (p == passes - 1)
      radix_pass_bits<K, kPay, true, kPairItems>(b, kb[cur], pb[cur], bound, w.eff_total, shift, w.hist, w.hoffs,
                                                 w.partials, o, s);
    else
      radix_pass_bits<K, kPay, false, kPairItems>(b, kb[cur], pb[cur], bound, w.eff_total, shift, w.hist, w.hoffs,
                                                  w.partials, o, s);
    cur ^= 1;
    shift += b;
  }
  hipLaunchKernelGGL((ranges_kernel<K>), dim3((unsigned)std::max<int64_t>(ceil_div(bound, kRangeBlock), 1)),
                     dim3(256), 0, s, kb[cur], bound, w.eff_total, key_id_bits, n_t, (uint2*)ranges);
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_bin_sort_workspace_size(int64_t n, int64_t capacity, int32_t n_tiles) {
  (void)n_tiles;
  if (n < 0 || capacity < 0) return 0;
  return layout(nullptr, n, capacity).bytes;
}

// Everything after the argument checks: queued on the stream, no host wait.
// prefix >= 0: the lists hold the pairs of the first `prefix` Gaussians in
// (depth, id) order only (every Gaussian when prefix >= n), and the counts
// are the prefix call's (w.counts[3] = the whole lists' pairs); -1: whole
// lists with the plain counts.
static int32_t bin_sort_queue(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                              const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y, float alpha_min,
                              uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* ranges, uint8_t* touched,
                              const SortWs& w, hipStream_t s, const char* who, int64_t prefix = -1) {
  const uint32_t n_t = (uint32_t)tiles_x * (uint32_t)tiles_y;
  // 2 ln(1/alpha_min) with a 0.1 % margin, rounded up to a multiple of 1/64
  const double lia = std::log(1.0 / (double)alpha_min);
  const double tau = std::ceil(128.0 * lia * 1.001) / 64.0;
  // empty ranges and the zeroed workspace region (counters, table padding)
  hipLaunchKernelGGL(zero2_u32_kernel, dim3((unsigned)ceil_div(2 * (int64_t)n_t + w.zeroed_words, 256)), dim3(256),
                     0, s, ranges, 2 * (int64_t)n_t, w.zeroed, w.zeroed_words);
  if (n == 0) {  // zero counts and pair total
    hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(64), 0, s, w.scalars, capacity, w.counts, w.eff_total);
    return hip_status(who);
  }
  const bool pre = prefix >= 0;
  const int64_t m = pre ? std::min(prefix, n) : n;
  if (!pre) {
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)ceil_div(n, kCountBatch)), dim3(kWave), 0, s,
                       (const int4*)rect, (const uint32_t*)nullptr, (const float4*)splat, depth, n, tile_slot,
                       tiles_x, tiles_y, tau, lia, w.dkeys[0], w.dvals[0], w.emit_cnt, touched, w.scalars);
    hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(64), 0, s, w.scalars, capacity, w.counts, w.eff_total);
    // (depth, id) order; Gaussians without pairs last
    sort_depth(w, (uint32_t)n, (const int4*)rect, tiles_x, tiles_y, s);
    // pair offsets (they wrap only past 2^32 pairs, where the capacity check has already set the total to 0)
    exclusive_scan<uint32_t>(w.cnt_sorted, w.off, n, w.partials, s);
  } else {
    // depth-prefix lists: (depth, id) order of the Gaussians with a
    // rectangle (the others last), then the counts of the first m only
    hipLaunchKernelGGL(key_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, (const int4*)rect, depth, n,
                       tiles_x, tiles_y, w.dkeys[0], w.dvals[0], w.scalars);
    sort_depth(w, (uint32_t)n, (const int4*)rect, tiles_x, tiles_y, s, false);
    if (m > 0)
      hipLaunchKernelGGL(count_kernel, dim3((unsigned)ceil_div(m, kCountBatch)), dim3(kWave), 0, s,
                         (const int4*)w.rect_sorted, (const uint32_t*)w.ids_sorted, (const float4*)splat, depth, m,
                         tile_slot, tiles_x, tiles_y, tau, lia, (uint32_t*)nullptr, (uint32_t*)nullptr,
                         w.cnt_sorted, touched, w.scalars);
    hipLaunchKernelGGL(prefix_totals_kernel, dim3(1), dim3(64), 0, s, w.scalars, m, capacity, w.counts,
                       w.eff_total);
    exclusive_scan<uint32_t>(w.cnt_sorted, w.off, m, w.partials, s);
  }
  if (capacity == 0) return hip_status(who);
  const uint32_t bound = (uint32_t)capacity;
  const int id_bits = std::max(1, bits_for((uint64_t)n - 1));
  const int tbits = bits_for(n_t);
  // with a tile subset only its tiles are emitted
  auto sort_all = [&](auto filter) {
    constexpr int kF = decltype(filter)::value ? kEmitCompact : kEmitAll;
    if (id_bits + tbits <= 32)
      sort_pairs<uint32_t, false, kF>(w, w.ids_sorted, m, bound, (const float4*)splat, tile_slot, tiles_x, n_t,
                                      id_bits, tbits, tau, lia, depth, vals, keys, ranges, s);
    else if (tbits <= 16)
      sort_pairs<uint16_t, true, kF>(w, w.ids_sorted, m, bound, (const float4*)splat, tile_slot, tiles_x, n_t,
                                     id_bits, tbits, tau, lia, depth, vals, keys, ranges, s);
    else
      sort_pairs<uint32_t, true, kF>(w, w.ids_sorted, m, bound, (const float4*)splat, tile_slot, tiles_x, n_t,
                                     id_bits, tbits, tau, lia, depth, vals, keys, ranges, s);
  };
  if (tile_slot != nullptr)
    sort_all(std::true_type{});
  else
    sort_all(std::false_type{});
  return hip_status(who);
}

// The continuation of depth-prefix lists: the pairs of the Gaussians from
// depth rank `prefix` on in the flagged tiles, from the depth order that
// the prefix call left in its workspace w1, sorted by tile (each tile's
// list in depth order) with the scratch and pair buffers of w2.
static int32_t continue_queue(const float* splat, int64_t n, const int32_t* flag_slot, const uint32_t* n_flagged,
                              int32_t tiles_x, int32_t tiles_y, float alpha_min, int64_t prefix, uint32_t* vals2,
                              int64_t capacity2, uint32_t* ranges2, const SortWs& w1, const SortWs& w2,
                              hipStream_t s, const char* who) {
  const uint32_t n_t = (uint32_t)tiles_x * (uint32_t)tiles_y;
  const double lia = std::log(1.0 / (double)alpha_min);
  const double tau = std::ceil(128.0 * lia * 1.001) / 64.0;
  hipLaunchKernelGGL(zero2_u32_kernel, dim3((unsigned)ceil_div(2 * (int64_t)n_t + w2.zeroed_words, 256)), dim3(256),
                     0, s, ranges2, 2 * (int64_t)n_t, w2.zeroed, w2.zeroed_words);
  const int64_t m = n - std::min(prefix, n);
  // the flagged tiles' summed-area table (or, for larger grids, per-row
  // running counts) in the pair-sort histogram (free until the sort)
  const int64_t sat_words = (int64_t)(tiles_x + 1) * (tiles_y + 1);
  const int64_t rc_words = (int64_t)(tiles_x + 1) * tiles_y;
  uint32_t* sat = sat_words <= kSatWords ? w2.hist : nullptr;
  uint32_t* rowc = sat == nullptr && rc_words <= 256 * 1024 ? w2.hist : nullptr;
  if (m > 0 && sat != nullptr)
    hipLaunchKernelGGL(flag_sat_kernel, dim3(1), dim3(1024), 0, s, flag_slot, tiles_x, tiles_y, n_flagged, sat);
  if (m > 0 && rowc != nullptr)
    hipLaunchKernelGGL(flag_rows_kernel, dim3((unsigned)tiles_y), dim3(kWave), 0, s, flag_slot, tiles_x, n_flagged,
                       rowc);
  if (m > 0)
    hipLaunchKernelGGL(count_cont_kernel, dim3((unsigned)ceil_div(m, kCountBatch)), dim3(kWave), 0, s,
                       w1.rect_sorted + prefix, w1.ids_sorted + prefix, (const uint32_t*)nullptr, m,
                       (const float4*)splat, flag_slot, n_flagged, (const uint32_t*)rowc, (const uint32_t*)sat,
                       tiles_x, tiles_y, tau, lia, w2.emit_cnt, w2.scalars);
  hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(64), 0, s, w2.scalars, capacity2, w2.counts, w2.eff_total);
  if (m == 0 || capacity2 == 0) return hip_status(who);
  exclusive_scan<uint32_t>(w2.emit_cnt, w2.off, m, w2.partials, s);
  SortWs wc = w2;
  wc.rect_sorted = w1.rect_sorted + prefix;
  const uint32_t bound = (uint32_t)capacity2;
  const int id_bits = std::max(1, bits_for((uint64_t)n - 1));
  const int tbits = bits_for(n_t);
  if (id_bits + tbits <= 32)
    sort_pairs<uint32_t, false, kEmitWalk>(wc, w1.ids_sorted + prefix, m, bound, (const float4*)splat, flag_slot, tiles_x,
                                      n_t, id_bits, tbits, tau, lia, nullptr, vals2, nullptr, ranges2, s);
  else if (tbits <= 16)
    sort_pairs<uint16_t, true, kEmitWalk>(wc, w1.ids_sorted + prefix, m, bound, (const float4*)splat, flag_slot, tiles_x,
                                     n_t, id_bits, tbits, tau, lia, nullptr, vals2, nullptr, ranges2, s);
  else
    sort_pairs<uint32_t, true, kEmitWalk>(wc, w1.ids_sorted + prefix, m, bound, (const float4*)splat, flag_slot, tiles_x,
                                     n_t, id_bits, tbits, tau, lia, nullptr, vals2, nullptr, ranges2, s);
  return hip_status(who);
}

static int32_t bin_sort_check(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                              int32_t tiles_x, int32_t tiles_y, float alpha_min, uint32_t* vals, int64_t capacity,
                              uint32_t* ranges, void* ws, size_t ws_bytes, const SortWs& w, const char* who) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "%s: n out of range", who);
  TGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && (int64_t)tiles_x * tiles_y < (1ll << 30), "%s: bad tile grid", who);
  TGS_REQUIRE(capacity >= 0 && capacity < (1ll << 32), "%s: capacity out of range", who);
  TGS_REQUIRE(alpha_min > 0.f && alpha_min < 1.f, "%s: alpha_min %g not in (0, 1)", who, (double)alpha_min);
  TGS_REQUIRE(vals && ranges && ws, "%s: null pointer", who);  // keys may be null
  TGS_REQUIRE(n == 0 || (rect && splat && depth), "%s: null rect/splat/depth", who);
  TGS_REQUIRE(((uintptr_t)rect & 15) == 0 && ((uintptr_t)splat & 15) == 0 && ((uintptr_t)ws & 15) == 0,
              "%s: rect, splat and ws must be 16-byte aligned", who);
  TGS_REQUIRE(ws_bytes >= w.bytes, "%s: workspace %zu bytes < %zu", who, ws_bytes, w.bytes);
  return TGS_OK;
}

extern "C" int32_t tgs_bin_sort_async(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                                      const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y, float alpha_min,
                                      uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* ranges,
                                      uint8_t* touched, int64_t* counts, void* ws, size_t ws_bytes, void* stream) {
  const SortWs w = layout(ws, n, capacity);
  if (int32_t e = bin_sort_check(rect, splat, depth, n, tiles_x, tiles_y, alpha_min, vals, capacity, ranges, ws,
                                 ws_bytes, w, "tgs_bin_sort_async"))
    return e;
  TGS_REQUIRE(counts != nullptr && ((uintptr_t)counts & 7) == 0,
              "tgs_bin_sort_async: counts must be an 8-byte aligned device pointer");
  hipStream_t s = as_stream(stream);
  if (int32_t e = bin_sort_queue(rect, splat, depth, n, tile_slot, tiles_x, tiles_y, alpha_min, keys, vals, capacity,
                                 ranges, touched, w, s, "tgs_bin_sort_async"))
    return e;
  hipLaunchKernelGGL(copy_counts_kernel, dim3(1), dim3(64), 0, s, (const unsigned long long*)w.counts,
                     (unsigned long long*)counts);
  return hip_status("tgs_bin_sort_async");
}

extern "C" int32_t tgs_bin_sort_prefix_async(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                                             const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y,
                                             float alpha_min, int64_t prefix, uint64_t* keys, uint32_t* vals,
                                             int64_t capacity, uint32_t* ranges, uint8_t* touched, int64_t* counts,
                                             void* ws, size_t ws_bytes, void* stream) {
  const SortWs w = layout(ws, n, capacity);
  if (int32_t e = bin_sort_check(rect, splat, depth, n, tiles_x, tiles_y, alpha_min, vals, capacity, ranges, ws,
                                 ws_bytes, w, "tgs_bin_sort_prefix_async"))
    return e;
  TGS_REQUIRE(prefix >= 0, "tgs_bin_sort_prefix_async: negative prefix");
  TGS_REQUIRE(counts != nullptr && ((uintptr_t)counts & 7) == 0,
              "tgs_bin_sort_prefix_async: counts must be an 8-byte aligned device pointer");
  hipStream_t s = as_stream(stream);
  if (int32_t e = bin_sort_queue(rect, splat, depth, n, tile_slot, tiles_x, tiles_y, alpha_min, keys, vals, capacity,
                                 ranges, touched, w, s, "tgs_bin_sort_prefix_async", prefix))
    return e;
  hipLaunchKernelGGL(copy_counts3_kernel, dim3(1), dim3(64), 0, s, (const unsigned long long*)w.counts,
                     (unsigned long long*)counts);
  return hip_status("tgs_bin_sort_prefix_async");
}

extern "C" int32_t tgs_bin_sort_continue_async(const float* splat, int64_t n, const int32_t* flag_slot,
                                               const uint32_t* n_flagged, int32_t tiles_x, int32_t tiles_y,
                                               float alpha_min, int64_t prefix,
                                               int64_t capacity, const void* ws, size_t ws_bytes, uint32_t* vals2,
                                               int64_t capacity2, uint32_t* ranges2, int64_t* counts2, void* ws2,
                                               size_t ws2_bytes, void* stream) {
  const char* who = "tgs_bin_sort_continue_async";
  TGS_REQUIRE(n >= 0 && n < (1ll << 31) && prefix >= 0, "%s: n or prefix out of range", who);
  TGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && (int64_t)tiles_x * tiles_y < (1ll << 30), "%s: bad tile grid", who);
  TGS_REQUIRE(capacity >= 0 && capacity2 >= 0 && capacity2 < (1ll << 32), "%s: capacity out of range", who);
  TGS_REQUIRE(alpha_min > 0.f && alpha_min < 1.f, "%s: alpha_min %g not in (0, 1)", who, (double)alpha_min);
  TGS_REQUIRE(splat && flag_slot && ws && vals2 && ranges2 && counts2 && ws2, "%s: null pointer", who);
  TGS_REQUIRE(((uintptr_t)splat & 15) == 0 && ((uintptr_t)ws & 15) == 0 && ((uintptr_t)ws2 & 15) == 0 &&
                  ((uintptr_t)counts2 & 7) == 0,
              "%s: splat, ws and ws2 must be 16-byte, counts2 8-byte aligned", who);
  const SortWs w1 = layout((void*)ws, n, capacity);
  const SortWs w2 = layout(ws2, n, capacity2);
  TGS_REQUIRE(ws_bytes >= w1.bytes && ws2_bytes >= w2.bytes, "%s: workspace too small", who);
  hipStream_t s = as_stream(stream);
  if (int32_t e = continue_queue(splat, n, flag_slot, n_flagged, tiles_x, tiles_y, alpha_min, prefix, vals2, capacity2,
                                 ranges2, w1, w2, s, who))
    return e;
  hipLaunchKernelGGL(copy_counts_kernel, dim3(1), dim3(64), 0, s, (const unsigned long long*)w2.counts,
                     (unsigned long long*)counts2);
  return hip_status(who);
}

extern "C" int32_t tgs_bin_sort(const int32_t* rect, const float* splat, const float* depth, int64_t n,
                                const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y, float alpha_min,
                                uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* ranges,
                                uint8_t* touched, int64_t* n_pairs, void* ws, size_t ws_bytes,
                                void* stream) {
  const SortWs w = layout(ws, n, capacity);
  if (int32_t e = bin_sort_check(rect, splat, depth, n, tiles_x, tiles_y, alpha_min, vals, capacity, ranges, ws,
                                 ws_bytes, w, "tgs_bin_sort"))
    return e;
  TGS_REQUIRE(n_pairs != nullptr, "tgs_bin_sort: null n_pairs");
  hipStream_t s = as_stream(stream);
  if (int32_t e = bin_sort_queue(rect, splat, depth, n, tile_slot, tiles_x, tiles_y, alpha_min, keys, vals, capacity,
                                 ranges, touched, w, s, "tgs_bin_sort"))
    return e;
  // the one synchronisation: the two counts, read back when the stream has run the call
  unsigned long long host[2] = {0, 0};
  if (hipMemcpyAsync(host, w.counts, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return hip_status("tgs_bin_sort: count readback");
  if ((int64_t)host[1] > capacity) {
    *n_pairs = (int64_t)host[1];
    set_error("tgs_bin_sort: %llu pairs exceed capacity %lld", host[1], (long long)capacity);
    return TGS_ERR_CAPACITY;
  }
  *n_pairs = (int64_t)host[0];
  return hip_status("tgs_bin_sort");
}
