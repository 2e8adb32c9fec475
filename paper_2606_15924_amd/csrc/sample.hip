// Tile-wise error/age pixel sampling (Sec. 3.5).
//
// Three kernels per view:
//   tile_weights  one wave per tile: integer tile weight (sum of E * 2^24), only
//                 when tiles are drawn in proportion to error;
//   tile_select   one workgroup: the tile draws (or every tile), the per-tile
//                 sample counts, their prefix offsets and the tile -> slot map;
//   tile_pixels   one wave per selected tile: N_hard sequential error-weighted
//                 draws without replacement, TopK age, uniform mixed draws.
// All decisions are integer: weights are exact integers (every finite
// non-negative half times 2^24 is one), a draw r = floor(u * W / 2^64) uses
// the high half of a 64 x 64-bit product, and the pick is the first pixel
// (ascending local index) whose running weight exceeds r.  Each lane owns four
// consecutive local indices, so lane order is index order and a wave prefix
// sum locates a draw.
#include <mutex>

#include "scan.h"

namespace tgs {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// SplitMix64 finaliser (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t absorb(uint64_t h, uint64_t field) {
  return mix64(h + kGamma * (field + 1ull));
}

// Key of the (seed, step, view, tile) stream; a draw is absorb(key, slot).
__device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t step, uint64_t view,
                                               uint64_t tile) {
  return absorb(absorb(absorb(seed, step), view), tile);
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// E * 2^24 for a half bit pattern; negative, infinite and NaN values weigh 0.
__device__ __forceinline__ uint64_t half_weight(uint16_t h) {
  const uint32_t sign = h >> 15, ex = (h >> 10) & 0x1f, man = h & 0x3ff;
  if (sign || ex == 0x1f) return 0;
  if (ex == 0) return man;
  return (uint64_t)(1024u + man) << (ex - 1);
}

// Lane l's value of a 64-bit register (l uniform).
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int tile_valid_w(int tx, int W) { return min(kTile, W - tx * kTile); }
__device__ __forceinline__ int tile_valid_h(int ty, int H) { return min(kTile, H - ty * kTile); }

// ------------------------------------------------------------------ tile weights
__global__ void __launch_bounds__(64) tile_weights_kernel(const uint16_t* __restrict__ E, int H,
                                                          int W, int tiles_x, int n_t,
                                                          uint64_t* __restrict__ tw) {
  const int t = blockIdx.x;
  if (t >= n_t) return;
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int lane = threadIdx.x;
  uint64_t s = 0;
  for (int k = 0; k < 4; ++k) {
    const int loc = lane * 4 + k;
    const int x = tx * kTile + (loc & 15), y = ty * kTile + (loc >> 4);
    if (x < W && y < H) s += half_weight(E[(int64_t)y * W + x]);
  }
  // wave sum of u64 as two 32-bit halves is not exact; use the inclusive scan
  s = wave_inclusive_scan_u64(s);
  if (lane == 63) tw[t] = s;
}

// Tile weights from predicted mean tile errors: floor(clamp(p, 0, 65504) *
// in-image pixels * 2^24), the units of the error-map sums; exact in FP64 (a
// float times a count up to 256 times a power of two).
__global__ void __launch_bounds__(256) tile_pred_weights_kernel(const float* __restrict__ pred, int H, int W,
                                                               int tiles_x, int n_t, uint64_t* __restrict__ tw) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n_t) return;
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int nx = min(kTile, W - tx * kTile), ny = min(kTile, H - ty * kTile);
  const float p = pred[t];
  const double q = p > 0.f ? (double)fminf(p, 65504.f) : 0.0;  // NaN and negatives give 0
  tw[t] = (uint64_t)floor(q * (double)(nx * ny) * 16777216.0);
}

// ------------------------------------------------------------------ tile select
// One workgroup.  The sequential tile draws (only when a subset of tiles is
// drawn) run on the first wave; then the whole workgroup lists the chosen
// tiles in ascending order with their sample counts and prefix offsets.
constexpr int kSelectThreads = 1024;
constexpr uint64_t kChosenBit = 1ull << 63;  // tile weights stay below 2^57 (256 pixels x 2^24 x 65504)
constexpr int kSelectMaxE = 5;               // tiles per lane in a chunk pass: n_t up to 20480 in LDS

// The draws on LDS (first wave only).  s_p[t] holds, for tile t in chunk
// [l C, (l + 1) C), the remaining weight of the chunk's tiles up to and
// including t (a chunk-local inclusive prefix), with bit 63 set once t is
// chosen; s_lsum[l] the chunk's total.  Lane l keeps its chunk's remaining
// weight and the inclusive prefix of those over the lanes up to date.  A
// draw r falls in the first lane o whose inclusive sum exceeds r; in o's
// chunk the tile is the first whose prefix exceeds r minus the chunks
// before, found by one ballot over the lanes (lane k holds the prefixes of
// tiles k E .. k E + E - 1, E = ceil(C / 64)) and a walk over E registers.
// Removing the tile lowers the prefixes from it to the chunk's end, written
// back from the registers that were read.  That is the first tile in
// ascending order whose running weight exceeds r, as the sequential
// definition has it, so the draws equal the plain loop's.  When every
// remaining weight is zero (all prefixes are then zero) the draw is uniform
// over the remaining tiles and is found on counts of the unchosen tiles.
// The draws' 64-bit counter values are hashed 64 at a time, one per lane.
template <int kE>
__device__ void select_tiles_lds(uint64_t* s_p, const uint64_t* s_lsum, int n_t, int n_sel, uint64_t key) {
  const int lane = lane_id();
  const int C = (n_t + kWave - 1) / kWave;
  const int c0 = min(n_t, lane * C), c1 = min(n_t, c0 + C);
  uint64_t lsum = s_lsum[lane];
  int lrem = c1 - c0;
  uint64_t incl = wave_inclusive_scan_u64_dpp(lsum);
  int icnt = wave_inclusive_scan_i_dpp(lrem);
  uint64_t ub = 0;
  for (int j = 0; j < n_sel; ++j) {
    if ((j & (kWave - 1)) == 0) ub = absorb(key, (uint64_t)(j + lane));
    const uint64_t u = readlane_u64(ub, j & (kWave - 1));
    const uint64_t total = readlane_u64(incl, kWave - 1);
    if (total > 0) {
      const uint64_t r = mulhi64(u, total);
      const uint64_t above = __ballot(incl > r);
      if (above == 0ull) break;  // never taken: the running sums are exact
      const int o = __ffsll((unsigned long long)above) - 1;
      const uint64_t rp = r - readlane_u64(incl - lsum, o);
      const int oc0 = o * C, olen = min(n_t, oc0 + C) - oc0;
      // this lane's prefixes (positions past the chunk read its last one,
      // which exceeds rp, so they never come before the true crossing)
      uint64_t raw[kE], P[kE];
#pragma unroll
      for (int e = 0; e < kE; ++e) {
        raw[e] = s_p[oc0 + min(lane * kE + e, olen - 1)];
        P[e] = raw[e] & ~kChosenBit;
      }
      // lane of the crossing (the chunk's last prefix exceeds rp, so some
      // lane's does; no branch here, so the loads above issue together)
      const int h = max(0, __ffsll((unsigned long long)__ballot(P[kE - 1] > rp)) - 1);
      const uint64_t prev_last = dpp_u64<kDppWaveShr1>(P[kE - 1]);  // lane 0 reads 0: the chunk starts at 0
      int pe = kE - 1;
      uint64_t wv = P[kE - 1] - (kE > 1 ? P[kE > 1 ? kE - 2 : 0] : prev_last);
#pragma unroll
      for (int e = kE - 2; e >= 0; --e) {
        if (P[e] > rp) {
          pe = e;
          wv = P[e] - (e > 0 ? P[e > 0 ? e - 1 : 0] : prev_last);
        }
      }
      const int pl = h * kE + __builtin_amdgcn_readlane(pe, h);  // chunk-local position of the pick
      const uint64_t w = readlane_u64(wv, h);
#pragma unroll
      for (int e = 0; e < kE; ++e) {
        const int idx = lane * kE + e;
        if (idx >= pl && idx < olen) s_p[oc0 + idx] = (raw[e] - w) | (idx == pl ? kChosenBit : 0ull);
      }
      if (lane >= o) incl -= w;
      if (lane == o) lsum -= w;
      if (lane >= o) icnt -= 1;
      if (lane == o) lrem -= 1;
    } else {
      // every remaining weight is zero: the r-th remaining tile, on counts
      const uint64_t nrem = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(icnt, kWave - 1);
      if (nrem == 0) break;
      const int r = (int)mulhi64(u, nrem);
      const uint64_t above = __ballot(icnt > r);
      const int o = __ffsll((unsigned long long)above) - 1;
      const int base = __builtin_amdgcn_readlane(icnt - lrem, o);
      const int oc0 = o * C, olen = min(n_t, oc0 + C) - oc0;
      int fl[kE], part = 0;
#pragma unroll
      for (int e = 0; e < kE; ++e) {
        const int idx = lane * kE + e;
        fl[e] = idx < olen && (s_p[oc0 + min(idx, olen - 1)] & kChosenBit) == 0 ? 1 : 0;
        part += fl[e];
      }
      const int run = base + wave_inclusive_scan_i_dpp(part);
      const uint64_t hit = __ballot(run > r);
      if (hit == 0ull) break;  // never taken
      const int h = __ffsll((unsigned long long)hit) - 1;
      int acc = run - part, pe = -1;
#pragma unroll
      for (int e = 0; e < kE; ++e) {
        acc += fl[e];
        if (pe < 0 && acc > r) pe = e;
      }
      const int pl = h * kE + __builtin_amdgcn_readlane(pe, h);
      if (lane == h && pl < olen) s_p[oc0 + pl] |= kChosenBit;
      if (lane >= o) icnt -= 1;
      if (lane == o) lrem -= 1;
    }
  }
}

// The chunk-local prefixes of the tile weights into s_p and the chunk
// totals into s_lsum: wave w takes chunks w, w + 16, ..., 64 tiles at a
// time (coalesced reads), the chunk boundaries being the first wave's lane
// chunks.
__device__ void chunk_prefixes(const uint64_t* __restrict__ tw, uint64_t* s_p, uint64_t* s_lsum, int n_t) {
  const int C = (n_t + kWave - 1) / kWave;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (int l = w; l < kWave; l += kSelectThreads / kWave) {
    const int c0 = min(n_t, l * C), c1 = min(n_t, c0 + C);
    uint64_t carry = 0;
    for (int t0 = c0; t0 < c1; t0 += kWave) {
      const int t = t0 + lane;
      const uint64_t x = wave_inclusive_scan_u64_dpp(t < c1 ? tw[t] : 0ull);
      if (t < c1) s_p[t] = carry + x;
      carry += readlane_u64(x, kWave - 1);
    }
    if (lane == 0) s_lsum[l] = carry;
  }
}

__global__ void __launch_bounds__(kSelectThreads) tile_select_kernel(
    uint64_t* __restrict__ tw, int H, int W, int tiles_x, int n_t, int n_sel, int n_pix,
    uint64_t seed, uint64_t step, uint64_t view, int32_t* __restrict__ valid_tiles,
    int32_t* __restrict__ tile_off, int32_t* __restrict__ tile_slot, int64_t* __restrict__ totals,
    uint8_t* __restrict__ chosen, int lds_tiles) {
  extern __shared__ uint64_t s_sel[];  // [n_t] chunk prefixes and chosen bits, when n_t <= lds_tiles
  __shared__ uint64_t s_lsum[kWave];
  const int tid = threadIdx.x;
  const bool all_tiles = n_sel < 0 || n_sel >= n_t;
  const bool in_lds = !all_tiles && n_t <= lds_tiles;
  if (in_lds) {
    chunk_prefixes(tw, s_sel, s_lsum, n_t);
    __syncthreads();
    if (tid < kWave) {
      const uint64_t key = stream_key(seed, step, view, (uint64_t)n_t);
      switch ((n_t + kWave * kWave - 1) / (kWave * kWave)) {  // tiles per lane in a chunk pass
        case 1: select_tiles_lds<1>(s_sel, s_lsum, n_t, n_sel, key); break;
        case 2: select_tiles_lds<2>(s_sel, s_lsum, n_t, n_sel, key); break;
        case 3: select_tiles_lds<3>(s_sel, s_lsum, n_t, n_sel, key); break;
        case 4: select_tiles_lds<4>(s_sel, s_lsum, n_t, n_sel, key); break;
        default: select_tiles_lds<5>(s_sel, s_lsum, n_t, n_sel, key); break;
      }
    }
  } else if (!all_tiles && tid < kWave) {
    // more tiles than LDS holds: each lane walks its own chunk in global memory
    const int lane = tid;
    const int chunk = (n_t + kWave - 1) / kWave;
    const int c0 = min(n_t, lane * chunk), c1 = min(n_t, c0 + chunk);
    for (int t = c0; t < c1; ++t) chosen[t] = 0;
    uint64_t lsum = 0;
    for (int t = c0; t < c1; ++t) lsum += tw[t];
    int lrem = c1 - c0;
    const uint64_t key = stream_key(seed, step, view, (uint64_t)n_t);
    for (int j = 0; j < n_sel; ++j) {
      const uint64_t u = absorb(key, (uint64_t)j);
      const uint64_t incl = wave_inclusive_scan_u64(lsum);
      const uint64_t total = __shfl(incl, 63, kWave);
      if (total > 0) {
        const uint64_t r = mulhi64(u, total);
        const uint64_t excl = incl - lsum;
        if (lsum > 0 && excl <= r && r < incl) {
          uint64_t run = excl;
          for (int t = c0; t < c1; ++t) {
            run += tw[t];
            if (run > r) {
              lsum -= tw[t];
              tw[t] = 0;
              chosen[t] = 1;
              --lrem;
              break;
            }
          }
        }
      } else {
        const int ic = wave_inclusive_scan_i(lrem);
        const int nrem = __shfl(ic, 63, kWave);
        const int r = (int)mulhi64(u, (uint64_t)nrem);
        const int ex = ic - lrem;
        if (lrem > 0 && ex <= r && r < ic) {
          int k = ex;
          for (int t = c0; t < c1; ++t) {
            if (!chosen[t]) {
              if (k == r) {
                chosen[t] = 1;
                --lrem;
                break;
              }
              ++k;
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // ascending list of the chosen tiles with their sample counts
  __shared__ uint32_t lds[kSelectThreads / kWave];
  const int chunk = (n_t + kSelectThreads - 1) / kSelectThreads;
  const int c0 = min(n_t, tid * chunk), c1 = min(n_t, c0 + chunk);
  uint32_t lcount = 0, lpix = 0;
  for (int t = c0; t < c1; ++t)
    if (all_tiles || (in_lds ? (s_sel[t] & kChosenBit) != 0 : chosen[t] != 0)) {
      ++lcount;
      lpix += (uint32_t)min(n_pix, tile_valid_w(t % tiles_x, W) * tile_valid_h(t / tiles_x, H));
    }
  uint32_t n_chosen, P;
  int slot = (int)block_exclusive_scan<kSelectThreads, uint32_t>(lcount, lds, &n_chosen);
  int off = (int)block_exclusive_scan<kSelectThreads, uint32_t>(lpix, lds, &P);
  for (int t = c0; t < c1; ++t) {
    if (all_tiles || (in_lds ? (s_sel[t] & kChosenBit) != 0 : chosen[t] != 0)) {
      valid_tiles[slot] = t;
      tile_off[slot] = off;
      tile_slot[t] = slot;
      off += min(n_pix, tile_valid_w(t % tiles_x, W) * tile_valid_h(t / tiles_x, H));
      ++slot;
    } else {
      tile_slot[t] = -1;
    }
  }
  if (tid == 0) {
    tile_off[n_chosen] = (int32_t)P;
    atomicAdd((unsigned long long*)&totals[0], (unsigned long long)P);
    atomicAdd((unsigned long long*)&totals[1], (unsigned long long)n_chosen);
  }
}

// ------------------------------------------------------------------ tile pixels
__device__ __forceinline__ int split_round(int permille, int n) { return (permille * n + 500) / 1000; }

__global__ void __launch_bounds__(64) tile_pixels_kernel(
    const uint16_t* __restrict__ E, const uint16_t* __restrict__ A, int H, int W, int tiles_x,
    int n_st, int n_pix, int hard_pm, int stable_pm, uint64_t seed, uint64_t step, uint64_t view,
    const int32_t* __restrict__ valid_tiles, const int32_t* __restrict__ tile_off,
    uint8_t* __restrict__ pix) {
  const int slot = blockIdx.x;
  if (slot >= n_st) return;
  const int lane = threadIdx.x;
  const int t = valid_tiles[slot];
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int n_valid = tile_valid_w(tx, W) * tile_valid_h(ty, H);
  const int n = min(n_pix, n_valid);
  int n_hard = split_round(hard_pm, n);
  int n_stable = split_round(stable_pm, n);
  if (n_hard + n_stable > n) n_stable = n - n_hard;
  int n_mixed = n - n_hard - n_stable;

  uint64_t w[4];
  uint32_t age[4];
  bool valid[4];
  for (int k = 0; k < 4; ++k) {
    const int loc = lane * 4 + k;
    const int x = tx * kTile + (loc & 15), y = ty * kTile + (loc >> 4);
    valid[k] = x < W && y < H;
    const int64_t idx = (int64_t)y * W + x;
    w[k] = valid[k] ? half_weight(E[idx]) : 0;
    age[k] = valid[k] ? A[idx] : 0;
  }
  uint32_t picked = 0;  // bit k: local index lane*4+k chosen
  const uint64_t key = stream_key(seed, step, view, (uint64_t)t);

  // --- hard: sequential error-weighted draws without replacement.  The
  // draws' random words are hashed up front, lane l holding draw l + 64 q
  // in uh[q].  The wave prefix sum of the lanes' unpicked weight is taken
  // once and kept up to date: a draw lands in the first lane whose
  // inclusive sum exceeds r, and removing the picked weight lowers the sums
  // of that lane and the lanes after it.
  int n_hard_done = 0;
  {
    uint64_t uh[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) uh[q] = kWave * q < n_hard ? absorb(key, (uint64_t)(lane + kWave * q)) : 0;
    uint64_t ls = w[0] + w[1] + w[2] + w[3];
    uint64_t incl = wave_inclusive_scan_u64(ls);
    uint64_t total = readlane_u64(incl, kWave - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      for (int jj = 0; jj < kWave && n_hard_done < n_hard && total != 0; ++jj) {
        const uint64_t r = mulhi64(readlane_u64(uh[q], jj), total);
        const int pl = (int)__builtin_ctzll(__ballot(incl > r));  // incl of lane 63 = total > r
        uint64_t wp = 0;
        if (lane == pl) {
          uint64_t run = incl - ls;
          for (int k = 0; k < 4; ++k) {
            if ((picked >> k) & 1u) continue;
            run += w[k];
            if (run > r) {
              picked |= 1u << k;
              wp = w[k];
              break;
            }
          }
          ls -= wp;
        }
        wp = readlane_u64(wp, pl);
        if (lane >= pl) incl -= wp;
        total -= wp;
        ++n_hard_done;
      }
    }
  }
  n_mixed += n_hard - n_hard_done;

  // --- stable: TopK age among the rest; key (age << 8) | (255 - loc) is
  // unique and orders by age, then by lower index.  The K-th largest key is
  // found by bisection on counts.
  if (n_stable > 0) {
    uint32_t kk[4];
    bool elig[4];
    for (int k = 0; k < 4; ++k) {
      elig[k] = valid[k] && !((picked >> k) & 1u);
      kk[k] = (age[k] << 8) | (uint32_t)(255 - (lane * 4 + k));
    }
    uint32_t lo = 0, hi = 1u << 24;  // count(key >= lo) >= n_stable > count(key >= hi)
    while (hi - lo > 1) {
      const uint32_t mid = lo + (hi - lo) / 2;
      int c = 0;
      for (int k = 0; k < 4; ++k) c += (elig[k] && kk[k] >= mid) ? 1 : 0;
      c = wave_sum_i(c);
      if (c >= n_stable) lo = mid; else hi = mid;
    }
    for (int k = 0; k < 4; ++k)
      if (elig[k] && kk[k] >= lo) picked |= 1u << k;
  }

  // --- mixed: uniform without replacement over the rest, ascending order
  // (the r-th remaining pixel; words hashed up front and the count prefix
  // kept up to date as above)
  {
    uint64_t um[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      um[q] = kWave * q < n_mixed ? absorb(key, (uint64_t)(256 + lane + kWave * q)) : 0;
    int lc = 0;
    for (int k = 0; k < 4; ++k) lc += (valid[k] && !((picked >> k) & 1u)) ? 1 : 0;
    int ic = wave_inclusive_scan_i(lc);
    int nrem = __builtin_amdgcn_readlane(ic, kWave - 1);
    int done = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // nrem == 0: nothing left, every later draw picks nothing
      for (int jj = 0; jj < kWave && done < n_mixed && nrem > 0; ++jj) {
        const int r = (int)mulhi64(readlane_u64(um[q], jj), (uint64_t)nrem);
        const int pl = (int)__builtin_ctzll(__ballot(ic > r));
        if (lane == pl) {
          int c = ic - lc;
          for (int k = 0; k < 4; ++k) {
            if (!valid[k] || ((picked >> k) & 1u)) continue;
            if (c == r) {
              picked |= 1u << k;
              break;
            }
            ++c;
          }
          --lc;
        }
        if (lane >= pl) --ic;
        --nrem;
        ++done;
      }
    }
  }

  // --- write the sorted local indices
  const int lc = __builtin_popcount(picked);
  const int ic = wave_inclusive_scan_i(lc);
  int pos = tile_off[slot] + ic - lc;
  for (int k = 0; k < 4; ++k)
    if ((picked >> k) & 1u) pix[pos++] = (uint8_t)(lane * 4 + k);
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_sample_workspace_size(int32_t height, int32_t width) {
  if (height <= 0 || width <= 0) return 0;
  const size_t n_t = (size_t)(ceil_div(width, kTile) * ceil_div(height, kTile));
  return align_up(n_t * sizeof(uint64_t), 256) + align_up(n_t, 256);
}

// Tiles whose weights the draws can hold in LDS on the current device: the
// workgroup's LDS limit (160 KiB on gfx950) less the kernel's static arrays,
// 8 bytes per tile, at most what a chunk pass covers (64 x 64 x kSelectMaxE).
// Queried, and the kernel's dynamic LDS limit raised, once per device.
static int select_lds_tiles() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static int cache[kMaxDevices];
  static bool known[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
  std::lock_guard<std::mutex> lock(mu);
  if (!known[dev]) {
    int bytes = 0;
    if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) bytes = 0;
    int dyn = bytes - 2048;  // static LDS of the kernel (chunk sums, scan partials) with margin
    if (dyn > 65536 && hipFuncSetAttribute((const void*)tile_select_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) {
      (void)hipGetLastError();
      dyn = 65536 - 2048;
    }
    cache[dev] = max(0, min(dyn / (int)sizeof(uint64_t), kWave * kWave * kSelectMaxE));
    known[dev] = true;
  }
  return cache[dev];
}

static int32_t sample_impl(const uint16_t* E, const uint16_t* A, int32_t height, int32_t width,
                           const tgs_sample_params* sp, const float* tile_pred, int32_t* valid_tiles,
                           int32_t* tile_off, uint8_t* pix, int32_t* tile_slot, int64_t* totals, void* ws,
                           size_t ws_bytes, void* stream) {
  TGS_REQUIRE(height > 0 && width > 0, "tgs_sample: bad image size %d x %d", width, height);
  TGS_REQUIRE(sp != nullptr, "tgs_sample: null params");
  TGS_REQUIRE(sp->n_pix >= 1 && sp->n_pix <= kTilePixels, "tgs_sample: n_pix %d not in 1..256",
              sp->n_pix);
  TGS_REQUIRE(sp->hard_permille >= 0 && sp->stable_permille >= 0 &&
                  sp->hard_permille + sp->stable_permille <= 1000,
              "tgs_sample: bad hard/stable ratios");
  TGS_REQUIRE(sp->view >= 0, "tgs_sample: negative view index");
  TGS_REQUIRE(E && A && valid_tiles && tile_off && pix && tile_slot && totals && ws,
              "tgs_sample: null pointer");
  TGS_REQUIRE(ws_bytes >= tgs_sample_workspace_size(height, width),
              "tgs_sample: workspace %zu bytes < %zu", ws_bytes,
              tgs_sample_workspace_size(height, width));
  const int tiles_x = (int)ceil_div(width, kTile), tiles_y = (int)ceil_div(height, kTile);
  const int n_t = tiles_x * tiles_y;
  const int n_st = tgs_sample_tile_count(height, width, sp);
  uint64_t* tw = (uint64_t*)ws;
  uint8_t* chosen = (uint8_t*)ws + align_up((size_t)n_t * sizeof(uint64_t), 256);
  hipStream_t s = as_stream(stream);
  const bool all_tiles = sp->n_tiles_sel < 0 || sp->n_tiles_sel >= n_t;
  if (!all_tiles && tile_pred != nullptr)
    hipLaunchKernelGGL(tile_pred_weights_kernel, dim3((unsigned)ceil_div(n_t, 256)), dim3(256), 0, s, tile_pred,
                       height, width, tiles_x, n_t, tw);
  else if (!all_tiles)
    hipLaunchKernelGGL(tile_weights_kernel, dim3(n_t), dim3(64), 0, s, E, height, width, tiles_x,
                       n_t, tw);
  const int lds_tiles = select_lds_tiles();
  const size_t sel_lds = !all_tiles && n_t <= lds_tiles ? (size_t)n_t * sizeof(uint64_t) : 0;
  hipLaunchKernelGGL(tile_select_kernel, dim3(1), dim3(kSelectThreads), sel_lds, s, tw, height, width,
                     tiles_x, n_t, sp->n_tiles_sel, sp->n_pix, sp->seed, sp->step,
                     (uint64_t)sp->view, valid_tiles, tile_off, tile_slot, totals, chosen, lds_tiles);
  if (n_st > 0)
    hipLaunchKernelGGL(tile_pixels_kernel, dim3(n_st), dim3(64), 0, s, E, A, height, width, tiles_x,
                       n_st, sp->n_pix, sp->hard_permille, sp->stable_permille, sp->seed, sp->step,
                       (uint64_t)sp->view, valid_tiles, tile_off, pix);
  return hip_status("tgs_sample");
}

extern "C" int32_t tgs_sample(const uint16_t* E, const uint16_t* A, int32_t height, int32_t width,
                              const tgs_sample_params* sp, const float* tile_pred, int32_t* valid_tiles,
                              int32_t* tile_off, uint8_t* pix, int32_t* tile_slot, int64_t* totals, void* ws,
                              size_t ws_bytes, void* stream) {
  return sample_impl(E, A, height, width, sp, tile_pred, valid_tiles, tile_off, pix, tile_slot, totals, ws,
                     ws_bytes, stream);
}

// ------------------------------------------------------------------ sampling without a workspace
// The sampler's scratch (tile weights and chosen flags, 9 bytes per tile)
// in a file-scope device array, for callers that cannot allocate.  Each
// GPU holds its own copy until the process ends; host code uses only the
// device address that hipGetSymbolAddress returns for the current device,
// never the array's name.  Every kernel of a call writes the scratch it
// reads, so nothing needs clearing between calls; calls that overlap on
// one GPU share it and race.
constexpr int kNoAllocMaxTiles = TGS_SAMPLE_NOALLOC_MAX_TILES;
constexpr size_t kNoAllocScratchBytes =
    ((size_t)kNoAllocMaxTiles * sizeof(uint64_t) + 255) / 256 * 256 + ((size_t)kNoAllocMaxTiles + 255) / 256 * 256;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of the scratch array, looked up on the
// first call on that device.
static void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

extern "C" int32_t tgs_sample_noalloc(const uint16_t* E, const uint16_t* A, int32_t height, int32_t width,
                                      const tgs_sample_params* sp, const float* tile_pred, int32_t* valid_tiles,
                                      int32_t* tile_off, uint8_t* pix, int32_t* tile_slot, int64_t* totals,
                                      void* stream) {
  TGS_REQUIRE(height > 0 && width > 0, "tgs_sample_noalloc: bad image size %d x %d", width, height);
  const int64_t n_t = ceil_div(width, kTile) * ceil_div(height, kTile);
  TGS_REQUIRE(n_t <= kNoAllocMaxTiles, "tgs_sample_noalloc: %lld tiles exceed the static scratch of %d tiles",
              (long long)n_t, kNoAllocMaxTiles);
  void* ws = scratch_address();
  if (ws == nullptr) {
    set_error("tgs_sample_noalloc: no device address for the static scratch");
    return TGS_ERR_HIP;
  }
  return sample_impl(E, A, height, width, sp, tile_pred, valid_tiles, tile_off, pix, tile_slot, totals, ws,
                     kNoAllocScratchBytes, stream);
}

// ------------------------------------------------------------------ per-view mean error
// Eq. anchor_view needs each view's mean error E_bar_v over the image: the
// exact integer sum of the half values times 2^24 (the weights above), one
// 64-bit atomic per workgroup; the host divides by 2^24 |Omega|.
namespace tgs {

__global__ void __launch_bounds__(256) view_error_sum_kernel(const uint16_t* __restrict__ E, int64_t pixels,
                                                             unsigned long long* __restrict__ sums) {
  __shared__ unsigned long long red[256];
  const int v = blockIdx.y;
  const uint16_t* map = E + (int64_t)v * pixels;
  unsigned long long acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < pixels; i += (int64_t)gridDim.x * 256)
    acc += half_weight(map[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0ull) atomicAdd(&sums[v], red[0]);
}

__global__ void __launch_bounds__(256) clear_u64_kernel(unsigned long long* __restrict__ p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace tgs

extern "C" int32_t tgs_view_error_sums(const uint16_t* E, int32_t n_views, int64_t pixels, uint64_t* sums,
                                       void* stream) {
  using namespace tgs;
  TGS_REQUIRE(n_views >= 0 && n_views <= 65535, "tgs_view_error_sums: n_views %d out of range", n_views);
  TGS_REQUIRE(pixels > 0 && pixels < (1ll << 31), "tgs_view_error_sums: pixels out of range");
  if (n_views == 0) return TGS_OK;
  TGS_REQUIRE(E && sums, "tgs_view_error_sums: null pointer");
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(clear_u64_kernel, dim3((unsigned)ceil_div(n_views, 256)), dim3(256), 0, s,
                     (unsigned long long*)sums, n_views);
  const unsigned bx = (unsigned)std::min<int64_t>(ceil_div(pixels, (int64_t)256 * 16), 256);
  hipLaunchKernelGGL(view_error_sum_kernel, dim3(bx, (unsigned)n_views), dim3(256), 0, s, E, pixels,
                     (unsigned long long*)sums);
  return hip_status("tgs_view_error_sums");
}
