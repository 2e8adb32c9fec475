// Tile-wise error/age pixel sampling (Sec. 3.5).
//
// Three kernels per view:
//   tile_keys     eight lanes per tile (one thread with predicted weights): the
//                 integer tile weight (sum of E * 2^24) and the tile's race
//                 key, only when a subset of tiles is drawn;
//   tile_select   one workgroup: the tiles of the smallest race keys, listed
//                 ascending with their sample counts, prefix offsets and the
//                 tile -> slot map (every tile: a thread per tile, closed
//                 form);
//   tile_pixels   one wave per selected tile: N_hard sequential error-weighted
//                 draws without replacement, TopK age, uniform mixed draws.
// All decisions are integer: weights are exact integers (every finite
// non-negative half times 2^24 is one), a draw r = floor(u * W / 2^64) uses
// the high half of a 64 x 64-bit product, and the pick is the first pixel
// (ascending local index) whose running weight exceeds r.  Each lane owns four
// consecutive local indices, so lane order is index order and a wave prefix
// sum locates a draw.
//
// The tile pass draws tiles without replacement in proportion to weight.  Its
// order does not matter (tiles are listed ascending), so it runs as the
// exponential race of Efraimidis and Spirakis (IPL 2006), which has the
// sequential draws' distribution: tile t runs an Exp(1) time over its weight
// and the earliest n_sel win.  The time is exact integer and IEEE arithmetic:
// L = -log2 of the tile's uniform to 47 fractional bits (binary logarithm by
// repeated squaring), one correctly rounded double division L / w, and its bit
// pattern as the key; zero-weight tiles key 2^63 + u / 2, after every weighted
// tile.  Selection is an exact MSB-first radix select on the 64-bit keys, ties
// to the lower tile index.
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

// ------------------------------------------------------------------ race keys
constexpr int kLogFrac = 47;  // fractional bits of a race time: 64 * 2^47 = 2^53 is exact in a double

// 2^47 * -log2(v / 2^64) for v = u | 1, the fraction truncated: with
// v = 2^e m, m in [1, 2), the time is 64 - e - log2(m), and each squaring of m
// (held in Q1.63, truncated) yields the next bit of log2(m): bit 1 and
// m <- m^2 / 2 when m^2 >= 2, else bit 0 and m <- m^2.
__device__ __forceinline__ uint64_t neg_log2_fixed(uint64_t u) {
  const uint64_t v = u | 1ull;
  const int e = 63 - __clzll((long long)v);
  uint64_t m = v << (63 - e);
  uint64_t frac = 0;
#pragma unroll 4
  for (int k = 0; k < kLogFrac; ++k) {
    const uint64_t hi = __umul64hi(m, m);
    const uint64_t lo_top = (m * m) >> 63;
    const uint64_t bit = hi >> 63;
    frac = (frac << 1) | bit;
    m = bit ? hi : ((hi << 1) | lo_top);
  }
  return ((uint64_t)(64 - e) << kLogFrac) - frac;
}

// Race key of a tile of weight w whose uniform is u: the bit pattern of the
// positive double L / w (ordered like the doubles, below 2^63), or 2^63 + u / 2
// for w = 0.
__device__ __forceinline__ uint64_t race_key(uint64_t w, uint64_t u) {
  if (w == 0) return (1ull << 63) | (u >> 1);
  return (uint64_t)__double_as_longlong(__ddiv_rn((double)neg_log2_fixed(u), (double)w));
}

// Eight tiles per wave, eight lanes per tile: lane k of a tile's group sums
// its pixels k, k + 8, ... (32 of them, a half row per load across the
// group), a butterfly over the group adds the eight 64-bit partial sums
// exactly, and the group's first lane computes the key, eight keys in
// parallel per wave.
constexpr int kKeyTiles = 8;

__global__ void __launch_bounds__(64) tile_keys_kernel(const uint16_t* __restrict__ E, int H, int W,
                                                       int tiles_x, int n_t, uint64_t seed, uint64_t step,
                                                       uint64_t view, uint64_t* __restrict__ keys) {
  const int lane = threadIdx.x;
  const int sub = lane & (kKeyTiles - 1);
  const int t = blockIdx.x * kKeyTiles + lane / kKeyTiles;
  uint64_t s = 0;
  if (t < n_t) {
    const int tx = t % tiles_x, ty = t / tiles_x;
#pragma unroll 8
    for (int k = 0; k < kTilePixels / kKeyTiles; ++k) {
      const int loc = sub + kKeyTiles * k;
      const int x = tx * kTile + (loc & 15), y = ty * kTile + (loc >> 4);
      if (x < W && y < H) s += half_weight(E[(int64_t)y * W + x]);
    }
  }
#pragma unroll
  for (int o = 1; o < kKeyTiles; o <<= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)s, o, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(s >> 32), o, kWave);
    s += ((uint64_t)hi << 32) | lo;
  }
  if (t < n_t && sub == 0)
    keys[t] = race_key(s, absorb(stream_key(seed, step, view, (uint64_t)n_t), (uint64_t)t));
}

// Keys from predicted mean tile errors: weight floor(clamp(p, 0, 65504) *
// in-image pixels * 2^24), the units of the error-map sums; exact in FP64 (a
// float times a count up to 256 times a power of two).
__global__ void __launch_bounds__(256) tile_pred_keys_kernel(const float* __restrict__ pred, int H, int W,
                                                            int tiles_x, int n_t, uint64_t seed, uint64_t step,
                                                            uint64_t view, uint64_t* __restrict__ keys) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n_t) return;
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int nx = min(kTile, W - tx * kTile), ny = min(kTile, H - ty * kTile);
  const float p = pred[t];
  const double q = p > 0.f ? (double)fminf(p, 65504.f) : 0.0;  // NaN and negatives give 0
  const uint64_t w = (uint64_t)floor(q * (double)(nx * ny) * 16777216.0);
  keys[t] = race_key(w, absorb(stream_key(seed, step, view, (uint64_t)n_t), (uint64_t)t));
}

// ------------------------------------------------------------------ tile select
// Every tile: a thread per tile writes its slot and its sample offset in
// closed form (every tile column but the last is 16 pixels wide, every row
// but the last 16 high), so no single-workgroup pass has to wait for a free
// compute unit while other streams' kernels fill the device.
__global__ void __launch_bounds__(256) tile_list_all_kernel(int H, int W, int tiles_x, int tiles_y, int n_pix,
                                                            int32_t* __restrict__ valid_tiles,
                                                            int32_t* __restrict__ tile_off,
                                                            int32_t* __restrict__ tile_slot,
                                                            int64_t* __restrict__ totals) {
  const int n_t = tiles_x * tiles_y;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t > n_t) return;
  const int wl = W - (tiles_x - 1) * kTile, hl = H - (tiles_y - 1) * kTile;  // last column's width, last row's height
  const int64_t row16 = (int64_t)(tiles_x - 1) * min(n_pix, kTile * kTile) + min(n_pix, wl * kTile);
  const int ty = t / tiles_x, tx = t % tiles_x;  // t = n_t: ty = tiles_y, tx = 0
  int64_t off = (int64_t)min(ty, tiles_y - 1) * row16;
  if (ty == tiles_y) off += (int64_t)(tiles_x - 1) * min(n_pix, kTile * hl) + min(n_pix, wl * hl);
  else off += (int64_t)tx * min(n_pix, kTile * (ty == tiles_y - 1 ? hl : kTile));
  tile_off[t] = (int32_t)off;
  if (t < n_t) {
    valid_tiles[t] = t;
    tile_slot[t] = t;
  } else {
    atomicAdd((unsigned long long*)&totals[0], (unsigned long long)off);
    atomicAdd((unsigned long long*)&totals[1], (unsigned long long)n_t);
  }
}

// A subset: one workgroup.  An MSB-first radix select over the race keys (8
// bits a pass, LDS histogram, keys staged in LDS when they fit) finds the
// n_sel-th smallest key thr and how many of the keys equal to it are taken
// (krem, the lowest tile indices first); then the whole workgroup lists the
// chosen tiles in ascending order with their sample counts and prefix
// offsets.
constexpr int kSelectThreads = 1024;

__global__ void __launch_bounds__(kSelectThreads) tile_select_kernel(
    const uint64_t* __restrict__ keys, int H, int W, int tiles_x, int n_t, int n_sel, int n_pix,
    int32_t* __restrict__ valid_tiles, int32_t* __restrict__ tile_off, int32_t* __restrict__ tile_slot,
    int64_t* __restrict__ totals, int lds_tiles) {
  extern __shared__ uint64_t s_keys[];  // [n_t] when n_t <= lds_tiles
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_thr;
  __shared__ int s_krem, s_done;
  const int tid = threadIdx.x, lane = lane_id();
  const bool in_lds = n_t <= lds_tiles;  // 0 <= n_sel < n_t here
  if (in_lds)
    for (int t = tid; t < n_t; t += kSelectThreads) s_keys[t] = keys[t];
  __syncthreads();
  const uint64_t* kk = in_lds ? s_keys : keys;
  uint64_t thr = 0;  // n_sel = 0: no key is below 0 and none is taken at it
  int krem = 0;
  int fs = 0;  // keys are compared on their bits from fs up
  if (n_sel > 0) {
    krem = n_sel;
    for (int shift = 56; shift >= 0; shift -= 8) {
      if (tid < 256) hist[tid] = 0;
      __syncthreads();
      const uint64_t hmask = shift == 56 ? 0ull : ~0ull << (shift + 8);  // bits already fixed
      for (int t0 = 0; t0 < n_t; t0 += kSelectThreads) {
        const int t = t0 + tid;
        const uint64_t k = t < n_t ? kk[t] : 0ull;
        const bool act = t < n_t && ((k ^ thr) & hmask) == 0;
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint64_t am = __ballot(act);
        if (am != 0ull) {
          // one atomic for the wave when its candidates share a digit (the
          // leading passes, where every key has the same exponent bits)
          const int o = __ffsll((unsigned long long)am) - 1;
          const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, o);
          if (__ballot(act && d == d0) == am) {
            if (lane == o) atomicAdd(&hist[d0], (uint32_t)__popcll(am));
          } else if (act) {
            atomicAdd(&hist[d], 1u);
          }
        }
      }
      __syncthreads();
      if (tid < kWave) {
        uint32_t h[4], sum = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          h[i] = hist[lane * 4 + i];
          sum += h[i];
        }
        const uint32_t incl = wave_inclusive_scan_t<uint32_t>(sum);
        // the candidates number at least krem, so some lane's sum reaches it
        const int o = __ffsll((unsigned long long)__ballot(incl >= (uint32_t)krem)) - 1;
        if (lane == o) {
          uint32_t below = incl - sum;  // candidates in the bins before this lane's
          int b = -1;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (b < 0) {
              if (below + h[i] >= (uint32_t)krem) b = i;
              else below += h[i];
            }
          }
          s_thr = thr | ((uint64_t)(lane * 4 + b) << shift);
          s_krem = krem - (int)below;
          // the bin holds exactly the keys still to take: every key with
          // this prefix is chosen and the lower bits decide nothing
          s_done = (int)h[b] == krem - (int)below;
        }
      }
      __syncthreads();
      thr = s_thr;
      krem = s_krem;
      if (s_done) {  // workgroup-uniform
        fs = shift;
        break;
      }
    }
  }
  // ascending list of the chosen tiles (keys below thr, and the first krem
  // tiles whose key equals thr, both on the bits from fs up) with their
  // sample counts
  __shared__ uint32_t lds[kSelectThreads / kWave];
  const int chunk = (n_t + kSelectThreads - 1) / kSelectThreads;
  const int c0 = min(n_t, tid * chunk), c1 = min(n_t, c0 + chunk);
  uint32_t lties = 0;
  const uint64_t thr_s = thr >> fs;
  for (int t = c0; t < c1; ++t) lties += kk[t] >> fs == thr_s ? 1u : 0u;
  uint32_t n_ties;
  const uint32_t tie0 = block_exclusive_scan<kSelectThreads, uint32_t>(lties, lds, &n_ties);
  uint32_t lcount = 0, lpix = 0;
  uint32_t tie = tie0;
  for (int t = c0; t < c1; ++t) {
    const uint64_t k = kk[t] >> fs;
    const bool ch = k < thr_s || (k == thr_s && tie++ < (uint32_t)krem);
    if (ch) {
      ++lcount;
      lpix += (uint32_t)min(n_pix, tile_valid_w(t % tiles_x, W) * tile_valid_h(t / tiles_x, H));
    }
  }
  uint32_t n_chosen, P;
  int slot = (int)block_exclusive_scan<kSelectThreads, uint32_t>(lcount, lds, &n_chosen);
  int off = (int)block_exclusive_scan<kSelectThreads, uint32_t>(lpix, lds, &P);
  tie = tie0;
  for (int t = c0; t < c1; ++t) {
    const uint64_t k = kk[t] >> fs;
    const bool ch = k < thr_s || (k == thr_s && tie++ < (uint32_t)krem);
    if (ch) {
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
  return align_up(n_t * sizeof(uint64_t), 256);
}

// Tiles whose race keys the select can stage in LDS on the current device:
// the workgroup's LDS limit (160 KiB on gfx950) less the kernel's static
// arrays, 8 bytes per tile.  Queried, and the kernel's dynamic LDS limit
// raised, once per device.
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
    int dyn = bytes - 2048;  // static LDS of the kernel (histogram, scan partials) with margin
    if (dyn > 65536 && hipFuncSetAttribute((const void*)tile_select_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) {
      (void)hipGetLastError();
      dyn = 65536 - 2048;
    }
    cache[dev] = max(0, dyn / (int)sizeof(uint64_t));
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
  uint64_t* keys = (uint64_t*)ws;
  hipStream_t s = as_stream(stream);
  const bool all_tiles = sp->n_tiles_sel < 0 || sp->n_tiles_sel >= n_t;
  if (!all_tiles && tile_pred != nullptr)
    hipLaunchKernelGGL(tile_pred_keys_kernel, dim3((unsigned)ceil_div(n_t, 256)), dim3(256), 0, s, tile_pred,
                       height, width, tiles_x, n_t, sp->seed, sp->step, (uint64_t)sp->view, keys);
  else if (!all_tiles)
    hipLaunchKernelGGL(tile_keys_kernel, dim3((unsigned)ceil_div(n_t, kKeyTiles)), dim3(64), 0, s, E, height, width,
                       tiles_x, n_t, sp->seed, sp->step, (uint64_t)sp->view, keys);
  if (all_tiles) {
    hipLaunchKernelGGL(tile_list_all_kernel, dim3((unsigned)ceil_div(n_t + 1, 256)), dim3(256), 0, s, height, width,
                       tiles_x, tiles_y, sp->n_pix, valid_tiles, tile_off, tile_slot, totals);
  } else {
    const int lds_tiles = select_lds_tiles();
    const size_t sel_lds = n_t <= lds_tiles ? (size_t)n_t * sizeof(uint64_t) : 0;
    hipLaunchKernelGGL(tile_select_kernel, dim3(1), dim3(kSelectThreads), sel_lds, s, keys, height, width,
                       tiles_x, n_t, sp->n_tiles_sel, sp->n_pix, valid_tiles, tile_off, tile_slot, totals,
                       lds_tiles);
  }
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
// The sampler's scratch (the tiles' race keys, 8 bytes per tile)
// in a file-scope device array, for callers that cannot allocate.  Each
// GPU holds its own copy until the process ends; host code uses only the
// device address that hipGetSymbolAddress returns for the current device,
// never the array's name.  Every kernel of a call writes the scratch it
// reads, so nothing needs clearing between calls; calls that overlap on
// one GPU share it and race.
constexpr int kNoAllocMaxTiles = TGS_SAMPLE_NOALLOC_MAX_TILES;
constexpr size_t kNoAllocScratchBytes =
    ((size_t)kNoAllocMaxTiles * sizeof(uint64_t) + 255) / 256 * 256;
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
