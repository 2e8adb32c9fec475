// Sparse supervision (Charbonnier L1 + tile NCC with gradient balance, or the
// tile S-SSIM of the ablation in its place) and the per-pixel error/age maps.
//
// loss: one wave per sampled tile; a lane holds up to four of the tile's
// samples (strided, so loads coalesce).  The tile statistics (means, centred
// second moments, NCC per channel, the two mean gradient norms) are wave
// sums through DPP; everything stays in registers between the passes.
// ema_age: one workgroup per band of eight tiles of a tile row; the sample
// lists are scattered into an LDS slot table and each thread updates eight
// consecutive pixels of a row (16-byte age-map accesses).
#include <hip/hip_fp16.h>

#include "common.h"

namespace tgs {

// SSIM constants for values in [0, 1]: (0.01)^2 and (0.03)^2.
constexpr float kSsimC1 = 1e-4f;
constexpr float kSsimC2 = 9e-4f;

template <bool kDense, bool kSsim = false>
__global__ void __launch_bounds__(64) loss_kernel(
    const float4* __restrict__ out, const float* __restrict__ gt, int H, int W, int tiles_x,
    const int32_t* __restrict__ valid_tiles, const int32_t* __restrict__ tile_off,
    const uint8_t* __restrict__ pix, const int64_t* __restrict__ totals, float eps_c2,
    float eps_n, float eps_l, float4* __restrict__ dL, float* __restrict__ err,
    float* __restrict__ lambda_out, float2* __restrict__ tile_loss) {
  const int slot = blockIdx.x, lane = threadIdx.x;
  const int tile = kDense ? slot : valid_tiles[slot];
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int p0 = kDense ? 0 : tile_off[slot];
  const int np = kDense ? kTilePixels : tile_off[slot + 1] - p0;
  const int64_t HW = (int64_t)H * W;

  bool in[4];
  int64_t oi[4];
  float x[4][3], y[4][3];
  float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = lane + 64 * r;
    int loc = -1;
    if (kDense) {
      loc = k;
    } else if (k < np) {
      loc = pix[p0 + k];
    }
    const int px = tx * kTile + (loc & 15), py = ty * kTile + (loc >> 4);
    in[r] = loc >= 0 && px < W && py < H;
    oi[r] = kDense ? (int64_t)py * W + px : (int64_t)p0 + k;
    if (in[r]) {
      const float4 o = out[oi[r]];
      const int64_t gi = (int64_t)py * W + px;
      x[r][0] = o.x; x[r][1] = o.y; x[r][2] = o.z;
      y[r][0] = gt[gi]; y[r][1] = gt[HW + gi]; y[r][2] = gt[2 * HW + gi];
      for (int c = 0; c < 3; ++c) {
        s[c] += x[r][c];
        s[3 + c] += y[r][c];
      }
      ++cnt;
    } else {
      for (int c = 0; c < 3; ++c) x[r][c] = y[r][c] = 0.f;
    }
  }
  const float n = (float)wave_sum_i(cnt);
  if (n == 0.f) return;
  const float inv_n = 1.f / n;
  float mx[3], my[3];
  for (int c = 0; c < 3; ++c) {
    mx[c] = wave_sum(s[c]) * inv_n;
    my[c] = wave_sum(s[3 + c]) * inv_n;
  }
  float m2[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // Vx, Vy, Cxy per channel
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (!in[r]) continue;
    for (int c = 0; c < 3; ++c) {
      const float xc = x[r][c] - mx[c], yc = y[r][c] - my[c];
      m2[c] += xc * xc;
      m2[3 + c] += yc * yc;
      m2[6 + c] += xc * yc;
    }
  }
  // structure term per channel: NCC, or SSIM (ncc[] then holds SSIM and the
  // per-sample gradient below uses the SSIM factors A1, A2, B1, B2)
  float Vy[3], D[3], rsD[3], ncc[3], A1[3], A2[3], B1[3], B2[3];
  for (int c = 0; c < 3; ++c) {
    const float Vx = wave_sum(m2[c]) * inv_n;
    Vy[c] = wave_sum(m2[3 + c]) * inv_n;
    const float Cxy = wave_sum(m2[6 + c]) * inv_n;
    if constexpr (kSsim) {
      A1[c] = 2.f * mx[c] * my[c] + kSsimC1;
      A2[c] = 2.f * Cxy + kSsimC2;
      B1[c] = mx[c] * mx[c] + my[c] * my[c] + kSsimC1;
      B2[c] = Vx + Vy[c] + kSsimC2;
      ncc[c] = (A1[c] * A2[c]) / (B1[c] * B2[c]);
    } else {
      D[c] = Vx * Vy[c] + eps_n;
      rsD[c] = 1.f / sqrtf(D[c]);
      ncc[c] = Cxy * rsD[c];
    }
  }
  // per-sample gradients and their mean L1 norms
  float g1[4][3], gn[4][3];
  float n1 = 0.f, nn = 0.f, rho_sum = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    for (int c = 0; c < 3; ++c) {
      g1[r][c] = 0.f;
      gn[r][c] = 0.f;
    }
    if (!in[r]) continue;
    for (int c = 0; c < 3; ++c) {
      const float d = x[r][c] - y[r][c];
      const float rho = sqrtf(d * d + eps_c2);
      rho_sum += rho;
      g1[r][c] = d / rho;
      const float xc = x[r][c] - mx[c], yc = y[r][c] - my[c];
      if constexpr (kSsim)
        gn[r][c] = -2.f * ncc[c] * (my[c] / A1[c] + yc / A2[c] - mx[c] / B1[c] - xc / B2[c]);
      else
        gn[r][c] = -(yc * rsD[c] - ncc[c] * Vy[c] * xc / D[c]);
      n1 += fabsf(g1[r][c]);
      nn += fabsf(gn[r][c]);
    }
  }
  const float gbar1 = wave_sum(n1) * inv_n, gbarn = wave_sum(nn) * inv_n;
  const float lam = fminf(fmaxf(gbar1 / (gbarn + eps_l), 0.f), 1.f);
  const float P_step = (float)totals[0], T_step = (float)totals[1];
  const float k1 = 1.f / (3.f * P_step), kn = lam / (3.f * n * T_step);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (!in[r]) continue;
    dL[oi[r]] = make_float4(g1[r][0] * k1 + gn[r][0] * kn, g1[r][1] * k1 + gn[r][1] * kn,
                            g1[r][2] * k1 + gn[r][2] * kn, 0.f);
    err[oi[r]] = fabsf(x[r][0] - y[r][0]) + fabsf(x[r][1] - y[r][1]) + fabsf(x[r][2] - y[r][2]);
  }
  const float rho_tot = wave_sum(rho_sum);
  if (lane == 0) {
    lambda_out[slot] = lam;
    tile_loss[slot] = make_float2(rho_tot * k1, lam * (1.f - (ncc[0] + ncc[1] + ncc[2]) / 3.f) / T_step);
  }
}

__device__ __forceinline__ uint16_t ema_half(uint16_t e_bits, float e, float beta, float omb) {
#pragma clang fp contract(off)
  const float E = __half2float(__ushort_as_half(e_bits));
  const float t1 = omb * E;
  const float t2 = beta * e;
  return __half_as_ushort(__float2half_rn(t1 + t2));
}

// One workgroup per band of kEmaTiles tiles of a tile row (16 rows x 128
// pixels); a thread takes 8 consecutive pixels of one row, so the age map
// moves in 16-byte accesses.  The band's sample lists are first scattered
// into LDS (for each pixel: its sample index or -1); a sampled pixel gets
// age 0 and its error blended, every other pixel age + 1 (saturating).
constexpr int kEmaTiles = 8;

__global__ void __launch_bounds__(256) ema_age_kernel(uint16_t* __restrict__ E, uint16_t* __restrict__ A,
                                                      int H, int W, int tiles_x,
                                                      const int32_t* __restrict__ tile_slot,
                                                      const int32_t* __restrict__ tile_off,
                                                      const uint8_t* __restrict__ pix,
                                                      const float* __restrict__ err, float beta,
                                                      float omb) {
  __shared__ int pos[kEmaTiles][kTilePixels];
  const int tid = threadIdx.x, ty = blockIdx.y, tx0 = blockIdx.x * kEmaTiles;
  for (int k = 0; k < kEmaTiles; ++k) pos[k][tid] = -1;
  __syncthreads();
  for (int k = 0; k < kEmaTiles; ++k) {
    const int tx = tx0 + k;
    if (tx >= tiles_x) break;
    const int slot = tile_slot[ty * tiles_x + tx];
    if (slot >= 0) {
      const int p0 = tile_off[slot], np = tile_off[slot + 1] - p0;
      if (tid < np) pos[k][pix[p0 + tid]] = p0 + tid;
    }
  }
  __syncthreads();
  const int row = tid >> 4, seg = tid & 15;  // 16 rows x 16 segments of 8 pixels
  const int y = ty * kTile + row, x0 = tx0 * kTile + seg * 8;
  if (y >= H || x0 >= W) return;
  const int k = seg >> 1, lx0 = (seg & 1) * 8;  // tile of the band, first local column
  const int64_t i0 = (int64_t)y * W + x0;
  uint16_t a[8];
  const bool vec = (W & 7) == 0 && x0 + 8 <= W;  // 16-byte aligned and inside the row
  if (vec) {
    const uint4 v = *reinterpret_cast<const uint4*>(A + i0);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    for (int j = 0; j < 4; ++j) {
      a[2 * j] = (uint16_t)(w[j] & 0xffffu);
      a[2 * j + 1] = (uint16_t)(w[j] >> 16);
    }
  } else {
    for (int j = 0; j < 8; ++j) a[j] = x0 + j < W ? A[i0 + j] : 0;
  }
  for (int j = 0; j < 8; ++j) {
    const int p = pos[k][row * kTile + lx0 + j];
    if (p >= 0) {
      a[j] = 0;
      E[i0 + j] = ema_half(E[i0 + j], err[p], beta, omb);
    } else {
      a[j] = a[j] == 0xffffu ? a[j] : (uint16_t)(a[j] + 1u);
    }
  }
  if (vec) {
    uint4 v;
    v.x = (uint32_t)a[0] | ((uint32_t)a[1] << 16);
    v.y = (uint32_t)a[2] | ((uint32_t)a[3] << 16);
    v.z = (uint32_t)a[4] | ((uint32_t)a[5] << 16);
    v.w = (uint32_t)a[6] | ((uint32_t)a[7] << 16);
    *reinterpret_cast<uint4*>(A + i0) = v;
  } else {
    for (int j = 0; j < 8; ++j)
      if (x0 + j < W) A[i0 + j] = a[j];
  }
}

__global__ void __launch_bounds__(256) error_init_kernel(const float4* __restrict__ out,
                                                         const float* __restrict__ gt, int64_t HW,
                                                         uint16_t* __restrict__ E) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= HW) return;
  const float4 o = out[i];
  float e;
  {
#pragma clang fp contract(off)
    e = (fabsf(o.x - gt[i]) + fabsf(o.y - gt[HW + i])) + fabsf(o.z - gt[2 * HW + i]);
  }
  E[i] = __half_as_ushort(__float2half_rn(e));
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_loss(const float* out, const float* gt, int32_t height, int32_t width,
                            const int32_t* valid_tiles, const int32_t* tile_off, const uint8_t* pix,
                            int32_t n_st, const int64_t* totals, const tgs_loss_params* lp,
                            float* dL_dout, float* err, float* lambda, float* tile_loss,
                            void* stream) {
  TGS_REQUIRE(height > 0 && width > 0, "tgs_loss: bad image size");
  TGS_REQUIRE(lp != nullptr, "tgs_loss: null params");
  TGS_REQUIRE(out && gt && totals && dL_dout && err && lambda && tile_loss, "tgs_loss: null pointer");
  TGS_REQUIRE(((uintptr_t)out & 15) == 0 && ((uintptr_t)dL_dout & 15) == 0,
              "tgs_loss: out and dL_dout must be 16-byte aligned");
  const int tiles_x = (int)ceil_div(width, kTile), tiles_y = (int)ceil_div(height, kTile);
  hipStream_t s = as_stream(stream);
  TGS_REQUIRE(lp->structure == TGS_STRUCTURE_NCC || lp->structure == TGS_STRUCTURE_SSIM,
              "tgs_loss: unknown structure term %d", lp->structure);
  const float eps_c2 = lp->eps_charb * lp->eps_charb;
  const bool ssim = lp->structure == TGS_STRUCTURE_SSIM;
#define TGS_LOSS(DENSE, SSIM, GRID)                                                                              \
  hipLaunchKernelGGL((loss_kernel<DENSE, SSIM>), dim3(GRID), dim3(64), 0, s, (const float4*)out, gt, height,     \
                     width, tiles_x, valid_tiles, tile_off, pix, totals, eps_c2, lp->eps_ncc, lp->eps_lambda,    \
                     (float4*)dL_dout, err, lambda, (float2*)tile_loss)
  if (valid_tiles == nullptr) {
    if (ssim) TGS_LOSS(true, true, tiles_x * tiles_y);
    else TGS_LOSS(true, false, tiles_x * tiles_y);
  } else {
    TGS_REQUIRE(tile_off && pix, "tgs_loss: null tile_off/pix");
    TGS_REQUIRE(n_st >= 0 && n_st <= tiles_x * tiles_y, "tgs_loss: bad n_st %d", n_st);
    if (n_st > 0) {
      if (ssim) TGS_LOSS(false, true, n_st);
      else TGS_LOSS(false, false, n_st);
    }
  }
#undef TGS_LOSS
  return hip_status("tgs_loss");
}

extern "C" int32_t tgs_ema_age_update(uint16_t* E, uint16_t* A, int32_t height, int32_t width,
                                      const int32_t* tile_slot, const int32_t* tile_off,
                                      const uint8_t* pix, const float* err, float beta,
                                      void* stream) {
  TGS_REQUIRE(height > 0 && width > 0, "tgs_ema_age_update: bad image size");
  TGS_REQUIRE(E && A && tile_slot && tile_off && pix && err, "tgs_ema_age_update: null pointer");
  const int tiles_x = (int)ceil_div(width, kTile), tiles_y = (int)ceil_div(height, kTile);
  const float omb = 1.0f - beta;
  TGS_REQUIRE((width & 7) != 0 || ((uintptr_t)A & 15) == 0,
              "tgs_ema_age_update: A must be 16-byte aligned when the width is a multiple of 8");
  hipLaunchKernelGGL(ema_age_kernel, dim3((unsigned)ceil_div(tiles_x, kEmaTiles), (unsigned)tiles_y), dim3(256), 0,
                     as_stream(stream), E, A, height, width, tiles_x, tile_slot, tile_off, pix, err, beta, omb);
  return hip_status("tgs_ema_age_update");
}

extern "C" int32_t tgs_error_init(const float* out_dense, const float* gt, int32_t height,
                                  int32_t width, uint16_t* E, void* stream) {
  TGS_REQUIRE(height > 0 && width > 0, "tgs_error_init: bad image size");
  TGS_REQUIRE(out_dense && gt && E, "tgs_error_init: null pointer");
  const int64_t HW = (int64_t)height * width;
  hipLaunchKernelGGL(error_init_kernel, dim3((unsigned)ceil_div(HW, 256)), dim3(256), 0,
                     as_stream(stream), (const float4*)out_dense, gt, HW, E);
  return hip_status("tgs_error_init");
}
