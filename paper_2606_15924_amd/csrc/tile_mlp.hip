// Learned tile priority: per-(view, tile) features, a 32 -> 64 -> 64 -> 1
// GELU network (added to the tile's stale mean error, feature 19: it
// predicts the change since the error map was written) evaluated with
// bfloat16 MFMA (float32 sums), and its online
// training step (exact gradient of the mean squared error against the
// measured tile errors, Adam on float32 master weights).  The model is not
// part of the paper; it ranks tiles by the error the sampler of Sec. 3.3
// would measure, for views whose error map is stale.
//
// Parameter vector (float32, 6337): W1[32][64] at 0, b1 at 2048,
// W2[64][64] at 2112, b2 at 6208, w3 at 6272, b3 at 6336.
#include <hip/hip_fp16.h>

#include <cmath>

#include "common.h"

namespace tgs {

constexpr int kFeat = 32, kHid = 64;
constexpr int kOffW1 = 0, kOffB1 = 2048, kOffW2 = 2112, kOffB2 = 6208, kOffW3 = 6272, kOffB3 = 6336;
constexpr int kParams = TGS_TILE_MLP_PARAMS;
static_assert(kOffB3 + 1 == kParams, "parameter layout");

typedef short short8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct PoseArgs {
  float f[16];
};

// One wave per tile: the tile's pixels (4 per lane) give the mean error and
// the mean age; lane 0 writes the tile's 32 features.
__global__ void __launch_bounds__(kWave) tile_features_kernel(const uint2* __restrict__ ranges,
                                                              const __half* __restrict__ E,
                                                              const uint16_t* __restrict__ A, int height,
                                                              int width, int tiles_x, PoseArgs pose,
                                                              float* __restrict__ X) {
  const int t = blockIdx.x, lane = lane_id();
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int x0 = tx * kTile, y0 = ty * kTile;
  float se = 0.f;
  int sa = 0, cnt = 0;
#pragma unroll
  for (int k = 0; k < kTilePixels / kWave; ++k) {
    const int q = lane + k * kWave, py = y0 + q / kTile, px = x0 + q % kTile;
    if (py < height && px < width) {
      const int64_t idx = (int64_t)py * width + px;
      se += __half2float(E[idx]);
      sa += (int)A[idx];
      ++cnt;
    }
  }
  se = wave_sum(se);
  sa = wave_sum_i(sa);
  cnt = wave_sum_i(cnt);
  if (lane == 0) {
    float* x = X + (int64_t)t * kFeat;
    x[0] = (float)(x0 + kTile / 2) / (float)width;
    x[1] = (float)(y0 + kTile / 2) / (float)height;
    for (int j = 0; j < 16; ++j) x[2 + j] = pose.f[j];
    const uint2 r = ranges[t];
    x[18] = log1pf((float)(r.y - r.x));
    x[19] = se / (float)cnt;
    x[20] = log1pf((float)sa / (float)cnt);
    for (int j = 21; j < kFeat; ++j) x[j] = 0.f;
  }
}

// Weights staged once per workgroup: W1, W2 as bfloat16, biases and w3 as float.
struct MlpLds {
  uint16_t w1[kFeat * kHid];
  uint16_t w2[kHid * kHid];
  float b1[kHid], b2[kHid], w3[kHid];
};

__device__ void stage_weights(const float* __restrict__ p, MlpLds& s) {
  for (int i = threadIdx.x; i < kFeat * kHid; i += blockDim.x) s.w1[i] = to_bf16(p[kOffW1 + i]);
  for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) s.w2[i] = to_bf16(p[kOffW2 + i]);
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
    s.b1[i] = p[kOffB1 + i];
    s.b2[i] = p[kOffB2 + i];
    s.w3[i] = p[kOffW3 + i];
  }
}

// The forward runs on gfx950's 16x16x32 bfloat16 MFMA in the transposed
// form Z^T = W^T X^T: A = W^T (16 outputs x 32 inputs), B = X^T (32 inputs x
// 16 rows); lane l holds row/output l % 16 and eight inputs of quarter
// q = l / 16, and receives outputs 4q .. 4q + 3 of row l % 16.  The sum
// over the 32 inputs does not depend on which input each (lane, element)
// slot carries, as long as A and B agree: layer 1 gives slot (q, e) input
// 8q + e (eight consecutive features, two 16-byte loads); layer 2 gives it
// 4q + e (e < 4) or 16 + 4q + e - 4 of its 32-input half, which are
// exactly the outputs of two consecutive output blocks that the previous
// layer left in this lane, so activations never leave registers.
constexpr int kMlpBlock = 256;
constexpr int kMlpRowsPerWave = 16;

__device__ __forceinline__ bf16x8 pack8(const short8& v) { return __builtin_bit_cast(bf16x8, v); }

// Slot e of quarter q: the input index within a 32-input half.
__device__ __forceinline__ int slot_in(int layer, int q, int e) {
  return layer == 1 ? 8 * q + e : (e < 4 ? 4 * q + e : 16 + 4 * q + e - 4);
}

// A operand of W^T for input half kh (inputs 32 kh ..) and output block ob.
__device__ __forceinline__ bf16x8 weight_frag8(const uint16_t* w, int layer, int kh, int ob, int lane) {
  const int q = lane >> 4, o = ob * 16 + (lane & 15);
  short8 a;
#pragma unroll
  for (int e = 0; e < 8; ++e) a[e] = (short)w[(32 * kh + slot_in(layer, q, e)) * kHid + o];
  return pack8(a);
}

__global__ void __launch_bounds__(kMlpBlock) tile_mlp_fwd_kernel(const float* __restrict__ p,
                                                                 const float* __restrict__ X, int64_t n,
                                                                 float* __restrict__ y, float* __restrict__ act) {
  __shared__ MlpLds s;
  stage_weights(p, s);
  __syncthreads();
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int64_t row0 = ((int64_t)blockIdx.x * (kMlpBlock / kWave) + wave) * kMlpRowsPerWave;
  if (row0 >= n) return;  // wave-uniform; no barrier follows
  const int64_t row = row0 + (lane & 15);
  const bool live = row < n;
  const int q = lane >> 4, kq = 4 * q;  // this lane's quarter; its 4 outputs within a block
  // layer 1: the 32 inputs as one MFMA operand (features 8q .. 8q + 7)
  short8 xs;
  {
    const float4 v0 = live ? *reinterpret_cast<const float4*>(X + row * kFeat + 8 * q) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 v1 =
        live ? *reinterpret_cast<const float4*>(X + row * kFeat + 8 * q + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) xs[e] = (short)to_bf16(v[e]);
  }
  const bf16x8 xf = pack8(xs);
  uint16_t h[4][4];  // bfloat16 activations: output block ob, outputs kq .. kq + 3
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(weight_frag8(s.w1, 1, 0, ob, lane), xf, acc, 0, 0, 0);
    float z[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) z[r] = acc[r] + s.b1[ob * 16 + kq + r];
    if (live && act != nullptr)
      *reinterpret_cast<float4*>(act + row * (2 * kHid) + ob * 16 + kq) = make_float4(z[0], z[1], z[2], z[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) h[ob][r] = to_bf16(gelu(z[r]));
  }
  // layer 2 (two 32-input halves) and the output unit
  bf16x8 hf[2];
#pragma unroll
  for (int kh = 0; kh < 2; ++kh) {
    short8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (short)h[2 * kh + (e >> 2)][e & 3];
    hf[kh] = pack8(v);
  }
  float part = 0.f;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kh = 0; kh < 2; ++kh)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(weight_frag8(s.w2, 2, kh, ob, lane), hf[kh], acc, 0, 0, 0);
    float z[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      z[r] = acc[r] + s.b2[ob * 16 + kq + r];
      part += s.w3[ob * 16 + kq + r] * gelu(z[r]);
    }
    if (live && act != nullptr)
      *reinterpret_cast<float4*>(act + row * (2 * kHid) + kHid + ob * 16 + kq) = make_float4(z[0], z[1], z[2], z[3]);
  }
  // the four lanes of a row (l, l + 16, l + 32, l + 48) hold its 64 products
  part += __shfl_xor(part, 16, kWave);
  part += __shfl_xor(part, 32, kWave);
  if (lane < 16 && live) y[row] = X[row * kFeat + 19] + (part + p[kOffB3]);
}

// Gradient of mean (y - target)^2 over n rows, per chunk of rows: the
// chunk's partial sums of every parameter's gradient (summed over chunks in
// a fixed order by the update kernel).
constexpr int kGradRows = 32;  // rows per chunk (the chunk's arrays fill 36 KB of LDS)

struct GradLds {
  float xb[kGradRows][kFeat];   // bfloat16-rounded inputs
  float h1b[kGradRows][kHid];   // bfloat16-rounded first activations
  float h2[kGradRows][kHid];
  float dz2[kGradRows][kHid];
  float dz1[kGradRows][kHid];   // first holds gelu'(z1)
  float dy[kGradRows];
};

__global__ void __launch_bounds__(256) tile_mlp_grad_kernel(const float* __restrict__ p, const float* __restrict__ X,
                                                            const float* __restrict__ act,
                                                            const float* __restrict__ y,
                                                            const float* __restrict__ target, int64_t n,
                                                            float* __restrict__ partials) {
  __shared__ GradLds s;
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kGradRows;
  const float inv_n = 2.0f / (float)n;
  for (int i = tid; i < kGradRows; i += 256) {
    const int64_t row = r0 + i;
    s.dy[i] = row < n ? (y[row] - target[row]) * inv_n : 0.f;
  }
  for (int i = tid; i < kGradRows * kFeat; i += 256) {
    const int rr = i / kFeat, c = i % kFeat;
    const int64_t row = r0 + rr;
    s.xb[rr][c] = row < n ? from_bf16(to_bf16(X[row * kFeat + c])) : 0.f;
  }
  for (int i = tid; i < kGradRows * kHid; i += 256) {
    const int rr = i / kHid, c = i % kHid;
    const int64_t row = r0 + rr;
    const float z1 = row < n ? act[row * 2 * kHid + c] : 0.f;
    const float z2 = row < n ? act[row * 2 * kHid + kHid + c] : 0.f;
    s.h1b[rr][c] = from_bf16(to_bf16(gelu(z1)));
    s.dz1[rr][c] = gelu_grad(z1);
    s.h2[rr][c] = gelu(z2);
    s.dz2[rr][c] = gelu_grad(z2);  // times dy w3 below
  }
  __syncthreads();
  for (int i = tid; i < kGradRows * kHid; i += 256) {
    const int rr = i / kHid, c = i % kHid;
    s.dz2[rr][c] *= s.dy[rr] * p[kOffW3 + c];
  }
  __syncthreads();
  // dz1 = gelu'(z1) * (W2b dz2): the forward's bfloat16 W2 carries the gradient back
  for (int i = tid; i < kGradRows * kHid; i += 256) {
    const int rr = i / kHid, k = i % kHid;
    float d = 0.f;
    for (int o = 0; o < kHid; ++o) d += from_bf16(to_bf16(p[kOffW2 + k * kHid + o])) * s.dz2[rr][o];
    s.dz1[rr][k] *= d;
  }
  __syncthreads();
  float* out = partials + (int64_t)blockIdx.x * kParams;
  for (int i = tid; i < kParams; i += 256) {
    float g = 0.f;
    if (i < kOffB1) {  // W1[j][k]
      const int j = i / kHid, k = i % kHid;
      for (int rr = 0; rr < kGradRows; ++rr) g += s.xb[rr][j] * s.dz1[rr][k];
    } else if (i < kOffW2) {
      const int k = i - kOffB1;
      for (int rr = 0; rr < kGradRows; ++rr) g += s.dz1[rr][k];
    } else if (i < kOffB2) {  // W2[k][o]
      const int k = (i - kOffW2) / kHid, o = (i - kOffW2) % kHid;
      for (int rr = 0; rr < kGradRows; ++rr) g += s.h1b[rr][k] * s.dz2[rr][o];
    } else if (i < kOffW3) {
      const int o = i - kOffB2;
      for (int rr = 0; rr < kGradRows; ++rr) g += s.dz2[rr][o];
    } else if (i < kOffB3) {
      const int o = i - kOffW3;
      for (int rr = 0; rr < kGradRows; ++rr) g += s.dy[rr] * s.h2[rr][o];
    } else {
      for (int rr = 0; rr < kGradRows; ++rr) g += s.dy[rr];
    }
    out[i] = g;
  }
}

// Sums the chunks' partial gradients (chunk order) and applies one
// bias-corrected Adam step in FP64 to the float32 master weights.
__global__ void __launch_bounds__(256) tile_mlp_adam_kernel(float* __restrict__ p, float* __restrict__ m,
                                                            float* __restrict__ v,
                                                            const float* __restrict__ partials, int chunks,
                                                            double lr, double bc1, double bc2,
                                                            float* __restrict__ grad_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kParams) return;
  // chunk order; eight loads in flight at a time
  float g = 0.f;
  int c = 0;
  for (; c + 8 <= chunks; c += 8) {
    float q[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = partials[(int64_t)(c + k) * kParams + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) g += q[k];
  }
  for (; c < chunks; ++c) g += partials[(int64_t)c * kParams + i];
  if (grad_out != nullptr) grad_out[i] = g;
  const double b1 = 0.9, b2 = 0.999;
  const double mm = b1 * (double)m[i] + (1.0 - b1) * (double)g;
  const double vv = b2 * (double)v[i] + (1.0 - b2) * (double)g * (double)g;
  m[i] = (float)mm;
  v[i] = (float)vv;
  p[i] = (float)((double)p[i] - lr * (mm / bc1) / (sqrt(vv / bc2) + 1e-8));
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_tile_features(const uint32_t* ranges, const uint16_t* E, const uint16_t* A, int32_t height,
                                     int32_t width, const tgs_camera* cam, float* X, void* stream) {
  TGS_REQUIRE(height > 0 && width > 0 && cam != nullptr, "tgs_tile_features: bad image or camera");
  TGS_REQUIRE(ranges && E && A && X, "tgs_tile_features: null pointer");
  // camera centre c = -R^T t, then the pose features
  double c[3];
  for (int i = 0; i < 3; ++i) c[i] = -(cam->R[0 + i] * cam->t[0] + cam->R[3 + i] * cam->t[1] + cam->R[6 + i] * cam->t[2]);
  const double rad = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  TGS_REQUIRE(rad > 0.0, "tgs_tile_features: camera at the origin");
  PoseArgs pa;
  const double kPi = 3.14159265358979323846;
  for (int j = 0; j < 3; ++j) pa.f[j] = (float)(c[j] / rad);
  pa.f[3] = (float)(rad / 3.0);
  for (int j = 0; j < 3; ++j) {
    const double d = c[j] / rad;
    pa.f[4 + 4 * j] = (float)std::sin(kPi * d);
    pa.f[5 + 4 * j] = (float)std::cos(kPi * d);
    pa.f[6 + 4 * j] = (float)std::sin(2.0 * kPi * d);
    pa.f[7 + 4 * j] = (float)std::cos(2.0 * kPi * d);
  }
  const int tiles_x = (int)ceil_div(width, kTile), tiles_y = (int)ceil_div(height, kTile);
  hipLaunchKernelGGL(tile_features_kernel, dim3((unsigned)(tiles_x * tiles_y)), dim3(kWave), 0, as_stream(stream),
                     (const uint2*)ranges, (const __half*)E, A, height, width, tiles_x, pa, X);
  return hip_status("tgs_tile_features");
}

extern "C" int32_t tgs_tile_mlp_fwd(const float* params, const float* X, int64_t n, float* y, float* act,
                                    void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_tile_mlp_fwd: n < 0");
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && X && y, "tgs_tile_mlp_fwd: null pointer");
  TGS_REQUIRE(((uintptr_t)X & 15) == 0 && ((uintptr_t)act & 15) == 0,
              "tgs_tile_mlp_fwd: X and act must be 16-byte aligned");
  const int64_t rows_per_block = (kMlpBlock / kWave) * kMlpRowsPerWave;
  hipLaunchKernelGGL(tile_mlp_fwd_kernel, dim3((unsigned)ceil_div(n, rows_per_block)), dim3(kMlpBlock), 0,
                     as_stream(stream), params, X, n, y, act);
  return hip_status("tgs_tile_mlp_fwd");
}

extern "C" size_t tgs_tile_mlp_workspace_size(int64_t n) {
  return n <= 0 ? 0 : (size_t)ceil_div(n, kGradRows) * kParams * sizeof(float);
}

extern "C" int32_t tgs_tile_mlp_train_step(float* params, float* m, float* v, const float* X, const float* act,
                                           const float* y, const float* target, int64_t n, int64_t step, float lr,
                                           float* grad, void* ws, size_t ws_bytes, void* stream) {
  TGS_REQUIRE(n > 0 && step >= 1, "tgs_tile_mlp_train_step: need n > 0 and step >= 1");
  TGS_REQUIRE(params && m && v && X && act && y && target && ws, "tgs_tile_mlp_train_step: null pointer");
  TGS_REQUIRE(ws_bytes >= tgs_tile_mlp_workspace_size(n), "tgs_tile_mlp_train_step: workspace %zu bytes < %zu",
              ws_bytes, tgs_tile_mlp_workspace_size(n));
  hipStream_t s = as_stream(stream);
  const int chunks = (int)ceil_div(n, kGradRows);
  hipLaunchKernelGGL(tile_mlp_grad_kernel, dim3((unsigned)chunks), dim3(256), 0, s, params, X, act, y, target, n,
                     (float*)ws);
  const double bc1 = 1.0 - std::pow(0.9, (double)step), bc2 = 1.0 - std::pow(0.999, (double)step);
  hipLaunchKernelGGL(tile_mlp_adam_kernel, dim3((unsigned)ceil_div(kParams, 256)), dim3(256), 0, s, params, m, v,
                     (const float*)ws, chunks, (double)lr, bc1, bc2, grad);
  return hip_status("tgs_tile_mlp_train_step");
}
