// Hybrid moment-damped LM / Adam update.
//
// HBM-bound: per touched Gaussian it reads params, grad, m, v (4 x 59 floats)
// and writes params, m, v.  Two launches split the rows by their kind of
// work so each runs at its own occupancy:
//   lm_kernel     one thread per Gaussian, the two LM blocks (rows 0-13):
//                 10x10 and 4x4 damped systems solved exactly in FP64
//   adam_kernel   the plain Adam rows (14-58, or all rows in Adam mode): a
//                 row per grid line, four consecutive Gaussians per thread
//                 with 16-byte loads when the row length allows
// Arithmetic is FP64 throughout; only the stored results are rounded.
#include "common.h"

namespace tgs {

struct OptArgs {
  double lr[6];  // mean, scale, quat, opacity, sh dc, sh rest
  double beta1, beta2, eps_adam, eps_lm;
  double bc1, bc2;  // 1 - beta^t
  int lm_mode;
};

__device__ __forceinline__ double row_lr(const OptArgs& o, int row) {
  if (row < 3) return o.lr[0];
  if (row < 6) return o.lr[1];
  if (row < 10) return o.lr[2];
  if (row == 10) return o.lr[3];
  if (row < 14) return o.lr[4];
  return o.lr[5];
}

// Solve (g g^T + diag(d)) x = -m (mode 0) or diag(g^2 + d) x = -m (mode 1)
// for one block of K rows.  The mode-0 matrix is diagonal plus rank one, so
// its inverse follows the Sherman-Morrison identity:
//   x = -(D^-1 m - D^-1 g (g^T D^-1 m) / (1 + g^T D^-1 g)),
// an exact solve in K divisions and two dot products (no K x K factor in
// registers).  d >= eps > 0 keeps D invertible and 1 + g^T D^-1 g >= 1.
template <int K>
__device__ __forceinline__ void lm_block(float* __restrict__ p, const float* __restrict__ grad,
                                         float* __restrict__ m, float* __restrict__ v, int64_t n,
                                         int64_t i, const int (&rows)[K], const OptArgs& o) {
  double g[K], mm[K], d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t idx = (int64_t)rows[k] * n + i;
    g[k] = grad[idx];
    mm[k] = o.beta1 * (double)m[idx] + (1.0 - o.beta1) * g[k];
    const double vv = o.beta2 * (double)v[idx] + (1.0 - o.beta2) * g[k] * g[k];
    d[k] = sqrt(vv) + o.eps_lm;
    m[idx] = (float)mm[k];
    v[idx] = (float)vv;
  }
  double x[K];
  if (o.lm_mode == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = -mm[k] / (g[k] * g[k] + d[k]);
  } else {
    double s = 0.0, t = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      d[k] = 1.0 / d[k];
      s += g[k] * g[k] * d[k];
      t += g[k] * mm[k] * d[k];
    }
    const double c = t / (1.0 + s);
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = (g[k] * c - mm[k]) * d[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t idx = (int64_t)rows[k] * n + i;
    p[idx] = (float)((double)p[idx] + row_lr(o, rows[k]) * x[k]);
  }
}

__device__ __forceinline__ void adam_elem(float& p, float g, float& m, float& v, double lr, const OptArgs& o) {
  const double gd = g;
  const double mm = o.beta1 * (double)m + (1.0 - o.beta1) * gd;
  const double vv = o.beta2 * (double)v + (1.0 - o.beta2) * gd * gd;
  m = (float)mm;
  v = (float)vv;
  const double mh = mm / o.bc1, vh = vv / o.bc2;
  p = (float)((double)p - lr * mh / (sqrt(vh) + o.eps_adam));
}

__global__ void __launch_bounds__(256) lm_kernel(float* __restrict__ p, const float* __restrict__ grad,
                                                 float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                 const uint8_t* __restrict__ touched, OptArgs o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;
  const int geom[10] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9};
  const int app[4] = {11, 12, 13, 10};
  lm_block<10>(p, grad, m, v, n, i, geom, o);
  lm_block<4>(p, grad, m, v, n, i, app, o);
}

// Rows row0 + blockIdx.y; thread handles Gaussians [i0, i0 + 4).  kVec: the
// row length is a multiple of 4, so the four values are one aligned float4.
template <bool kVec>
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   const uint8_t* __restrict__ touched, int row0, OptArgs o) {
  const int row = row0 + (int)blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  const double lr = row_lr(o, row);
  const int64_t base = (int64_t)row * n + i0;
  if (kVec) {
    bool t[4] = {true, true, true, true};
    if (touched != nullptr) {
      const uchar4 tt = *reinterpret_cast<const uchar4*>(touched + i0);
      t[0] = tt.x != 0; t[1] = tt.y != 0; t[2] = tt.z != 0; t[3] = tt.w != 0;
      if (!(t[0] || t[1] || t[2] || t[3])) return;
    }
    float4 pp = *reinterpret_cast<const float4*>(p + base);
    const float4 gg = *reinterpret_cast<const float4*>(grad + base);
    float4 mm = *reinterpret_cast<const float4*>(m + base);
    float4 vv = *reinterpret_cast<const float4*>(v + base);
    if (t[0]) adam_elem(pp.x, gg.x, mm.x, vv.x, lr, o);
    if (t[1]) adam_elem(pp.y, gg.y, mm.y, vv.y, lr, o);
    if (t[2]) adam_elem(pp.z, gg.z, mm.z, vv.z, lr, o);
    if (t[3]) adam_elem(pp.w, gg.w, mm.w, vv.w, lr, o);
    // untouched lanes store back the values they read
    *reinterpret_cast<float4*>(p + base) = pp;
    *reinterpret_cast<float4*>(m + base) = mm;
    *reinterpret_cast<float4*>(v + base) = vv;
  } else {
    for (int k = 0; k < 4 && i0 + k < n; ++k) {
      if (touched != nullptr && touched[i0 + k] == 0) continue;
      const int64_t idx = base + k;
      float pp = p[idx], mm = m[idx], vv = v[idx];
      adam_elem(pp, grad[idx], mm, vv, lr, o);
      p[idx] = pp;
      m[idx] = mm;
      v[idx] = vv;
    }
  }
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_optimizer_step(float* params, const float* grad, float* m, float* v,
                                      int64_t n, const uint8_t* touched,
                                      const tgs_optim_params* op, int64_t step, void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_optimizer_step: n < 0");
  TGS_REQUIRE(op != nullptr, "tgs_optimizer_step: null params");
  TGS_REQUIRE(step >= 1, "tgs_optimizer_step: step must be >= 1");
  TGS_REQUIRE(op->lm_mode >= 0 && op->lm_mode <= 2, "tgs_optimizer_step: bad lm_mode %d", op->lm_mode);
  TGS_REQUIRE(op->beta1 >= 0.0 && op->beta1 < 1.0 && op->beta2 >= 0.0 && op->beta2 < 1.0,
              "tgs_optimizer_step: betas must lie in [0, 1)");
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && grad && m && v, "tgs_optimizer_step: null pointer");
  OptArgs o;
  o.lr[0] = op->lr_mean;
  o.lr[1] = op->lr_scale;
  o.lr[2] = op->lr_quat;
  o.lr[3] = op->lr_opacity;
  o.lr[4] = op->lr_sh_dc;
  o.lr[5] = op->lr_sh_rest;
  o.beta1 = op->beta1;
  o.beta2 = op->beta2;
  o.eps_adam = op->eps_adam;
  o.eps_lm = op->eps_lm;
  o.bc1 = 1.0 - pow(op->beta1, (double)step);
  o.bc2 = 1.0 - pow(op->beta2, (double)step);
  o.lm_mode = op->lm_mode;
  hipStream_t s = as_stream(stream);
  if (o.lm_mode != 2)
    hipLaunchKernelGGL(lm_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, params, grad, m, v, n,
                       touched, o);
  const int row0 = o.lm_mode == 2 ? 0 : 14;
  const dim3 grid((unsigned)ceil_div(n, 1024), (unsigned)(TGS_PARAM_ROWS - row0));
  const bool vec = n % 4 == 0 && ((uintptr_t)params & 15) == 0 && ((uintptr_t)grad & 15) == 0 &&
                   ((uintptr_t)m & 15) == 0 && ((uintptr_t)v & 15) == 0 && ((uintptr_t)touched & 3) == 0;
  if (vec)
    hipLaunchKernelGGL(adam_kernel<true>, grid, dim3(256), 0, s, params, grad, m, v, n, touched, row0, o);
  else
    hipLaunchKernelGGL(adam_kernel<false>, grid, dim3(256), 0, s, params, grad, m, v, n, touched, row0, o);
  return hip_status("tgs_optimizer_step");
}
