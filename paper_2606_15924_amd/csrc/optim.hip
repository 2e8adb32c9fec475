// Hybrid moment-damped LM / Adam update, one thread per Gaussian.
//
// HBM-bound: per touched Gaussian it reads params, grad, m, v (4 x 59 floats)
// and writes params, m, v.  The 10x10 and 4x4 systems are assembled and
// solved by Cholesky in FP64 registers; at one solve per Gaussian the FP64
// arithmetic is a small fraction of the memory time on gfx950.
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

// Solve (g g^T + diag(d)) x = -m (mode 0) or (diag(g^2 + d)) x = -m (mode 1)
// for one block of K rows; Cholesky factorisation in place (lower triangle).
template <int K>
__device__ __forceinline__ void lm_solve(const double* g, const double* m, const double* d, int mode,
                                         double* x) {
  if (mode == 1) {
    for (int i = 0; i < K; ++i) x[i] = -m[i] / (g[i] * g[i] + d[i]);
    return;
  }
  double L[K * (K + 1) / 2];
#define LIDX(i, j) ((i) * ((i) + 1) / 2 + (j))
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) L[LIDX(i, j)] = g[i] * g[j] + (i == j ? d[i] : 0.0);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double s = L[LIDX(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[LIDX(j, k)] * L[LIDX(j, k)];
    const double ljj = sqrt(s);
    L[LIDX(j, j)] = ljj;
#pragma unroll
    for (int i = j + 1; i < K; ++i) {
      double t = L[LIDX(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[LIDX(i, k)] * L[LIDX(j, k)];
      L[LIDX(i, j)] = t / ljj;
    }
  }
  double y[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double t = -m[i];
#pragma unroll
    for (int k = 0; k < i; ++k) t -= L[LIDX(i, k)] * y[k];
    y[i] = t / L[LIDX(i, i)];
  }
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
    double t = y[i];
#pragma unroll
    for (int k = i + 1; k < K; ++k) t -= L[LIDX(k, i)] * x[k];
    x[i] = t / L[LIDX(i, i)];
  }
#undef LIDX
}

template <int K>
__device__ __forceinline__ void lm_block(float* __restrict__ p, const float* __restrict__ grad,
                                         float* __restrict__ m, float* __restrict__ v, int64_t n,
                                         int64_t i, const int (&rows)[K], const OptArgs& o) {
  double g[K], mm[K], d[K], x[K];
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
  lm_solve<K>(g, mm, d, o.lm_mode, x);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t idx = (int64_t)rows[k] * n + i;
    p[idx] = (float)((double)p[idx] + row_lr(o, rows[k]) * x[k]);
  }
}

__device__ __forceinline__ void adam_row(float* __restrict__ p, const float* __restrict__ grad,
                                         float* __restrict__ m, float* __restrict__ v, int64_t idx,
                                         double lr, const OptArgs& o) {
  const double g = grad[idx];
  const double mm = o.beta1 * (double)m[idx] + (1.0 - o.beta1) * g;
  const double vv = o.beta2 * (double)v[idx] + (1.0 - o.beta2) * g * g;
  m[idx] = (float)mm;
  v[idx] = (float)vv;
  const double mh = mm / o.bc1, vh = vv / o.bc2;
  p[idx] = (float)((double)p[idx] - lr * mh / (sqrt(vh) + o.eps_adam));
}

__global__ void __launch_bounds__(256) optimizer_kernel(float* __restrict__ p,
                                                        const float* __restrict__ grad,
                                                        float* __restrict__ m, float* __restrict__ v,
                                                        int64_t n, const uint8_t* __restrict__ touched,
                                                        OptArgs o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;
  if (o.lm_mode == 2) {
    for (int r = 0; r < 14; ++r) adam_row(p, grad, m, v, (int64_t)r * n + i, row_lr(o, r), o);
  } else {
    const int geom[10] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9};
    const int app[4] = {11, 12, 13, 10};
    lm_block<10>(p, grad, m, v, n, i, geom, o);
    lm_block<4>(p, grad, m, v, n, i, app, o);
  }
  for (int r = 14; r < TGS_PARAM_ROWS; ++r) adam_row(p, grad, m, v, (int64_t)r * n + i, o.lr[5], o);
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
  hipLaunchKernelGGL(optimizer_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0,
                     as_stream(stream), params, grad, m, v, n, touched, o);
  return hip_status("tgs_optimizer_step");
}
