// Update rules of the hybrid moment-damped LM / Adam optimizer, shared by
// the optimizer kernels and the fused backward + optimizer kernel.  Each
// function fixes its own operation order (no multiply-add contraction), so
// every kernel using them produces the same values bit for bit; arithmetic
// is FP64 and only stored results are rounded.
#pragma once

#include <math.h>

#include "common.h"

namespace tgs {

// The moments m, v are Gaussian-major: row r of Gaussian i at
// i * kMom + r (TGS_MOMENT_STRIDE floats per Gaussian).
constexpr int kMom = TGS_MOMENT_STRIDE;
__host__ __device__ inline int64_t mom(int64_t i, int row) { return i * kMom + row; }

struct OptArgs {
  double lr[6];  // mean, scale, quat, opacity, sh dc, sh rest
  double beta1, beta2, eps_adam, eps_lm;
  double bc1, bc2;  // 1 - beta^t
  double inv_sqrt_bc2;  // 1 / sqrt(bc2)
  int lm_mode;
};

__host__ __device__ inline double row_lr(const OptArgs& o, int row) {
  if (row < 3) return o.lr[0];
  if (row < 6) return o.lr[1];
  if (row < 10) return o.lr[2];
  if (row == 10) return o.lr[3];
  if (row < 14) return o.lr[4];
  return o.lr[5];
}

// Rows of the two LM blocks: geometry (mean, log-scale, quaternion) and
// base appearance (SH DC r, g, b, opacity).
constexpr int kGeomRows[10] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9};
constexpr int kAppRows[4] = {11, 12, 13, 10};

// Adam step of one entry with gradient g (p, m, v updated in place).
// Adam with bias correction, lr mh / (sqrt(vh) + eps), mh = m / bc1,
// vh = v / bc2, evaluated as (lr / bc1) m / (sqrt(v) / sqrt(bc2) + eps):
// the same value in exact arithmetic with one division and one square root
// per element (lr_bc1 = lr / bc1 is per row group).
__device__ __forceinline__ void adam_elem(float& p, float g, float& m, float& v, double lr_bc1, const OptArgs& o) {
#pragma clang fp contract(off)
  const double gd = g;
  const double mm = o.beta1 * (double)m + (1.0 - o.beta1) * gd;
  const double vv = o.beta2 * (double)v + (1.0 - o.beta2) * gd * gd;
  m = (float)mm;
  v = (float)vv;
  p = (float)((double)p - (lr_bc1 * mm) / (sqrt(vv) * o.inv_sqrt_bc2 + o.eps_adam));
}

// Learning rate of a row divided by the first-moment bias correction.
__host__ __device__ inline double row_lr_bc1(const OptArgs& o, int row) { return row_lr(o, row) / o.bc1; }

// LM step of one block of K rows of a Gaussian (p, m, v updated in place)
// with block gradient gf.
// Solves (g g^T + diag(d)) x = -m (mode 0) or diag(g^2 + d) x = -m (mode 1)
// with the updated moments, d = sqrt(v) + eps.  The mode-0 matrix is
// diagonal plus rank one, so its inverse follows the Sherman-Morrison
// identity:
//   x = -(D^-1 m - D^-1 g (g^T D^-1 m) / (1 + g^T D^-1 g)),
// an exact solve in K divisions and two dot products (no K x K factor in
// registers).  d >= eps > 0 keeps D invertible and 1 + g^T D^-1 g >= 1.
template <int K>
__device__ __forceinline__ void lm_block(float (&p)[K], float (&m)[K], float (&v)[K], const int (&rows)[K],
                                         const float (&gf)[K], const OptArgs& o) {
#pragma clang fp contract(off)
  double g[K], mm[K], d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    g[k] = gf[k];
    mm[k] = o.beta1 * (double)m[k] + (1.0 - o.beta1) * g[k];
    const double vv = o.beta2 * (double)v[k] + (1.0 - o.beta2) * g[k] * g[k];
    d[k] = sqrt(vv) + o.eps_lm;
    m[k] = (float)mm[k];
    v[k] = (float)vv;
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
  for (int k = 0; k < K; ++k) p[k] = (float)((double)p[k] + row_lr(o, rows[k]) * x[k]);
}

// The same on the stores (params [59][n], moments Gaussian-major): loads the block's rows of Gaussian i,
// updates them and stores them back.
template <int K>
__device__ __forceinline__ void lm_update(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                          int64_t n, int64_t i, const int (&rows)[K], const float (&gf)[K],
                                          const OptArgs& o) {
  float pk[K], mk[K], vk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    pk[k] = p[(int64_t)rows[k] * n + i];
    mk[k] = m[mom(i, rows[k])];
    vk[k] = v[mom(i, rows[k])];
  }
  lm_block<K>(pk, mk, vk, rows, gf, o);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    m[mom(i, rows[k])] = mk[k];
    v[mom(i, rows[k])] = vk[k];
    p[(int64_t)rows[k] * n + i] = pk[k];
  }
}

inline int32_t make_opt_args(const tgs_optim_params* op, int64_t step, const char* who, OptArgs& o) {
  TGS_REQUIRE(op != nullptr, "%s: null optimizer params", who);
  TGS_REQUIRE(step >= 1, "%s: step must be >= 1", who);
  TGS_REQUIRE(op->lm_mode >= 0 && op->lm_mode <= 2, "%s: bad lm_mode %d", who, op->lm_mode);
  TGS_REQUIRE(op->beta1 >= 0.0 && op->beta1 < 1.0 && op->beta2 >= 0.0 && op->beta2 < 1.0,
              "%s: betas must lie in [0, 1)", who);
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
  o.inv_sqrt_bc2 = 1.0 / sqrt(o.bc2);
  o.lm_mode = op->lm_mode;
  return TGS_OK;
}

}  // namespace tgs
