// Projection geometry shared by the projection kernels and the fused
// backward + optimizer kernel: camera record, real SH basis terms, the
// forward EWA geometry of one Gaussian and the chain rule back to its
// parameters.  Every function fixes its own operation order (no
// multiply-add contraction), so each kernel that uses them computes the
// same values bit for bit.
#pragma once

#include <math.h>

#include "common.h"

namespace tgs {


struct CamArgs {
  double R[9];
  double t[3];
  double center[3];
  double fx, fy, cx, cy;
  int width, height, tiles_x, tiles_y;
};

inline CamArgs make_cam(const tgs_camera* c) {
  CamArgs a;
  for (int i = 0; i < 9; ++i) a.R[i] = c->R[i];
  for (int i = 0; i < 3; ++i) a.t[i] = c->t[i];
  // camera centre = -R^T t
  for (int j = 0; j < 3; ++j)
    a.center[j] = -(c->R[0 * 3 + j] * c->t[0] + c->R[1 * 3 + j] * c->t[1] + c->R[2 * 3 + j] * c->t[2]);
  a.fx = c->fx;
  a.fy = c->fy;
  a.cx = c->cx;
  a.cy = c->cy;
  a.width = c->width;
  a.height = c->height;
  a.tiles_x = (int)ceil_div(c->width, kTile);
  a.tiles_y = (int)ceil_div(c->height, kTile);
  return a;
}

// Real SH basis up to degree 3 as Cartesian polynomials of the unit
// direction (Condon-Shortley phase, order l then m = -l..l).  Constants are
// the normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (x sqrt(2) for
// m != 0) folded with the polynomial factors:
constexpr double kC0 = 0.28209479177387814;    // 1/(2 sqrt(pi))
constexpr double kC1 = 0.4886025119029199;     // sqrt(3/(4 pi))
constexpr double kC2a = 1.0925484305920792;    // sqrt(15/(4 pi))
constexpr double kC2b = 0.31539156525252005;   // sqrt(5/(16 pi))
constexpr double kC2c = 0.5462742152960396;    // sqrt(15/(16 pi))
constexpr double kC3a = 0.5900435899266435;    // sqrt(35/(32 pi))
constexpr double kC3b = 2.890611442640554;     // sqrt(105/(4 pi))
constexpr double kC3c = 0.4570457994644658;    // sqrt(21/(32 pi))
constexpr double kC3d = 0.3731763325901154;    // sqrt(7/(16 pi))
constexpr double kC3e = 1.445305721320277;     // sqrt(105/(16 pi))

// Term k of the basis: Y_k and its gradient with respect to (x, y, z).
// With k a constant (an unrolled loop) only that term is computed, so no
// arrays of the basis are kept.
__device__ __forceinline__ void sh_term(int k, double x, double y, double z, double& Y, double& gx,
                                        double& gy, double& gz) {
#pragma clang fp contract(off)
  const double xx = x * x, yy = y * y, zz = z * z;
  switch (k) {
    case 0: Y = kC0; gx = 0; gy = 0; gz = 0; break;
    case 1: Y = -kC1 * y; gx = 0; gy = -kC1; gz = 0; break;
    case 2: Y = kC1 * z; gx = 0; gy = 0; gz = kC1; break;
    case 3: Y = -kC1 * x; gx = -kC1; gy = 0; gz = 0; break;
    case 4: Y = kC2a * x * y; gx = kC2a * y; gy = kC2a * x; gz = 0; break;
    case 5: Y = -kC2a * y * z; gx = 0; gy = -kC2a * z; gz = -kC2a * y; break;
    case 6:
      Y = kC2b * (2.0 * zz - xx - yy);
      gx = -2.0 * kC2b * x; gy = -2.0 * kC2b * y; gz = 4.0 * kC2b * z;
      break;
    case 7: Y = -kC2a * x * z; gx = -kC2a * z; gy = 0; gz = -kC2a * x; break;
    case 8: Y = kC2c * (xx - yy); gx = 2.0 * kC2c * x; gy = -2.0 * kC2c * y; gz = 0; break;
    case 9:
      Y = -kC3a * y * (3.0 * xx - yy);
      gx = -kC3a * 6.0 * x * y; gy = -kC3a * (3.0 * xx - 3.0 * yy); gz = 0;
      break;
    case 10:
      Y = kC3b * x * y * z;
      gx = kC3b * y * z; gy = kC3b * x * z; gz = kC3b * x * y;
      break;
    case 11:
      Y = -kC3c * y * (4.0 * zz - xx - yy);
      gx = -kC3c * (-2.0 * x * y); gy = -kC3c * (4.0 * zz - xx - 3.0 * yy); gz = -kC3c * (8.0 * y * z);
      break;
    case 12:
      Y = kC3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
      gx = kC3d * (-6.0 * x * z); gy = kC3d * (-6.0 * y * z); gz = kC3d * (6.0 * zz - 3.0 * xx - 3.0 * yy);
      break;
    case 13:
      Y = -kC3c * x * (4.0 * zz - xx - yy);
      gx = -kC3c * (4.0 * zz - 3.0 * xx - yy); gy = -kC3c * (-2.0 * x * y); gz = -kC3c * (8.0 * x * z);
      break;
    case 14:
      Y = kC3e * z * (xx - yy);
      gx = kC3e * 2.0 * x * z; gy = -kC3e * 2.0 * y * z; gz = kC3e * (xx - yy);
      break;
    default:
      Y = -kC3a * x * (xx - 3.0 * yy);
      gx = -kC3a * (3.0 * xx - 3.0 * yy); gy = -kC3a * (-6.0 * x * y); gz = 0;
      break;
  }
}

__device__ __forceinline__ int n_sh(int degree) { return (degree + 1) * (degree + 1); }

// Forward geometry shared by both kernels (recomputed in the backward).
struct Geom {
  double mu[3], t[3];
  double s[3], qn[4], qnorm;
  double Rq[3][3], M[3][3], Sigma[3][3];
  double J00, J02, J11, J12;
  double T[2][3];
  double a, b, c, det;
  double px, py, radius;
  bool visible;
  int rect[4];
};

template <typename PT>
__device__ __forceinline__ void geometry(const PT* __restrict__ params, int64_t n, int64_t i,
                                         const CamArgs& cam, double z_near, double dil, Geom& g) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; ++k) g.mu[k] = (double)params[(int64_t)k * n + i];
  for (int r = 0; r < 3; ++r)
    g.t[r] = ((cam.R[r * 3 + 0] * g.mu[0] + cam.R[r * 3 + 1] * g.mu[1]) + cam.R[r * 3 + 2] * g.mu[2]) +
             cam.t[r];
  const double tx = g.t[0], ty = g.t[1], tz = g.t[2];
  const bool in_front = tz > z_near;
  const double tzs = in_front ? tz : 1.0;

  for (int k = 0; k < 3; ++k) g.s[k] = exp((double)params[(int64_t)(3 + k) * n + i]);
  const double qw = params[6 * n + i], qx = params[7 * n + i], qy = params[8 * n + i],
               qz = params[9 * n + i];
  g.qnorm = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  const double w = qw / g.qnorm, x = qx / g.qnorm, y = qy / g.qnorm, z = qz / g.qnorm;
  g.qn[0] = w; g.qn[1] = x; g.qn[2] = y; g.qn[3] = z;
  g.Rq[0][0] = 1.0 - 2.0 * (y * y + z * z);
  g.Rq[0][1] = 2.0 * (x * y - w * z);
  g.Rq[0][2] = 2.0 * (x * z + w * y);
  g.Rq[1][0] = 2.0 * (x * y + w * z);
  g.Rq[1][1] = 1.0 - 2.0 * (x * x + z * z);
  g.Rq[1][2] = 2.0 * (y * z - w * x);
  g.Rq[2][0] = 2.0 * (x * z - w * y);
  g.Rq[2][1] = 2.0 * (y * z + w * x);
  g.Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) g.M[r][k] = g.Rq[r][k] * g.s[k];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      g.Sigma[r][k] = (g.M[r][0] * g.M[k][0] + g.M[r][1] * g.M[k][1]) + g.M[r][2] * g.M[k][2];

  g.J00 = cam.fx / tzs;
  g.J02 = -(cam.fx * tx) / (tzs * tzs);
  g.J11 = cam.fy / tzs;
  g.J12 = -(cam.fy * ty) / (tzs * tzs);
  for (int j = 0; j < 3; ++j) {
    g.T[0][j] = g.J00 * cam.R[0 * 3 + j] + g.J02 * cam.R[2 * 3 + j];
    g.T[1][j] = g.J11 * cam.R[1 * 3 + j] + g.J12 * cam.R[2 * 3 + j];
  }
  double TS[2][3];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      TS[r][k] = (g.T[r][0] * g.Sigma[0][k] + g.T[r][1] * g.Sigma[1][k]) + g.T[r][2] * g.Sigma[2][k];
  const double s00 = (TS[0][0] * g.T[0][0] + TS[0][1] * g.T[0][1]) + TS[0][2] * g.T[0][2];
  const double s01 = (TS[0][0] * g.T[1][0] + TS[0][1] * g.T[1][1]) + TS[0][2] * g.T[1][2];
  const double s11 = (TS[1][0] * g.T[1][0] + TS[1][1] * g.T[1][1]) + TS[1][2] * g.T[1][2];
  g.a = s00 + dil;
  g.b = s01;
  g.c = s11 + dil;
  g.det = g.a * g.c - g.b * g.b;
  const bool ok_det = g.det > 0.0;

  const double mid = 0.5 * (g.a + g.c);
  const double lam1 = mid + sqrt(fmax(0.1, mid * mid - g.det));
  g.radius = ceil(3.0 * sqrt(lam1));
  g.px = ((cam.fx * tx) / tzs + cam.cx) - 0.5;
  g.py = ((cam.fy * ty) / tzs + cam.cy) - 0.5;

  auto tclamp = [](double v, int hi) -> int {
    double tv = trunc(v);
    if (!(tv > 0.0)) return 0;  // also maps NaN to 0
    if (tv > (double)hi) return hi;
    return (int)tv;
  };
  const double r = g.radius;
  g.rect[0] = tclamp((g.px - r) / 16.0, cam.tiles_x);
  g.rect[1] = tclamp((g.py - r) / 16.0, cam.tiles_y);
  g.rect[2] = tclamp(((g.px + r) + 15.0) / 16.0, cam.tiles_x);
  g.rect[3] = tclamp(((g.py + r) + 15.0) / 16.0, cam.tiles_y);
  const int area = (g.rect[2] - g.rect[0]) * (g.rect[3] - g.rect[1]);
  g.visible = in_front && ok_det && area > 0;
}


// ---- chain rule from the screen-space gradient gg (centre x, y; conic a,
// b, c; opacity; r, g, b) of Gaussian i to its 59 parameter rows.  A sink
// sink(row, value) receives each row's gradient exactly once (zero for SH
// rows above the degree).  The pieces below are used whole by chain_rule
// and separately by the fused backward + optimizer kernels; each fixes its
// own operation order.

// Unit view direction u = (mu - camera centre) / |mu - camera centre|.
struct ViewDir {
  double ux, uy, uz, dn;
};

__device__ __forceinline__ ViewDir view_dir(const double (&mu)[3], const CamArgs& cam) {
#pragma clang fp contract(off)
  const double vx = mu[0] - cam.center[0], vy = mu[1] - cam.center[1], vz = mu[2] - cam.center[2];
  ViewDir u;
  u.dn = sqrt(vx * vx + vy * vy + vz * vz);
  u.ux = vx / u.dn;
  u.uy = vy / u.dn;
  u.uz = vz / u.dn;
  return u;
}

// Colour gradient after the clamp at zero (clamped channels pass nothing).
__device__ __forceinline__ void color_grad(const double (&gg)[9], uint8_t cm, double (&drgb)[3]) {
  for (int ch = 0; ch < 3; ++ch) drgb[ch] = (cm >> ch) & 1u ? 0.0 : gg[6 + ch];
}

// SH rows of the coefficients k in [k0, k1): their gradient Y_k * drgb goes
// to the sink and dL/du accumulates grad Y_k * (coefficients . drgb) in k
// order.  Every coefficient is read before the sink sees its row, and
// params is not restrict-qualified, so a sink may update it in place.
template <typename PT, typename Sink>
__device__ __forceinline__ void sh_backward(const PT* params, int64_t n, int64_t i, const ViewDir& u,
                                            const double (&drgb)[3], int nk, int k0, int k1,
                                            double (&dL_du)[3], Sink&& sink) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (k < k0 || k >= k1) continue;
    if (k < nk) {
      double Yk, d0, d1, d2;
      sh_term(k, u.ux, u.uy, u.uz, Yk, d0, d1, d2);
      double gk = 0.0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const int row = 11 + 3 * k + ch;
        gk += (double)params[(int64_t)row * n + i] * drgb[ch];
        sink(row, Yk * drgb[ch]);
      }
      dL_du[0] += d0 * gk;
      dL_du[1] += d1 * gk;
      dL_du[2] += d2 * gk;
    } else {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) sink(11 + 3 * k + ch, 0.0);
    }
  }
}

// Rows 0-10 (mean, log-scale, quaternion, opacity) from the screen-space
// gradient, the geometry and the complete dL/du of the SH rows.
template <typename PT, typename Sink>
__device__ __forceinline__ void geom_backward(const PT* params, int64_t n, int64_t i, const CamArgs& cam,
                                              const Geom& g, const double (&gg)[9], const ViewDir& u,
                                              const double (&dL_du)[3], Sink&& sink) {
#pragma clang fp contract(off)
  const double tx = g.t[0], ty = g.t[1], tz = g.t[2];
  const double ux = u.ux, uy = u.uy, uz = u.uz, dn = u.dn;
  // d Y(v/|v|) / dv = (I - u u^T) grad Y(u) / |v|
  const double udot = ux * dL_du[0] + uy * dL_du[1] + uz * dL_du[2];
  double dmu[3] = {(dL_du[0] - ux * udot) / dn, (dL_du[1] - uy * udot) / dn,
                   (dL_du[2] - uz * udot) / dn};

  // ---- opacity
  const double o = 1.0 / (1.0 + exp(-(double)params[10 * n + i]));
  sink(10, gg[5] * o * (1.0 - o));

  // ---- centre
  const double tz2 = tz * tz, tz3 = tz2 * tz;
  double dt[3];
  dt[0] = gg[0] * cam.fx / tz;
  dt[1] = gg[1] * cam.fy / tz;
  dt[2] = gg[0] * (-cam.fx * tx / tz2) + gg[1] * (-cam.fy * ty / tz2);

  // ---- conic (ca, cb, cc) = (c, -b, a) / det  ->  Sigma' entries
  const double a = g.a, b = g.b, c = g.c, det = g.det, d2 = det * det;
  const double gca = gg[2], gcb = gg[3], gcc = gg[4];
  const double dLa = gca * (-c * c / d2) + gcb * (b * c / d2) + gcc * (1.0 / det - a * c / d2);
  const double dLb = gca * (2.0 * b * c / d2) + gcb * (-1.0 / det - 2.0 * b * b / d2) + gcc * (2.0 * a * b / d2);
  const double dLc = gca * (1.0 / det - a * c / d2) + gcb * (a * b / d2) + gcc * (-a * a / d2);
  const double G[2][2] = {{dLa, 0.5 * dLb}, {0.5 * dLb, dLc}};

  // dSigma = T^T G T ; dT = 2 G T Sigma
  double GT[2][3];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) GT[r][k] = G[r][0] * g.T[0][k] + G[r][1] * g.T[1][k];
  double dSigma[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) dSigma[r][k] = g.T[0][r] * GT[0][k] + g.T[1][r] * GT[1][k];
  double dT[2][3];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      dT[r][k] = 2.0 * (GT[r][0] * g.Sigma[0][k] + GT[r][1] * g.Sigma[1][k] + GT[r][2] * g.Sigma[2][k]);
  // T = J W  ->  dJ = dT W^T (only the four non-zero entries of J matter)
  auto dJ = [&](int r, int k) {
    return dT[r][0] * cam.R[k * 3 + 0] + dT[r][1] * cam.R[k * 3 + 1] + dT[r][2] * cam.R[k * 3 + 2];
  };
  const double dJ00 = dJ(0, 0), dJ02 = dJ(0, 2), dJ11 = dJ(1, 1), dJ12 = dJ(1, 2);
  dt[0] += dJ02 * (-cam.fx / tz2);
  dt[1] += dJ12 * (-cam.fy / tz2);
  dt[2] += dJ00 * (-cam.fx / tz2) + dJ02 * (2.0 * cam.fx * tx / tz3) + dJ11 * (-cam.fy / tz2) +
           dJ12 * (2.0 * cam.fy * ty / tz3);
  // t = W mu + t_cam
  for (int k = 0; k < 3; ++k)
    dmu[k] += cam.R[0 * 3 + k] * dt[0] + cam.R[1 * 3 + k] * dt[1] + cam.R[2 * 3 + k] * dt[2];

  // ---- Sigma = M M^T, M = R(q) diag(s)
  double dM[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      dM[r][k] = 2.0 * (dSigma[r][0] * g.M[0][k] + dSigma[r][1] * g.M[1][k] + dSigma[r][2] * g.M[2][k]);
  double dR[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ds = g.Rq[0][k] * dM[0][k] + g.Rq[1][k] * dM[1][k] + g.Rq[2][k] * dM[2][k];
    sink(3 + k, ds * g.s[k]);
    for (int r = 0; r < 3; ++r) dR[r][k] = dM[r][k] * g.s[k];
  }
  const double w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
  // dL/dq_n from the derivative of each rotation entry
  double dq[4];
  dq[0] = 2.0 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
  dq[1] = 2.0 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0 * x * dR[1][1] - w * dR[1][2] +
                 z * dR[2][0] + w * dR[2][1] - 2.0 * x * dR[2][2]);
  dq[2] = 2.0 * (-2.0 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                 w * dR[2][0] + z * dR[2][1] - 2.0 * y * dR[2][2]);
  dq[3] = 2.0 * (-2.0 * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.0 * z * dR[1][1] +
                 y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  const double qdot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  sink(6, (dq[0] - w * qdot) / g.qnorm);
  sink(7, (dq[1] - x * qdot) / g.qnorm);
  sink(8, (dq[2] - y * qdot) / g.qnorm);
  sink(9, (dq[3] - z * qdot) / g.qnorm);
#pragma unroll
  for (int k = 0; k < 3; ++k) sink(k, dmu[k]);
}

template <typename PT, typename Sink>
__device__ __forceinline__ void chain_rule(const PT* params, int64_t n, int64_t i,
                                           const CamArgs& cam, int sh_degree, const Geom& g,
                                           const double (&gg)[9], uint8_t cm, Sink&& sink) {
  const ViewDir u = view_dir(g.mu, cam);
  double drgb[3];
  color_grad(gg, cm, drgb);
  double dL_du[3] = {0.0, 0.0, 0.0};
  sh_backward(params, n, i, u, drgb, n_sh(sh_degree), 0, 16, dL_du, sink);
  geom_backward(params, n, i, cam, g, gg, u, dL_du, sink);
}

inline int32_t check_raster_params(const tgs_raster_params* rp) {
  TGS_REQUIRE(rp != nullptr, "raster params: null");
  TGS_REQUIRE(rp->sh_degree >= 0 && rp->sh_degree <= 3, "raster params: sh_degree %d not in 0..3",
              rp->sh_degree);
  return TGS_OK;
}

}  // namespace tgs
