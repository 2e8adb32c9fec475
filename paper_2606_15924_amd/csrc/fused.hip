// Projection backward fused with the optimizer step, for the last view of
// a training step: the chain rule produces each parameter row's gradient in
// registers and the row is updated in the same pass, so the gradient never
// goes through HBM.  Two launches split the rows by their work:
//   sh_rest_kernel   the SH rows of degree >= 1 (rows 14-58, always Adam
//                    rows): their gradient Y_k(u) * dL/drgb,
//                    the Adam update, and the partial dL/du of these rows
//                    (three doubles per Gaussian in the workspace); each
//                    SH term's rows are loaded while the previous term is
//                    updated, so the kernel streams at close to HBM rate
//   geom_lm_kernel   the geometry chain rule and rows 0-13 (SH DC, opacity,
//                    mean, scale, quaternion) with the LM (or Adam) update;
//                    its rows reach LDS while the chain rule runs
// The SH-rest kernel reads the coefficients before updating them, and the
// geometry kernel only touches rows 0-13, so running them in this order
// gives each the values the unfused path sees.  Results equal
// tgs_project_bwd followed by tgs_optimizer_step bit for bit: gradients are
// rounded to float as the unfused path stores them, the dL/du sum keeps
// its order (the DC term contributes an exact zero), and both paths share
// the update functions.
#include <algorithm>

#include "optimizer.h"
#include "projection.h"

namespace tgs {

template <int kDeg>
__global__ void __launch_bounds__(256) sh_rest_kernel(
    float* params, int64_t n, CamArgs cam, const int* __restrict__ radius, const uint8_t* __restrict__ clampm,
    const float* __restrict__ g2d, const float* __restrict__ grad_prev, float* __restrict__ m,
    float* __restrict__ v, const uint8_t* __restrict__ touched, OptArgs o, double* __restrict__ dL_du_out) {
#pragma clang fp contract(off)
  constexpr int nk = (kDeg + 1) * (kDeg + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;  // untouched: parameters and moments stay
  const bool vis = radius[i] != 0;
  double drgb[3] = {0.0, 0.0, 0.0}, dL_du[3] = {0.0, 0.0, 0.0};
  ViewDir u{};
  if (vis) {
    double mu[3], gg[9];
    for (int k = 0; k < 3; ++k) mu[k] = (double)params[(int64_t)k * n + i];
    for (int k = 0; k < 9; ++k) gg[k] = (double)g2d[i * 9 + k];
    u = view_dir(mu, cam);
    color_grad(gg, clampm[i], drgb);
  }
  // SH terms k = 1..15 (rows 11 + 3k + ch), software-pipelined: the rows of
  // term k + 1 are loaded before term k is updated and stored.  The
  // arithmetic is that of the projection backward (SH part) followed by Adam.
  struct Rows { float p[3], m[3], v[3], g[3]; };
  auto load = [&](int k, Rows& r) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const int64_t idx = (int64_t)(11 + 3 * k + ch) * n + i;
      r.p[ch] = params[idx];
      r.m[ch] = m[mom(i, 11 + 3 * k + ch)];
      r.v[ch] = v[mom(i, 11 + 3 * k + ch)];
      r.g[ch] = grad_prev != nullptr ? grad_prev[idx] : 0.f;
    }
  };
  Rows cur, nxt;
  load(1, cur);
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    if (k + 1 < 16) load(k + 1, nxt);
    __builtin_amdgcn_sched_barrier(0);
    double grad[3] = {0.0, 0.0, 0.0};
    if (vis && k < nk) {
      double Yk, d0, d1, d2;
      sh_term(k, u.ux, u.uy, u.uz, Yk, d0, d1, d2);
      double gk = 0.0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gk += (double)cur.p[ch] * drgb[ch];
        grad[ch] = Yk * drgb[ch];
      }
      dL_du[0] += d0 * gk;
      dL_du[1] += d1 * gk;
      dL_du[2] += d2 * gk;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const int row = 11 + 3 * k + ch;
      const int64_t idx = (int64_t)row * n + i;
      float pp = cur.p[ch], mm = cur.m[ch], vv = cur.v[ch];
      const float gf = grad_prev != nullptr ? cur.g[ch] + (float)grad[ch] : (float)grad[ch];
      adam_elem(pp, gf, mm, vv, row_lr_bc1(o, row), o);
      params[idx] = pp;
      m[mom(i, row)] = mm;
      v[mom(i, row)] = vv;
    }
    if (k + 1 < 16) cur = nxt;
  }
  if (vis)
    for (int k = 0; k < 3; ++k) dL_du_out[i * 3 + k] = dL_du[k];
}

// Rows 0-13 of every Gaussian the wave updates: parameters, moments and (when
// there is one) the earlier views' gradient are copied into LDS by the
// memory system while the chain rule runs, so the update does not wait for
// them at the end.  One wave per workgroup; LDS holds kPre (or kPre + 14)
// rows of 64 floats.
constexpr int kGeoRows = 14;
constexpr int kPre = 3 * kGeoRows;  // params, m, v

__global__ void __launch_bounds__(kWave) geom_lm_kernel(
    float* params, int64_t n, CamArgs cam, int sh_degree, double z_near, double dil,
    const int* __restrict__ radius, const uint8_t* __restrict__ clampm, const float* __restrict__ g2d,
    const float* __restrict__ grad_prev, float* __restrict__ m, float* __restrict__ v,
    const uint8_t* __restrict__ touched, OptArgs o, const double* __restrict__ dL_du_in) {
  extern __shared__ float s_rows[];  // [kPre (+ 14)][64]
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kWave + lane;
  const int64_t ic = i < n ? i : n - 1;  // lanes past the end load a valid element
  // asynchronous row copies global -> LDS: lane l's value lands at [row][l]
  // (params and the gradient row-major [59][n], the moments Gaussian-major)
  const float* srcs[4] = {params, m, v, grad_prev};
  const int n_src = grad_prev != nullptr ? 4 : 3;
  for (int q = 0; q < n_src; ++q)
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) {
      const int64_t at_q = q == 1 || q == 2 ? mom(ic, r) : (int64_t)r * n + ic;
      __builtin_amdgcn_global_load_lds(srcs[q] + at_q, s_rows + (q * kGeoRows + r) * kWave, 4, 0, 0);
    }

  const bool live = i < n && (touched == nullptr || touched[i] != 0);  // untouched: nothing changes
  float gl[kGeoRows];  // this view's gradient of rows 0-13, rounded to float
  if (live) {
    auto sink = [&](int row, double val) { gl[row] = (float)val; };
    if (radius[i] != 0) {
      Geom g;
      geometry(params, n, i, cam, z_near, dil, g);
      double gg[9];
      for (int k = 0; k < 9; ++k) gg[k] = (double)g2d[i * 9 + k];
      const ViewDir u = view_dir(g.mu, cam);
      double drgb[3];
      color_grad(gg, clampm[i], drgb);
      double dc_du[3] = {0.0, 0.0, 0.0};  // the DC basis is constant: no dL/du
      sh_backward(params, n, i, u, drgb, n_sh(sh_degree), 0, 1, dc_du, sink);
      const double dL_du[3] = {dL_du_in[i * 3], dL_du_in[i * 3 + 1], dL_du_in[i * 3 + 2]};
      geom_backward(params, n, i, cam, g, gg, u, dL_du, sink);
    } else {
#pragma unroll
      for (int r = 0; r < kGeoRows; ++r) gl[r] = 0.f;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // the row copies have landed
  __syncthreads();
  if (!live) return;
  auto at = [&](int q, int row) -> float& { return s_rows[(q * kGeoRows + row) * kWave + lane]; };
  // the step's gradient as the unfused path stores it
  if (grad_prev != nullptr)
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) gl[r] = at(3, r) + gl[r];
  auto store = [&](int row, float pp, float mm, float vv) {
    m[mom(i, row)] = mm;
    v[mom(i, row)] = vv;
    params[(int64_t)row * n + i] = pp;
  };
  if (o.lm_mode == 2) {
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) {
      float pp = at(0, r), mm = at(1, r), vv = at(2, r);
      adam_elem(pp, gl[r], mm, vv, row_lr_bc1(o, r), o);
      store(r, pp, mm, vv);
    }
    return;
  }
  float pg[10], mg[10], vg[10], gg[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    pg[k] = at(0, kGeomRows[k]);
    mg[k] = at(1, kGeomRows[k]);
    vg[k] = at(2, kGeomRows[k]);
    gg[k] = gl[kGeomRows[k]];
  }
  lm_block<10>(pg, mg, vg, kGeomRows, gg, o);
#pragma unroll
  for (int k = 0; k < 10; ++k) store(kGeomRows[k], pg[k], mg[k], vg[k]);
  float pa[4], ma[4], va[4], ga[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pa[k] = at(0, kAppRows[k]);
    ma[k] = at(1, kAppRows[k]);
    va[k] = at(2, kAppRows[k]);
    ga[k] = gl[kAppRows[k]];
  }
  lm_block<4>(pa, ma, va, kAppRows, ga, o);
#pragma unroll
  for (int k = 0; k < 4; ++k) store(kAppRows[k], pa[k], ma[k], va[k]);
}

// ---- every view of a step in one pass: the chain rule of each view is
// evaluated in registers and summed before the update, so neither the
// earlier views' projection backward nor their gradient array is needed.
// The SH kernel leaves, per Gaussian, the mean's gradient through the view
// directions of the SH terms of degree >= 1 (three doubles in the
// workspace) for the geometry kernel.
constexpr int kMaxViews = 16;

struct ViewSet {
  CamArgs cam[kMaxViews];
  const int* radius[kMaxViews];
  const uint8_t* clampm[kMaxViews];
  const float* g2d[kMaxViews];
  int nv;
};

// SH rows in three groups of five terms (15 rows), one wave per group: a
// block holds 64 Gaussians in three waves.  Each wave sums its rows'
// gradients over the views (each view's value rounded to float and added
// in view order, as the per-view path's gradient array sums them), updates
// its rows, and forms its share of the mean's gradient through u:
// (I - u u^T) dL/du / |mu - centre| per view, summed in FP64.  The block
// adds the three shares in group order and stores the sum.
// The update touches few Gaussians (those composited at a sample: ~6% of
// 1.5M in the full step, spread at random), so a wave over 64 consecutive
// Gaussians would run its FP64 work for a handful of live lanes.  A
// workgroup therefore takes a window of kWindow consecutive Gaussians,
// lists the touched ones in LDS (ballots over the window's flags, in
// order) and gives each wave lane one listed Gaussian, 64 at a time.  The
// window's rows span 16 cache lines each, so its loads touch the lines a
// streaming pass would, with a fraction of the waves.
constexpr int kWindow = 512;

// The touched Gaussians of [w0, w0 + kWindow) as offsets from w0, in
// order, into lds[0..c); returns c (wave-uniform).  Every Gaussian when
// touched is null.  Called by one whole wave.
__device__ __forceinline__ int window_list(const uint8_t* __restrict__ touched, int64_t n, int64_t w0,
                                           uint16_t* __restrict__ lds) {
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  int c = 0;
#pragma unroll
  for (int r = 0; r < kWindow / kWave; ++r) {
    const int64_t i = w0 + r * kWave + lane;
    const bool t = i < n && (touched == nullptr || touched[i] != 0);
    const uint64_t mask = __ballot(t);
    if (t) lds[c + __popcll(mask & below)] = (uint16_t)(r * kWave + lane);
    c += __popcll(mask);
  }
  return c;
}

constexpr int kShGroups = 3;

template <int kDeg, int kGrp>
__device__ __forceinline__ void sh_group_views(float* params, int64_t n, const ViewSet& vs, float* __restrict__ m,
                                               float* __restrict__ v, bool live, int64_t i, const OptArgs& o,
                                               double (&dmu)[3]) {
#pragma clang fp contract(off)
  constexpr int nk = (kDeg + 1) * (kDeg + 1);
  constexpr bool kTerms = 1 + 5 * kGrp < nk;
  if (!live) return;
  float cf[15], gs[15];
#pragma unroll
  for (int r = 0; r < 15; ++r) {
    cf[r] = params[(int64_t)(14 + 15 * kGrp + r) * n + i];
    gs[r] = 0.f;
  }
  if (kTerms) {
    double mu[3];
    for (int k = 0; k < 3; ++k) mu[k] = (double)params[(int64_t)k * n + i];
    for (int j = 0; j < vs.nv; ++j) {
      if (vs.radius[j][i] == 0) continue;
      double gg[9];
      for (int k = 0; k < 9; ++k) gg[k] = (double)vs.g2d[j][i * 9 + k];
      const ViewDir u = view_dir(mu, vs.cam[j]);
      double drgb[3];
      color_grad(gg, vs.clampm[j][i], drgb);
      double du[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        const int k = 1 + 5 * kGrp + t;
        if (k >= nk) break;
        double Yk, d0, d1, d2;
        sh_term(k, u.ux, u.uy, u.uz, Yk, d0, d1, d2);
        double gk = 0.0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          gk += (double)cf[3 * t + ch] * drgb[ch];
          gs[3 * t + ch] += (float)(Yk * drgb[ch]);
        }
        du[0] += d0 * gk;
        du[1] += d1 * gk;
        du[2] += d2 * gk;
      }
      const double udot = u.ux * du[0] + u.uy * du[1] + u.uz * du[2];
      const double inv = 1.0 / u.dn;
      dmu[0] += (du[0] - u.ux * udot) * inv;
      dmu[1] += (du[1] - u.uy * udot) * inv;
      dmu[2] += (du[2] - u.uz * udot) * inv;
    }
  }
#pragma unroll
  for (int r = 0; r < 15; ++r) {
    const int row = 14 + 15 * kGrp + r;
    float pp = cf[r], mm = m[mom(i, row)], vv = v[mom(i, row)];
    adam_elem(pp, gs[r], mm, vv, row_lr_bc1(o, row), o);
    params[(int64_t)row * n + i] = pp;
    m[mom(i, row)] = mm;
    v[mom(i, row)] = vv;
  }
}

template <int kDeg>
__global__ void __launch_bounds__(kShGroups * kWave) sh_rest_views_kernel(float* params, int64_t n, ViewSet vs,
                                                                           float* __restrict__ m,
                                                                           float* __restrict__ v,
                                                                           const uint8_t* __restrict__ touched,
                                                                           OptArgs o, double* __restrict__ dmu_out) {
  __shared__ double share[kShGroups - 1][3][kWave];
  __shared__ uint16_t wl[kShGroups][kWindow];  // each wave lists the window itself (no barrier)
  const int grp = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  const int64_t w0 = (int64_t)blockIdx.x * kWindow;
  const int c = window_list(touched, n, w0, wl[grp]);  // the same count in every wave
  for (int g = 0; g < c; g += kWave) {
    // untouched Gaussians are not listed: their parameters and moments stay
    const bool live = g + lane < c;
    const int64_t i = live ? w0 + wl[grp][g + lane] : 0;
    double dmu[3] = {0.0, 0.0, 0.0};
    if (grp == 0)
      sh_group_views<kDeg, 0>(params, n, vs, m, v, live, i, o, dmu);
    else if (grp == 1)
      sh_group_views<kDeg, 1>(params, n, vs, m, v, live, i, o, dmu);
    else
      sh_group_views<kDeg, 2>(params, n, vs, m, v, live, i, o, dmu);
    if (grp > 0)
      for (int k = 0; k < 3; ++k) share[grp - 1][k][lane] = dmu[k];
    __syncthreads();
    if (grp == 0 && live)
      for (int k = 0; k < 3; ++k) dmu_out[i * 3 + k] = (dmu[k] + share[0][k][lane]) + share[1][k][lane];
    __syncthreads();  // the shares are read before the next group writes them
  }
}

// Rows 0-13 (mean, log-scale, quaternion, opacity, SH DC) of one Gaussian
// summed over the views.  The shape (scales, rotation, 3D covariance) is
// formed once; per view only the projection Jacobian, the 2D covariance
// and the backward through them run.  The maps from the summed covariance
// gradient to the scale and quaternion rows, from the summed opacity
// gradient to its logit and from the summed colour gradient to the DC rows
// are linear, so each is applied once to the sum.  Products by reciprocals
// stand for the divisions of the per-view chain rule.
__device__ __forceinline__ void geom_views_grad(const float* params, int64_t n, const ViewSet& vs, int64_t i,
                                                double dil, const double (&dmu_sh)[3], double (&gr)[kGeoRows]) {
#pragma clang fp contract(off)
  // the shape: only the 3D covariance and the scales stay live through the
  // view loop; rotation and M are formed again for the linear tail
  const double mu[3] = {params[i], params[n + i], params[2 * n + i]};
  double s[3];
  for (int k = 0; k < 3; ++k) s[k] = exp((double)params[(int64_t)(3 + k) * n + i]);
  auto quat = [&](double (&q)[4]) {
    const double qw = params[6 * n + i], qx = params[7 * n + i], qy = params[8 * n + i], qz = params[9 * n + i];
    const double iq = 1.0 / sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    q[0] = qw * iq;
    q[1] = qx * iq;
    q[2] = qy * iq;
    q[3] = qz * iq;
    return iq;
  };
  auto rot = [](const double (&q)[4], double (&Rq)[3][3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    Rq[0][0] = 1.0 - 2.0 * (y * y + z * z);
    Rq[0][1] = 2.0 * (x * y - w * z);
    Rq[0][2] = 2.0 * (x * z + w * y);
    Rq[1][0] = 2.0 * (x * y + w * z);
    Rq[1][1] = 1.0 - 2.0 * (x * x + z * z);
    Rq[1][2] = 2.0 * (y * z - w * x);
    Rq[2][0] = 2.0 * (x * z - w * y);
    Rq[2][1] = 2.0 * (y * z + w * x);
    Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
  };
  double S[3][3];
  {
    double q[4], Rq[3][3], M[3][3];
    (void)quat(q);
    rot(q, Rq);
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) M[r][k] = Rq[r][k] * s[k];
    for (int r = 0; r < 3; ++r)
      for (int k = r; k < 3; ++k) S[r][k] = (M[r][0] * M[k][0] + M[r][1] * M[k][1]) + M[r][2] * M[k][2];
    for (int r = 1; r < 3; ++r)
      for (int k = 0; k < r; ++k) S[r][k] = S[k][r];
  }

  double dS[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  double dmu[3] = {dmu_sh[0], dmu_sh[1], dmu_sh[2]};
  double dop = 0.0, dc[3] = {0.0, 0.0, 0.0};
#pragma clang loop unroll(disable)
  for (int j = 0; j < vs.nv; ++j) {
    if (vs.radius[j][i] == 0) continue;  // listed views only (in front of the camera)
    const CamArgs& cam = vs.cam[j];
    double gg[9];
    for (int k = 0; k < 9; ++k) gg[k] = (double)vs.g2d[j][i * 9 + k];
    double t[3];
    for (int r = 0; r < 3; ++r)
      t[r] = ((cam.R[r * 3 + 0] * mu[0] + cam.R[r * 3 + 1] * mu[1]) + cam.R[r * 3 + 2] * mu[2]) + cam.t[r];
    const double tx = t[0], ty = t[1];
    const double itz = 1.0 / t[2], itz2 = itz * itz, itz3 = itz2 * itz;
    const double J00 = cam.fx * itz, J02 = -(cam.fx * tx) * itz2, J11 = cam.fy * itz, J12 = -(cam.fy * ty) * itz2;
    double T[2][3];
    for (int k = 0; k < 3; ++k) {
      T[0][k] = J00 * cam.R[0 * 3 + k] + J02 * cam.R[2 * 3 + k];
      T[1][k] = J11 * cam.R[1 * 3 + k] + J12 * cam.R[2 * 3 + k];
    }
    double TS[2][3];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) TS[r][k] = (T[r][0] * S[0][k] + T[r][1] * S[1][k]) + T[r][2] * S[2][k];
    const double a = ((TS[0][0] * T[0][0] + TS[0][1] * T[0][1]) + TS[0][2] * T[0][2]) + dil;
    const double b = (TS[0][0] * T[1][0] + TS[0][1] * T[1][1]) + TS[0][2] * T[1][2];
    const double c = ((TS[1][0] * T[1][0] + TS[1][1] * T[1][1]) + TS[1][2] * T[1][2]) + dil;
    const double idet = 1.0 / (a * c - b * b), id2 = idet * idet;

    // centre
    double dt[3];
    dt[0] = gg[0] * cam.fx * itz;
    dt[1] = gg[1] * cam.fy * itz;
    dt[2] = gg[0] * (-cam.fx * tx * itz2) + gg[1] * (-cam.fy * ty * itz2);
    // conic (c, -b, a) / det -> 2D covariance entries
    const double gca = gg[2], gcb = gg[3], gcc = gg[4];
    const double dLa = gca * (-c * c * id2) + gcb * (b * c * id2) + gcc * (idet - a * c * id2);
    const double dLb = gca * (2.0 * b * c * id2) + gcb * (-idet - 2.0 * b * b * id2) + gcc * (2.0 * a * b * id2);
    const double dLc = gca * (idet - a * c * id2) + gcb * (a * b * id2) + gcc * (-a * a * id2);
    const double G[2][2] = {{dLa, 0.5 * dLb}, {0.5 * dLb, dLc}};
    double GT[2][3];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) GT[r][k] = G[r][0] * T[0][k] + G[r][1] * T[1][k];
    // dSigma += T^T G T ; dT = 2 G T Sigma
    for (int r = 0; r < 3; ++r)
      for (int k = r; k < 3; ++k) dS[r][k] += T[0][r] * GT[0][k] + T[1][r] * GT[1][k];
    double dT[2][3];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) dT[r][k] = 2.0 * (GT[r][0] * S[0][k] + GT[r][1] * S[1][k] + GT[r][2] * S[2][k]);
    auto dJ = [&](int r, int k) {
      return dT[r][0] * cam.R[k * 3 + 0] + dT[r][1] * cam.R[k * 3 + 1] + dT[r][2] * cam.R[k * 3 + 2];
    };
    const double dJ00 = dJ(0, 0), dJ02 = dJ(0, 2), dJ11 = dJ(1, 1), dJ12 = dJ(1, 2);
    dt[0] += dJ02 * (-cam.fx * itz2);
    dt[1] += dJ12 * (-cam.fy * itz2);
    dt[2] += dJ00 * (-cam.fx * itz2) + dJ02 * (2.0 * cam.fx * tx * itz3) + dJ11 * (-cam.fy * itz2) +
             dJ12 * (2.0 * cam.fy * ty * itz3);
    for (int k = 0; k < 3; ++k)
      dmu[k] += cam.R[0 * 3 + k] * dt[0] + cam.R[1 * 3 + k] * dt[1] + cam.R[2 * 3 + k] * dt[2];
    dop += gg[5];
    double drgb[3];
    color_grad(gg, vs.clampm[j][i], drgb);
    for (int ch = 0; ch < 3; ++ch) dc[ch] += drgb[ch];
  }

  // Sigma = M M^T, M = R(q) diag(s): scale and quaternion rows
  for (int r = 1; r < 3; ++r)
    for (int k = 0; k < r; ++k) dS[r][k] = dS[k][r];
  double q[4], Rq[3][3], M[3][3];
  const double iq = quat(q);
  rot(q, Rq);
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) M[r][k] = Rq[r][k] * s[k];
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  double dM[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) dM[r][k] = 2.0 * (dS[r][0] * M[0][k] + dS[r][1] * M[1][k] + dS[r][2] * M[2][k]);
  double dR[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ds = Rq[0][k] * dM[0][k] + Rq[1][k] * dM[1][k] + Rq[2][k] * dM[2][k];
    gr[3 + k] = ds * s[k];
    for (int r = 0; r < 3; ++r) dR[r][k] = dM[r][k] * s[k];
  }
  double dq[4];
  dq[0] = 2.0 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
  dq[1] = 2.0 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0 * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                 w * dR[2][1] - 2.0 * x * dR[2][2]);
  dq[2] = 2.0 * (-2.0 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                 z * dR[2][1] - 2.0 * y * dR[2][2]);
  dq[3] = 2.0 * (-2.0 * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.0 * z * dR[1][1] +
                 y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  const double qdot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  gr[6] = (dq[0] - w * qdot) * iq;
  gr[7] = (dq[1] - x * qdot) * iq;
  gr[8] = (dq[2] - y * qdot) * iq;
  gr[9] = (dq[3] - z * qdot) * iq;
  for (int k = 0; k < 3; ++k) gr[k] = dmu[k];
  const double op = 1.0 / (1.0 + exp(-(double)params[10 * n + i]));
  gr[10] = dop * op * (1.0 - op);
  for (int ch = 0; ch < 3; ++ch) gr[11 + ch] = kC0 * dc[ch];
}

__device__ __forceinline__ void geom_lm_views_one(float* params, int64_t n, const ViewSet& vs, double dil,
                                                  float* __restrict__ m, float* __restrict__ v, const OptArgs& o,
                                                  const double* __restrict__ dmu_sh, int64_t i);

__global__ void __launch_bounds__(64) geom_lm_views_kernel(float* params, int64_t n, ViewSet vs, double dil,
                                                           float* __restrict__ m, float* __restrict__ v,
                                                           const uint8_t* __restrict__ touched, OptArgs o,
                                                           const double* __restrict__ dmu_sh) {
  __shared__ uint16_t wl[kWindow];
  const int64_t w0 = (int64_t)blockIdx.x * kWindow;
  const int c = window_list(touched, n, w0, wl);
  for (int g = 0; g < c; g += kWave)
    if (g + (int)threadIdx.x < c) geom_lm_views_one(params, n, vs, dil, m, v, o, dmu_sh, w0 + wl[g + threadIdx.x]);
}

__device__ __forceinline__ void geom_lm_views_one(float* params, int64_t n, const ViewSet& vs, double dil,
                                                  float* __restrict__ m, float* __restrict__ v, const OptArgs& o,
                                                  const double* __restrict__ dmu_sh, int64_t i) {
  const double dsh[3] = {dmu_sh[i * 3], dmu_sh[i * 3 + 1], dmu_sh[i * 3 + 2]};
  double gsum[kGeoRows];
  geom_views_grad(params, n, vs, i, dil, dsh, gsum);
  auto store = [&](int row, float pp, float mm, float vv) {
    m[mom(i, row)] = mm;
    v[mom(i, row)] = vv;
    params[(int64_t)row * n + i] = pp;
  };
  auto load = [&](int row, float& pp, float& mm, float& vv) {
    pp = params[(int64_t)row * n + i];
    mm = m[mom(i, row)];
    vv = v[mom(i, row)];
  };
  if (o.lm_mode == 2) {
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) {
      float pp, mm, vv;
      load(r, pp, mm, vv);
      adam_elem(pp, (float)gsum[r], mm, vv, row_lr_bc1(o, r), o);
      store(r, pp, mm, vv);
    }
    return;
  }
  float pg[10], mg[10], vg[10], gq[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    load(kGeomRows[k], pg[k], mg[k], vg[k]);
    gq[k] = (float)gsum[kGeomRows[k]];
  }
  lm_block<10>(pg, mg, vg, kGeomRows, gq, o);
#pragma unroll
  for (int k = 0; k < 10; ++k) store(kGeomRows[k], pg[k], mg[k], vg[k]);
  float pa[4], ma[4], va[4], ga[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    load(kAppRows[k], pa[k], ma[k], va[k]);
    ga[k] = (float)gsum[kAppRows[k]];
  }
  lm_block<4>(pa, ma, va, kAppRows, ga, o);
#pragma unroll
  for (int k = 0; k < 4; ++k) store(kAppRows[k], pa[k], ma[k], va[k]);
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_project_bwd_optimizer_views_workspace_size(int64_t n, int32_t n_views) {
  if (n < 0 || n_views < 0) return 0;
  return align_up((size_t)(3 * std::max<int64_t>(n, 1)) * sizeof(double), 256);
}

extern "C" int32_t tgs_project_bwd_optimizer_step_views(float* params, int64_t n, int32_t n_views,
                                                        const tgs_camera* cams, const tgs_raster_params* rp,
                                                        const int32_t* const* radius, const uint8_t* const* clamp,
                                                        const float* const* g2d, float* m, float* v,
                                                        const uint8_t* touched, const tgs_optim_params* op,
                                                        int64_t step, void* ws, size_t ws_bytes, void* stream) {
  const char* who = "tgs_project_bwd_optimizer_step_views";
  TGS_REQUIRE(n >= 0, "%s: n < 0", who);
  TGS_REQUIRE(n_views >= 1 && n_views <= kMaxViews, "%s: %d views not in 1..%d", who, n_views, kMaxViews);
  TGS_REQUIRE(cams && radius && clamp && g2d, "%s: null view arrays", who);
  if (int32_t e = check_raster_params(rp)) return e;
  OptArgs o;
  if (int32_t e = make_opt_args(op, step, who, o)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && m && v && ws, "%s: null pointer", who);
  ViewSet vs;
  vs.nv = n_views;
  for (int j = 0; j < n_views; ++j) {
    TGS_REQUIRE(cams[j].width > 0 && cams[j].height > 0, "%s: bad camera %d", who, j);
    TGS_REQUIRE(radius[j] && clamp[j] && g2d[j], "%s: null pointer of view %d", who, j);
    vs.cam[j] = make_cam(&cams[j]);
    vs.radius[j] = radius[j];
    vs.clampm[j] = clamp[j];
    vs.g2d[j] = g2d[j];
  }
  for (int j = n_views; j < kMaxViews; ++j) {
    vs.cam[j] = vs.cam[0];
    vs.radius[j] = nullptr;
    vs.clampm[j] = nullptr;
    vs.g2d[j] = nullptr;
  }
  const size_t need = tgs_project_bwd_optimizer_views_workspace_size(n, n_views);
  TGS_REQUIRE(ws_bytes >= need, "%s: workspace %zu bytes < %zu", who, ws_bytes, need);
  TGS_REQUIRE(((uintptr_t)ws & 7) == 0, "%s: workspace must be 8-byte aligned", who);
  hipStream_t s = as_stream(stream);
  const dim3 grid((unsigned)ceil_div(n, kWindow));
#define TGS_SH_VIEWS(D)                                                                                        \
  hipLaunchKernelGGL(sh_rest_views_kernel<D>, grid, dim3(kShGroups * kWave), 0, s, params, n, vs, m, v, touched, \
                     o, (double*)ws)
  switch (rp->sh_degree) {
    case 0: TGS_SH_VIEWS(0); break;
    case 1: TGS_SH_VIEWS(1); break;
    case 2: TGS_SH_VIEWS(2); break;
    default: TGS_SH_VIEWS(3); break;
  }
#undef TGS_SH_VIEWS
  hipLaunchKernelGGL(geom_lm_views_kernel, grid, dim3(kWave), 0, s, params, n, vs, (double)rp->dilation, m, v,
                     touched, o, (const double*)ws);
  return hip_status(who);
}

extern "C" size_t tgs_project_bwd_optimizer_workspace_size(int64_t n) {
  return n < 0 ? 0 : align_up((size_t)(3 * std::max<int64_t>(n, 1)) * sizeof(double), 256);
}

extern "C" int32_t tgs_project_bwd_optimizer_step(float* params, int64_t n, const tgs_camera* cam,
                                                  const tgs_raster_params* rp, const int32_t* radius,
                                                  const uint8_t* clamp, const float* g2d,
                                                  const float* grad_prev, float* m, float* v,
                                                  const uint8_t* touched, const tgs_optim_params* op,
                                                  int64_t step, void* ws, size_t ws_bytes, void* stream) {
  const char* who = "tgs_project_bwd_optimizer_step";
  TGS_REQUIRE(n >= 0, "%s: n < 0", who);
  TGS_REQUIRE(cam != nullptr && cam->width > 0 && cam->height > 0, "%s: bad camera", who);
  if (int32_t e = check_raster_params(rp)) return e;
  OptArgs o;
  if (int32_t e = make_opt_args(op, step, who, o)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && radius && clamp && g2d && m && v && ws, "%s: null pointer", who);
  TGS_REQUIRE(ws_bytes >= tgs_project_bwd_optimizer_workspace_size(n), "%s: workspace %zu bytes < %zu", who,
              ws_bytes, tgs_project_bwd_optimizer_workspace_size(n));
  TGS_REQUIRE(((uintptr_t)ws & 7) == 0, "%s: workspace must be 8-byte aligned", who);
  const CamArgs ca = make_cam(cam);
  hipStream_t s = as_stream(stream);
  const dim3 grid((unsigned)ceil_div(n, 256));
#define TGS_SH_REST(D)                                                                                \
  hipLaunchKernelGGL(sh_rest_kernel<D>, grid, dim3(256), 0, s, params, n, ca, radius, clamp, g2d, grad_prev, m, v, \
                     touched, o, (double*)ws)
  switch (rp->sh_degree) {
    case 0: TGS_SH_REST(0); break;
    case 1: TGS_SH_REST(1); break;
    case 2: TGS_SH_REST(2); break;
    default: TGS_SH_REST(3); break;
  }
#undef TGS_SH_REST
  const size_t lds = (size_t)(grad_prev != nullptr ? kPre + kGeoRows : kPre) * kWave * sizeof(float);
  hipLaunchKernelGGL(geom_lm_kernel, dim3((unsigned)ceil_div(n, kWave)), dim3(kWave), lds, s, params, n, ca,
                     rp->sh_degree, (double)rp->z_near, (double)rp->dilation, radius, clamp, g2d, grad_prev, m, v,
                     touched, o, (const double*)ws);
  return hip_status(who);
}
