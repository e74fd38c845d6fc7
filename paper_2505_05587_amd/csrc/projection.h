// fp64 projection of one Gaussian through one camera (Sec. 3: Eq. sigma_3D,
// Eq. sigma_2D and the footnote on Pi).  Used by the projection kernel and,
// to recompute the same quantities, by the projection backward.
//
// Every operation that decides something discrete (culling, footprint
// radius, tile rectangle, depth key, colour clamp) is evaluated in fp64 with
// contraction disabled and a fixed operation order, so the decisions are
// reproducible from the fp32 inputs.
#pragma once

#include "common.h"

namespace sg {

// Real spherical harmonics, Condon-Shortley phase, index k = l*l + l + m,
// written as polynomials on the unit sphere.  Normalisation constants:
constexpr double kSH0 = 0.28209479177387814;   // sqrt(1/(4 pi))
constexpr double kSH1 = 0.4886025119029199;    // sqrt(3/(4 pi))
constexpr double kSH2a = 1.0925484305920792;   // sqrt(15/pi) / 2
constexpr double kSH2b = 0.31539156525252005;  // sqrt(5/pi) / 4
constexpr double kSH2c = 0.5462742152960396;   // sqrt(15/pi) / 4
constexpr double kSH3a = 0.5900435899266435;   // sqrt(35/(2 pi)) / 4
constexpr double kSH3b = 2.890611442640554;    // sqrt(105/pi) / 2
constexpr double kSH3c = 0.4570457994644658;   // sqrt(21/(2 pi)) / 4
constexpr double kSH3d = 0.3731763325901154;   // sqrt(7/pi) / 4
constexpr double kSH3e = 1.445305721320277;    // sqrt(105/pi) / 4

template <class T>
SG_DEV void sh_eval(int deg, T x, T y, T z, T* Y) {
  Y[0] = T(kSH0);
  if (deg < 1) return;
  Y[1] = T(-kSH1) * y;
  Y[2] = T(kSH1) * z;
  Y[3] = T(-kSH1) * x;
  if (deg < 2) return;
  const T xx = x * x, yy = y * y, zz = z * z;
  Y[4] = T(kSH2a) * x * y;
  Y[5] = T(-kSH2a) * y * z;
  Y[6] = T(kSH2b) * (T(2) * zz - xx - yy);
  Y[7] = T(-kSH2a) * x * z;
  Y[8] = T(kSH2c) * (xx - yy);
  if (deg < 3) return;
  Y[9] = T(-kSH3a) * y * (T(3) * xx - yy);
  Y[10] = T(kSH3b) * x * y * z;
  Y[11] = T(-kSH3c) * y * (T(4) * zz - xx - yy);
  Y[12] = T(kSH3d) * z * (T(2) * zz - T(3) * xx - T(3) * yy);
  Y[13] = T(-kSH3c) * x * (T(4) * zz - xx - yy);
  Y[14] = T(kSH3e) * z * (xx - yy);
  Y[15] = T(-kSH3a) * x * (xx - T(3) * yy);
}

// g += sum_k w_k * grad_(x,y,z) Y_k   (polynomial gradient; the caller
// projects it onto the sphere's tangent plane)
template <class T>
SG_DEV void sh_grad(int deg, T x, T y, T z, const T* w, T g[3]) {
  if (deg < 1) return;
  g[1] += T(-kSH1) * w[1];
  g[2] += T(kSH1) * w[2];
  g[0] += T(-kSH1) * w[3];
  if (deg < 2) return;
  const T xx = x * x, yy = y * y, zz = z * z;
  g[0] += T(kSH2a) * y * w[4];
  g[1] += T(kSH2a) * x * w[4];
  g[1] += T(-kSH2a) * z * w[5];
  g[2] += T(-kSH2a) * y * w[5];
  g[0] += T(-2.0 * kSH2b) * x * w[6];
  g[1] += T(-2.0 * kSH2b) * y * w[6];
  g[2] += T(4.0 * kSH2b) * z * w[6];
  g[0] += T(-kSH2a) * z * w[7];
  g[2] += T(-kSH2a) * x * w[7];
  g[0] += T(2.0 * kSH2c) * x * w[8];
  g[1] += T(-2.0 * kSH2c) * y * w[8];
  if (deg < 3) return;
  // Y9 = -a (3 x^2 y - y^3)
  g[0] += T(-6.0 * kSH3a) * x * y * w[9];
  g[1] += T(-kSH3a) * (T(3) * xx - T(3) * yy) * w[9];
  // Y10 = b x y z
  g[0] += T(kSH3b) * y * z * w[10];
  g[1] += T(kSH3b) * x * z * w[10];
  g[2] += T(kSH3b) * x * y * w[10];
  // Y11 = -c (4 y z^2 - x^2 y - y^3)
  g[0] += T(2.0 * kSH3c) * x * y * w[11];
  g[1] += T(-kSH3c) * (T(4) * zz - xx - T(3) * yy) * w[11];
  g[2] += T(-8.0 * kSH3c) * y * z * w[11];
  // Y12 = d (2 z^3 - 3 x^2 z - 3 y^2 z)
  g[0] += T(-6.0 * kSH3d) * x * z * w[12];
  g[1] += T(-6.0 * kSH3d) * y * z * w[12];
  g[2] += T(kSH3d) * (T(6) * zz - T(3) * xx - T(3) * yy) * w[12];
  // Y13 = -c (4 x z^2 - x^3 - x y^2)
  g[0] += T(-kSH3c) * (T(4) * zz - T(3) * xx - yy) * w[13];
  g[1] += T(2.0 * kSH3c) * x * y * w[13];
  g[2] += T(-8.0 * kSH3c) * x * z * w[13];
  // Y14 = e (x^2 z - y^2 z)
  g[0] += T(2.0 * kSH3e) * x * z * w[14];
  g[1] += T(-2.0 * kSH3e) * y * z * w[14];
  g[2] += T(kSH3e) * (xx - yy) * w[14];
  // Y15 = -a (x^3 - 3 x y^2)
  g[0] += T(-kSH3a) * (T(3) * xx - T(3) * yy) * w[15];
  g[1] += T(6.0 * kSH3a) * x * y * w[15];
}

// Smallest value of q(d) = a dx^2 + 2 b dx dy + c dy^2, d = x - m, over the box
// [x0, x1] x [y0, y1] for a positive-definite conic: 0 when m lies inside,
// otherwise the smallest of the four edge minima, each the one-dimensional
// minimiser clamped to its edge (q is convex).  fp64, fixed operation order.
SG_DEV double box_min_q(double a, double b, double c, double mx, double my, double x0, double x1, double y0,
                        double y1) {
#pragma clang fp contract(off)
  if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.0;
  double best = INFINITY;
  for (int e = 0; e < 2; ++e) {
    const double dx = (e == 0 ? x0 : x1) - mx;
    double dy = -(b * dx) / c;
    if (dy < y0 - my) dy = y0 - my;
    if (dy > y1 - my) dy = y1 - my;
    double q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
    if (q < best) best = q;
    const double ey = (e == 0 ? y0 : y1) - my;
    double ex = -(b * ey) / a;
    if (ex < x0 - mx) ex = x0 - mx;
    if (ex > x1 - mx) ex = x1 - mx;
    q = a * ex * ex + 2.0 * b * ex * ey + c * ey * ey;
    if (q < best) best = q;
  }
  return best;
}

// A tile belongs to a Gaussian's footprint when its box of pixel centres
// meets the ellipse q <= radius_sigmas^2 (1e-6 relative slack).  Evaluated on
// the stored float32 mean and conic, so that any consumer of the record (the
// sort's walk and emission here, the oracle's tile lists) takes the same
// decision.
SG_DEV bool tile_hit_fp64(float mx, float my, float a, float b, float c, const steepgs_opts& opt, int tx, int ty) {
#pragma clang fp contract(off)
  const double k2 = (double)opt.radius_sigmas * (double)opt.radius_sigmas;
  const double x0 = (double)tx * opt.tile_w, y0 = (double)ty * opt.tile_h;
  const double q = box_min_q((double)a, (double)b, (double)c, (double)mx, (double)my, x0, x0 + (opt.tile_w - 1), y0,
                             y0 + (opt.tile_h - 1));
  return q <= k2 * (1.0 + 1e-6);
}

// The same decision, certified in fp32 where it can be.  With the mean
// outside the box the minimum lies on a face seen from the mean (the segment
// from the mean to any point of the box enters it through such a face, and
// the quadratic grows along it), so only those faces -- at most one across x
// and one across y -- are evaluated.  Each face minimum is computed in fp32
// together with M = a dx^2 + 2|b dx dy| + c dy^2, which bounds its rounding
// error by ~10 ulp * M (the fp64 evaluation's own error is far smaller).
// When a face's estimate plus 1e-5 M (and a 1e-6 margin on the threshold) is
// below the threshold the tile is hit; when every evaluated face's estimate
// minus that bound is above it the tile is missed; otherwise the fp64 rule
// decides.  Mean inside the box: hit (the same comparisons either way).
// Result identical to tile_hit_fp64.  ia, ic: the reciprocals 1/a and 1/c
// (the edge minimiser is a product instead of a division; its rounding
// enters the edge value only at second order, inside the certified bound).
SG_DEV bool tile_hit_rcp(float mx, float my, float a, float b, float c, float ia, float ic, const steepgs_opts& opt,
                         int tx, int ty) {
  const float x0 = (float)(tx * opt.tile_w), x1 = (float)(tx * opt.tile_w + opt.tile_w - 1);
  const float y0 = (float)(ty * opt.tile_h), y1 = (float)(ty * opt.tile_h + opt.tile_h - 1);
  const bool fxl = mx < x0, fxh = mx > x1, fyl = my < y0, fyh = my > y1;
  if (!(fxl || fxh || fyl || fyh)) return true;
  const float T = opt.radius_sigmas * opt.radius_sigmas * (1.f + 1e-6f);
  const float tm = 1e-6f * T;
  bool sure_hit = false, all_miss = true;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    // the face seen across x (x = x0 or x1, free coordinate y), then across y
    const bool xe = e == 0;
    if (xe ? !(fxl || fxh) : !(fyl || fyh)) continue;
    const float fixed = xe ? ((fxl ? x0 : x1) - mx) : ((fyl ? y0 : y1) - my);
    const float lo = xe ? (y0 - my) : (x0 - mx), hi = xe ? (y1 - my) : (x1 - mx);
    const float pf = xe ? a : c, pv = xe ? c : a;  // coefficient of fixed^2 and of free^2
    float fr = -(b * fixed) * (xe ? ic : ia);
    fr = fminf(fmaxf(fr, lo), hi);
    const float q = pf * fixed * fixed + 2.f * b * fixed * fr + pv * fr * fr;
    const float M = pf * fixed * fixed + 2.f * fabsf(b * fixed * fr) + pv * fr * fr;
    const float err = 1e-5f * M;
    sure_hit |= q + err + tm <= T;
    all_miss &= q - err - tm > T;
  }
  if (sure_hit) return true;
  if (all_miss) return false;
  return tile_hit_fp64(mx, my, a, b, c, opt, tx, ty);
}

// view-independent part of a Gaussian
struct Gauss {
  double p[3];
  double qw, qx, qy, qz, qn;  // unit quaternion and the input's norm
  double R[3][3];             // rotation of the unit quaternion
  double s[3];                // scales
  double Sig[3][3];           // R diag(s^2) R^T
  double o;                   // opacity
};

SG_DEV void load_gauss(const float* __restrict__ params, int64_t n, int64_t i, Gauss& g) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; ++k) g.p[k] = (double)params[(STEEPGS_ROW_MEAN + k) * n + i];
  const double w0 = params[(STEEPGS_ROW_QUAT + 0) * n + i], x0 = params[(STEEPGS_ROW_QUAT + 1) * n + i];
  const double y0 = params[(STEEPGS_ROW_QUAT + 2) * n + i], z0 = params[(STEEPGS_ROW_QUAT + 3) * n + i];
  g.qn = sqrt(w0 * w0 + x0 * x0 + y0 * y0 + z0 * z0);
  const double w = w0 / g.qn, x = x0 / g.qn, y = y0 / g.qn, z = z0 / g.qn;
  g.qw = w;
  g.qx = x;
  g.qy = y;
  g.qz = z;
  g.R[0][0] = 1.0 - 2.0 * (y * y + z * z);
  g.R[0][1] = 2.0 * (x * y - w * z);
  g.R[0][2] = 2.0 * (x * z + w * y);
  g.R[1][0] = 2.0 * (x * y + w * z);
  g.R[1][1] = 1.0 - 2.0 * (x * x + z * z);
  g.R[1][2] = 2.0 * (y * z - w * x);
  g.R[2][0] = 2.0 * (x * z - w * y);
  g.R[2][1] = 2.0 * (y * z + w * x);
  g.R[2][2] = 1.0 - 2.0 * (x * x + y * y);
  double s2[3];
  for (int k = 0; k < 3; ++k) {
    g.s[k] = exp((double)params[(STEEPGS_ROW_LOG_SCALE + k) * n + i]);
    s2[k] = g.s[k] * g.s[k];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      g.Sig[a][b] = g.R[a][0] * s2[0] * g.R[b][0] + g.R[a][1] * s2[1] * g.R[b][1] + g.R[a][2] * s2[2] * g.R[b][2];
  g.o = 1.0 / (1.0 + exp(-(double)params[STEEPGS_ROW_OPACITY * n + i]));
}

// camera in fp64
struct CamD {
  double R[9], t[3], fx, fy, cx, cy;
  int W, H, model, tiles_x, tiles_y;
};

// per (Gaussian, view) quantities
struct ViewProj {
  double pc[3];
  double mx, my;
  double gx, gy;          // x/z and y/z after the frustum guard
  bool gx_free, gy_free;  // guard inactive (derivative passes)
  double J[2][3];         // Jacobian of the projection (guarded), or the affine map
  double P[2][3];         // J W
  double S2[2][2];        // Pi(Sigma) + dilation
  double det;
  double A00, A01, A11;  // conic
  double ax, ay;          // unit long axis of the footprint ellipse
  double lam_long, lam_short;  // the conic's eigenvalues along it and across it
  int rect[4];
};

// Per-view constants of the projection and the colour, the same for every
// Gaussian, in fp64: the camera centre -R^T t, the frustum-guard limits on
// x/z and y/z, then R, t, fx, fy, cx, cy.  Computed once per workgroup and
// view.
constexpr int kCamCentre = 0, kCamLim = 3, kCamR = 5, kCamT = 14, kCamF = 17;
constexpr int kCamConsts = 21;

SG_DEV void camera_centre(const steepgs_camera& c, double out[3]) {
#pragma clang fp contract(off)
  double R[9], t[3];
  for (int k = 0; k < 9; ++k) R[k] = c.R[k];
  for (int k = 0; k < 3; ++k) t[k] = c.t[k];
  for (int k = 0; k < 3; ++k) out[k] = -(R[0 + k] * t[0] + R[3 + k] * t[1] + R[6 + k] * t[2]);
}

SG_DEV void camera_constants(const steepgs_camera& c, const steepgs_opts& opt, double out[kCamConsts]) {
#pragma clang fp contract(off)
  camera_centre(c, out + kCamCentre);
  const double guard = opt.frustum_guard;
  out[kCamLim + 0] = guard * (0.5 * c.width / (double)c.fx);
  out[kCamLim + 1] = guard * (0.5 * c.height / (double)c.fy);
  for (int k = 0; k < 9; ++k) out[kCamR + k] = c.R[k];
  for (int k = 0; k < 3; ++k) out[kCamT + k] = c.t[k];
  out[kCamF + 0] = c.fx;
  out[kCamF + 1] = c.fy;
  out[kCamF + 2] = c.cx;
  out[kCamF + 3] = c.cy;
}

// the camera of one view from its constants (fp64 part) and the record
SG_DEV void load_cam(const double* cc, const steepgs_camera& c, CamD& d) {
  for (int k = 0; k < 9; ++k) d.R[k] = cc[kCamR + k];
  for (int k = 0; k < 3; ++k) d.t[k] = cc[kCamT + k];
  d.fx = cc[kCamF + 0];
  d.fy = cc[kCamF + 1];
  d.cx = cc[kCamF + 2];
  d.cy = cc[kCamF + 3];
  d.W = c.width;
  d.H = c.height;
  d.model = c.model;
  d.tiles_x = c.tiles_x;
  d.tiles_y = c.tiles_y;
}

// Geometry of one view; returns false when culled.  lim: the frustum-guard
// limits of camera_constants.  Operation order as written, no contraction:
// the tile rectangle and the culling decisions are reproducible from the
// fp32 inputs.  The structural zeros of J (and of the orthographic map) are
// left out of P = J W: the sums they would join are unchanged by them.
SG_DEV bool project_view(const Gauss& g, const CamD& cam, const steepgs_opts& opt, const double lim[2], ViewProj& v) {
#pragma clang fp contract(off)
  for (int r = 0; r < 3; ++r)
    v.pc[r] = cam.R[3 * r + 0] * g.p[0] + cam.R[3 * r + 1] * g.p[1] + cam.R[3 * r + 2] * g.p[2] + cam.t[r];
  if (!(v.pc[2] > (double)opt.near_z)) return false;
  if (cam.model == 0) {
    v.gx = v.pc[0] / v.pc[2];
    v.gy = v.pc[1] / v.pc[2];
    v.mx = cam.fx * v.gx + cam.cx;
    v.my = cam.fy * v.gy + cam.cy;
    v.gx_free = v.gy_free = true;
    if (opt.frustum_guard > 0.f) {
      if (v.gx < -lim[0]) { v.gx = -lim[0]; v.gx_free = false; }
      if (v.gx > lim[0]) { v.gx = lim[0]; v.gx_free = false; }
      if (v.gy < -lim[1]) { v.gy = -lim[1]; v.gy_free = false; }
      if (v.gy > lim[1]) { v.gy = lim[1]; v.gy_free = false; }
    }
    const double iz = 1.0 / v.pc[2];
    v.J[0][0] = cam.fx * iz;
    v.J[0][1] = 0.0;
    v.J[0][2] = -(cam.fx * v.gx) * iz;
    v.J[1][0] = 0.0;
    v.J[1][1] = cam.fy * iz;
    v.J[1][2] = -(cam.fy * v.gy) * iz;
    for (int c = 0; c < 3; ++c) {
      v.P[0][c] = v.J[0][0] * cam.R[0 + c] + v.J[0][2] * cam.R[6 + c];
      v.P[1][c] = v.J[1][1] * cam.R[3 + c] + v.J[1][2] * cam.R[6 + c];
    }
  } else {
    v.mx = cam.fx * v.pc[0] + cam.cx;
    v.my = cam.fy * v.pc[1] + cam.cy;
    v.gx = v.gy = 0.0;
    v.gx_free = v.gy_free = false;
    v.J[0][0] = cam.fx;
    v.J[0][1] = 0.0;
    v.J[0][2] = 0.0;
    v.J[1][0] = 0.0;
    v.J[1][1] = cam.fy;
    v.J[1][2] = 0.0;
    for (int c = 0; c < 3; ++c) {
      v.P[0][c] = cam.fx * cam.R[0 + c];
      v.P[1][c] = cam.fy * cam.R[3 + c];
    }
  }
  // Pi(Sigma) = (P Sigma) P^T, its lower entry the mirror of the upper one
  double PS[2][3];
  for (int a = 0; a < 2; ++a)
    for (int d = 0; d < 3; ++d) PS[a][d] = v.P[a][0] * g.Sig[0][d] + v.P[a][1] * g.Sig[1][d] + v.P[a][2] * g.Sig[2][d];
  v.S2[0][0] = PS[0][0] * v.P[0][0] + PS[0][1] * v.P[0][1] + PS[0][2] * v.P[0][2];
  v.S2[0][1] = PS[0][0] * v.P[1][0] + PS[0][1] * v.P[1][1] + PS[0][2] * v.P[1][2];
  v.S2[1][1] = PS[1][0] * v.P[1][0] + PS[1][1] * v.P[1][1] + PS[1][2] * v.P[1][2];
  v.S2[1][0] = v.S2[0][1];
  v.S2[0][0] = v.S2[0][0] + (double)opt.dilation;
  v.S2[1][1] = v.S2[1][1] + (double)opt.dilation;
  v.det = v.S2[0][0] * v.S2[1][1] - v.S2[0][1] * v.S2[1][0];
  if (!(v.det > 0.0)) return false;
  const double idet = 1.0 / v.det;
  v.A00 = v.S2[1][1] * idet;
  v.A01 = -v.S2[0][1] * idet;
  v.A11 = v.S2[0][0] * idet;

  const double a = v.S2[0][0], b = v.S2[0][1], c = v.S2[1][1];
  const double half = 0.5 * (a - c);
  const double rt = sqrt(half * half + b * b);
  const double lam = 0.5 * (a + c) + rt;
  // eigen form of the conic: the long axis is the eigenvector of Pi(Sigma)'s
  // larger eigenvalue lam (the cancellation-free one of the two textbook
  // forms), the conic's eigenvalues are 1 / lam along it and lam / det across
  {
    double ex = half + rt, ey = b;
    if (half < 0.0) {
      ex = b;
      ey = rt - half;
    }
    const double en = sqrt(ex * ex + ey * ey);
    if (en > 0.0) {
      const double ien = 1.0 / en;
      v.ax = ex * ien;
      v.ay = ey * ien;
    } else {
      v.ax = 1.0;
      v.ay = 0.0;
    }
    v.lam_long = 1.0 / lam;
    v.lam_short = lam * idet;
  }
  const double r = ceil((double)opt.radius_sigmas * sqrt(lam));
  // tile sizes are powers of two: the products below equal the quotients
  const double itw = 1.0 / opt.tile_w, ith = 1.0 / opt.tile_h;
  double x0 = floor((v.mx - r) * itw), x1 = floor((v.mx + r) * itw);
  double y0 = floor((v.my - r) * ith), y1 = floor((v.my + r) * ith);
  x0 = fmax(x0, 0.0);
  y0 = fmax(y0, 0.0);
  x1 = fmin(x1, (double)(cam.tiles_x - 1));
  y1 = fmin(y1, (double)(cam.tiles_y - 1));
  if (x0 > x1 || y0 > y1) return false;
  v.rect[0] = (int)x0;
  v.rect[1] = (int)y0;
  v.rect[2] = (int)x1;
  v.rect[3] = (int)y1;

  return true;
}

// fp64 colour of one channel in the reference operation order (no
// contraction, the direction divided by its length): the value that decides
// the clamp max(0, .) when a faster evaluation lands within 1e-5 of zero.
SG_DEV double colour_channel_fp64(const float* __restrict__ params, int64_t n, int64_t i, int deg,
                                  const double campos[3], int ch) {
#pragma clang fp contract(off)
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = (double)params[(STEEPGS_ROW_MEAN + k) * n + i] - campos[k];
  const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double Y[16];
  sh_eval<double>(deg, d[0] / len, d[1] / len, d[2] / len, Y);
  double acc = 0.0;
  for (int k = 0; k < (deg + 1) * (deg + 1); ++k) acc = acc + (double)params[(STEEPGS_ROW_SH + 3 * k + ch) * n + i] * Y[k];
  return acc + 0.5;
}

// SH colour of one view (Sec. 3: colour stored as SH coefficients):
// max(0, sum_k sh_k Y_k(dir) + 1/2), dir the unit vector from the camera
// centre to the mean.  sh[(3 k + ch) * stride] holds coefficient k of
// channel ch.  Evaluated in fp32 (error ~1e-7 of the terms' magnitude);
// returns a bit per channel that lies within 1e-5 of the clamp, whose
// decision and value the caller takes from colour_channel_fp64 instead.
template <int D>
SG_DEV uint32_t view_colour(const float p[3], const double campos[3], const float* sh, int stride, float rgb[3]) {
  constexpr int NB = (D + 1) * (D + 1);
  const float d0 = p[0] - (float)campos[0], d1 = p[1] - (float)campos[1], d2 = p[2] - (float)campos[2];
  const float il = 1.f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
  float Y[16];
  sh_eval<float>(D, d0 * il, d1 * il, d2 * il, Y);
  uint32_t near = 0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
#pragma unroll
    for (int k = 0; k < NB; ++k) acc = fmaf(sh[(3 * k + ch) * stride], Y[k], acc);
    near |= (fabsf(acc) < 1e-5f ? 1u : 0u) << ch;
    rgb[ch] = acc < 0.f ? 0.f : acc;
  }
  return near;
}

}  // namespace sg
