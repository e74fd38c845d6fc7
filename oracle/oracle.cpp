// Plain, slow, single-threaded FP64 oracle of the SteepGS hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
// load this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header, table or constant with the
// GPU library.
//
// What it computes (paper: "Steepest Descent Density Control for Compact 3D
// Gaussian Splatting", arXiv 2505.05587):
//   * the Gaussian primitive of Sec. 3, Eq. (sigma_3D): position p, covariance
//     from a quaternion and per-axis scales, opacity o, SH colour;
//   * its projection Pi (Sec. 3, Eq. (sigma_2D) and the footnote on Pi): the
//     mean maps through the camera, the covariance through the local affine
//     map P Sigma P^T;
//   * the front-to-back alpha blend of Eq. (alpha_blend), nearest first, over
//     the Gaussians whose screen-space footprint covers the pixel's tile;
//   * the L1 photometric loss of Eq. (loss), one mean per view, summed over
//     views;
//   * exact derivatives of that loss.  The blend's own derivative w.r.t. each
//     alpha is the product rule written out (suffix sums); every other
//     derivative comes from forward-mode dual numbers, so no hand-derived
//     chain rule appears here;
//   * the splitting matrix of Theorem 1, S_i = sum over views and pixels of
//     dL/dalpha_i(x) * Hessian_p alpha_i(x), with the Hessian of Sec. 4.4 and
//     App. C.4 (P, Pi(Sigma) and colour held fixed w.r.t. p);
//   * its eigen-decomposition by cyclic Jacobi rotations (the paper uses the
//     closed trigonometric root formula of App. A.3; this oracle uses a
//     different method on purpose);
//   * Steepest Density Control (Theorem 2, Algorithm 1): split iff
//     lambda_min < eps_split into p +/- eps * v_min, each child with half the
//     parent's opacity, other attributes copied.
//
// Parameter layout, planar [F][n]: p(3), log-scale(3), quaternion (w,x,y,z)(4),
// opacity logit(1), SH coefficients 3*(d+1)^2 (row 11 + 3*k + channel).
//
// Built with -O2 -ffp-contract=off so that every double operation rounds
// exactly as written.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// inputs

struct Cam {
  double R[9];  // world->camera rotation, row-major
  double t[3];
  double fx, fy, cx, cy;
  int W, H, model;  // model 0: pinhole, 1: orthographic
  int tiles_x, tiles_y;
  int64_t tile_offset;   // global id of this view's first tile
  int64_t pixel_offset;  // index of this view's first pixel in packed images
};

struct Opts {
  int tw, th;
  double near_z, radius_sigmas, dilation, guard;
  double alpha_min, alpha_max, t_min;
  double bg[3];
};

Opts read_opts(const double* o) {
  Opts r;
  r.tw = (int)o[0];
  r.th = (int)o[1];
  r.near_z = o[2];
  r.radius_sigmas = o[3];
  r.dilation = o[4];
  r.guard = o[5];
  r.alpha_min = o[6];
  // alpha stays below one even where alpha_max = 1 (smooth mode): capped at
  // the largest float below one, 1 - 2^-24, so that 1 - alpha (the
  // transmittance factor and the divisor of the blend's derivative) never
  // vanishes for a saturated opacity
  r.alpha_max = std::min(o[7], 1.0 - std::ldexp(1.0, -24));
  r.t_min = o[8];
  r.bg[0] = o[9];
  r.bg[1] = o[10];
  r.bg[2] = o[11];
  return r;
}

std::vector<Cam> read_cams(const float* cf, const int32_t* ci, int V, const Opts& opt) {
  std::vector<Cam> cams(V);
  int64_t toff = 0, poff = 0;
  for (int v = 0; v < V; ++v) {
    Cam& c = cams[v];
    for (int k = 0; k < 9; ++k) c.R[k] = cf[16 * v + k];
    for (int k = 0; k < 3; ++k) c.t[k] = cf[16 * v + 9 + k];
    c.fx = cf[16 * v + 12];
    c.fy = cf[16 * v + 13];
    c.cx = cf[16 * v + 14];
    c.cy = cf[16 * v + 15];
    c.W = ci[3 * v + 0];
    c.H = ci[3 * v + 1];
    c.model = ci[3 * v + 2];
    c.tiles_x = (c.W + opt.tw - 1) / opt.tw;
    c.tiles_y = (c.H + opt.th - 1) / opt.th;
    c.tile_offset = toff;
    c.pixel_offset = poff;
    toff += (int64_t)c.tiles_x * c.tiles_y;
    poff += (int64_t)c.W * c.H;
  }
  return cams;
}

int num_params(int deg) { return 11 + 3 * (deg + 1) * (deg + 1); }

// ---------------------------------------------------------------------------
// forward-mode dual numbers: value plus N partial derivatives

template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT: constants promote
};

template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v + b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v - b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N> Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r(-a.v);
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v * b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v / b.v);
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

template <int N> Dual<N> exp(const Dual<N>& a) {
  Dual<N> r(std::exp(a.v));
  for (int k = 0; k < N; ++k) r.d[k] = r.v * a.d[k];
  return r;
}
template <int N> Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r(std::sqrt(a.v));
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r;
}

double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }

double sqrt_(double x) { return std::sqrt(x); }
template <int N> Dual<N> sqrt_(const Dual<N>& x) { return sqrt(x); }
double exp_(double x) { return std::exp(x); }
template <int N> Dual<N> exp_(const Dual<N>& x) { return exp(x); }

// clamp to [lo, hi]; a clamped value is a constant (zero derivative)
template <class T> T clamp_(const T& x, double lo, double hi) {
  if (val(x) < lo) return T(lo);
  if (val(x) > hi) return T(hi);
  return x;
}

// ---------------------------------------------------------------------------
// real spherical harmonics from the associated Legendre functions
// (Condon-Shortley phase), index k = l*l + l + m, m = -l..l.
//   Y_l0  = K_l0 P_l^0(z)
//   Y_lm  = sqrt(2) K_lm P_l^m(cos t) cos(m phi)   (m > 0)
//   Y_l-m = sqrt(2) K_lm P_l^m(cos t) sin(m phi)   (m > 0)
// With Q_l^m = P_l^m / (1 - z^2)^(m/2) and, on the unit sphere,
// sin^m(t) e^{i m phi} = (x + i y)^m, every term is a polynomial in x, y, z.

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

template <class T>
void sh_basis(int deg, const T& x, const T& y, const T& z, T* Y) {
  T Q[4][4];
  for (int m = 0; m <= deg; ++m) {
    double dfact = 1.0;  // (2m-1)!!
    for (int i = 2 * m - 1; i > 1; i -= 2) dfact *= i;
    Q[m][m] = T(((m % 2) ? -1.0 : 1.0) * dfact);
    if (m + 1 <= deg) Q[m + 1][m] = z * (double)(2 * m + 1) * Q[m][m];
    for (int l = m + 2; l <= deg; ++l)
      Q[l][m] = ((double)(2 * l - 1) * z * Q[l - 1][m] - (double)(l + m - 1) * Q[l - 2][m]) /
                (double)(l - m);
  }
  T re[4], im[4];
  re[0] = T(1.0);
  im[0] = T(0.0);
  for (int m = 1; m <= deg; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
  for (int l = 0; l <= deg; ++l) {
    for (int m = 0; m <= l; ++m) {
      double K = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * factorial(l - m) / factorial(l + m));
      if (m == 0) {
        Y[l * l + l] = K * Q[l][0];
      } else {
        Y[l * l + l + m] = std::sqrt(2.0) * K * Q[l][m] * re[m];
        Y[l * l + l - m] = std::sqrt(2.0) * K * Q[l][m] * im[m];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// one Gaussian through one camera

template <class T>
struct Proj {
  bool visible = false;
  T mx, my;          // projected mean Pi(p), pixels
  T A00, A01, A11;   // conic: inverse of the 2D covariance Pi(Sigma) (+ dilation)
  T o;               // opacity
  T rgb[3];          // view-dependent colour, clamped at 0
  double depth = 0;  // camera-space z
  double rgb_raw[3] = {0, 0, 0};
  int rect[4] = {0, 0, -1, -1};  // tile x0, y0, x1, y1 (inclusive)
  float fmx, fmy, fa, fb, fc;    // mean and conic rounded to float32 (the stored record)
  int ntiles = 0;                // tiles of the rectangle that meet the cut-off ellipse
  // at the point (values only): the map of the 2D covariance P = J W (J at
  // the frustum-guarded point), the exact Jacobian of the projected mean
  // w.r.t. p, the rotation of the Gaussian and its log-scales
  double Pg[2][3] = {{0, 0, 0}, {0, 0, 0}};
  double Pe[2][3] = {{0, 0, 0}, {0, 0, 0}};
  double Rot[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double logs[3] = {0, 0, 0};
};

// Smallest value of q(d) = a dx^2 + 2 b dx dy + c dy^2, d = x - m, over the box
// [x0, x1] x [y0, y1] for a positive-definite conic: 0 when m lies inside,
// otherwise the smallest of the four edge minima, each the one-dimensional
// minimiser clamped to its edge (q is convex).
double box_min_q(double a, double b, double c, double mx, double my, double x0, double x1, double y0, double y1) {
  if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.0;
  double best = INFINITY;
  for (int e = 0; e < 2; ++e) {
    double dx = (e == 0 ? x0 : x1) - mx;
    double dy = -(b * dx) / c;
    if (dy < y0 - my) dy = y0 - my;
    if (dy > y1 - my) dy = y1 - my;
    double q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
    if (q < best) best = q;
    double ey = (e == 0 ? y0 : y1) - my;
    double ex = -(b * ey) / a;
    if (ex < x0 - mx) ex = x0 - mx;
    if (ex > x1 - mx) ex = x1 - mx;
    q = a * ex * ex + 2.0 * b * ex * ey + c * ey * ey;
    if (q < best) best = q;
  }
  return best;
}

// Tile (tx, ty) belongs to the footprint when its box of pixel centres meets
// the ellipse q <= radius_sigmas^2 (1e-6 relative slack), evaluated on the
// float32 record so that any implementation storing that record can repeat it.
template <class T>
bool tile_hit(const Proj<T>& p, const Opts& opt, int tx, int ty) {
  double k2 = (double)opt.radius_sigmas * (double)opt.radius_sigmas;
  double x0 = (double)tx * opt.tw, y0 = (double)ty * opt.th;
  double q = box_min_q((double)p.fa, (double)p.fb, (double)p.fc, (double)p.fmx, (double)p.fmy, x0, x0 + (opt.tw - 1),
                       y0, y0 + (opt.th - 1));
  return q <= k2 * (1.0 + 1e-6);
}

template <class T>
void project(const T* th, int deg, const Cam& cam, const Opts& opt, Proj<T>& out) {
  out.visible = false;
  // covariance from quaternion (w,x,y,z) and scales: Sigma = R diag(s^2) R^T
  T qn = sqrt_(th[6] * th[6] + th[7] * th[7] + th[8] * th[8] + th[9] * th[9]);
  T w = th[6] / qn, x = th[7] / qn, y = th[8] / qn, z = th[9] / qn;
  T Rq[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  T s2[3];
  for (int k = 0; k < 3; ++k) {
    T s = exp_(th[3 + k]);
    s2[k] = s * s;
  }
  T Sig[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Sig[a][b] = Rq[a][0] * s2[0] * Rq[b][0] + Rq[a][1] * s2[1] * Rq[b][1] + Rq[a][2] * s2[2] * Rq[b][2];
  out.o = 1.0 / (1.0 + exp_(-th[10]));
  for (int a = 0; a < 3; ++a) {
    out.logs[a] = val(th[3 + a]);
    for (int b = 0; b < 3; ++b) out.Rot[a][b] = val(Rq[a][b]);
  }

  // camera space
  T pc[3];
  for (int r = 0; r < 3; ++r)
    pc[r] = cam.R[3 * r + 0] * th[0] + cam.R[3 * r + 1] * th[1] + cam.R[3 * r + 2] * th[2] + cam.t[r];
  out.depth = val(pc[2]);
  if (!(out.depth > opt.near_z)) return;

  // projected mean and the local affine map J (pinhole: Jacobian of the
  // perspective division at the frustum-guarded point)
  T J[2][3];
  if (cam.model == 0) {
    out.mx = cam.fx * (pc[0] / pc[2]) + cam.cx;
    out.my = cam.fy * (pc[1] / pc[2]) + cam.cy;
    T gx = pc[0] / pc[2], gy = pc[1] / pc[2];
    if (opt.guard > 0.0) {
      double limx = opt.guard * (0.5 * cam.W / cam.fx);
      double limy = opt.guard * (0.5 * cam.H / cam.fy);
      gx = clamp_(gx, -limx, limx);
      gy = clamp_(gy, -limy, limy);
    }
    const T iz = 1.0 / pc[2];
    J[0][0] = cam.fx * iz;
    J[0][1] = T(0.0);
    J[0][2] = -(cam.fx * gx) * iz;
    J[1][0] = T(0.0);
    J[1][1] = cam.fy * iz;
    J[1][2] = -(cam.fy * gy) * iz;
  } else {
    out.mx = cam.fx * pc[0] + cam.cx;
    out.my = cam.fy * pc[1] + cam.cy;
    J[0][0] = T(cam.fx);
    J[0][1] = T(0.0);
    J[0][2] = T(0.0);
    J[1][0] = T(0.0);
    J[1][1] = T(cam.fy);
    J[1][2] = T(0.0);
  }
  // P = J W (2x3), Pi(Sigma) = P Sigma P^T + dilation * I
  T P[2][3];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 3; ++c) P[a][c] = J[a][0] * cam.R[0 + c] + J[a][1] * cam.R[3 + c] + J[a][2] * cam.R[6 + c];
  {
    // exact (unguarded) Jacobian of the projected mean w.r.t. p
    double Je[2][3] = {{cam.fx, 0.0, 0.0}, {0.0, cam.fy, 0.0}};
    if (cam.model == 0) {
      const double z = val(pc[2]);
      Je[0][0] = cam.fx / z;
      Je[0][2] = -cam.fx * val(pc[0]) / (z * z);
      Je[1][1] = cam.fy / z;
      Je[1][2] = -cam.fy * val(pc[1]) / (z * z);
    }
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) {
        out.Pg[a][c] = val(P[a][c]);
        out.Pe[a][c] = Je[a][0] * cam.R[0 + c] + Je[a][1] * cam.R[3 + c] + Je[a][2] * cam.R[6 + c];
      }
  }
  // (P Sigma) P^T; the matrix is symmetric, so its lower entry is the upper one
  T PS[2][3];
  for (int a = 0; a < 2; ++a)
    for (int d = 0; d < 3; ++d) PS[a][d] = P[a][0] * Sig[0][d] + P[a][1] * Sig[1][d] + P[a][2] * Sig[2][d];
  T S2[2][2];
  S2[0][0] = PS[0][0] * P[0][0] + PS[0][1] * P[0][1] + PS[0][2] * P[0][2];
  S2[0][1] = PS[0][0] * P[1][0] + PS[0][1] * P[1][1] + PS[0][2] * P[1][2];
  S2[1][1] = PS[1][0] * P[1][0] + PS[1][1] * P[1][1] + PS[1][2] * P[1][2];
  S2[1][0] = S2[0][1];
  S2[0][0] = S2[0][0] + opt.dilation;
  S2[1][1] = S2[1][1] + opt.dilation;
  T det = S2[0][0] * S2[1][1] - S2[0][1] * S2[1][0];
  if (!(val(det) > 0.0)) return;
  // the conic A = Pi(Sigma)^-1 through one reciprocal of the determinant
  const T idet = 1.0 / det;
  out.A00 = S2[1][1] * idet;
  out.A01 = -S2[0][1] * idet;
  out.A11 = S2[0][0] * idet;

  // footprint: radius_sigmas standard deviations along the major axis, in
  // whole pixels; tiles whose pixel span meets [m - r, m + r]
  double a = val(S2[0][0]), b = val(S2[0][1]), c = val(S2[1][1]);
  double half = 0.5 * (a - c);
  double lam = 0.5 * (a + c) + std::sqrt(half * half + b * b);
  double r = std::ceil(opt.radius_sigmas * std::sqrt(lam));
  double mxv = val(out.mx), myv = val(out.my);
  double x0 = std::floor((mxv - r) / opt.tw), x1 = std::floor((mxv + r) / opt.tw);
  double y0 = std::floor((myv - r) / opt.th), y1 = std::floor((myv + r) / opt.th);
  x0 = std::max(x0, 0.0);
  y0 = std::max(y0, 0.0);
  x1 = std::min(x1, (double)(cam.tiles_x - 1));
  y1 = std::min(y1, (double)(cam.tiles_y - 1));
  if (x0 > x1 || y0 > y1) return;
  out.rect[0] = (int)x0;
  out.rect[1] = (int)y0;
  out.rect[2] = (int)x1;
  out.rect[3] = (int)y1;
  // of the rectangle, the tiles that meet the cut-off ellipse
  out.fmx = (float)val(out.mx);
  out.fmy = (float)val(out.my);
  out.fa = (float)val(out.A00);
  out.fb = (float)val(out.A01);
  out.fc = (float)val(out.A11);
  out.ntiles = 0;
  for (int ty = out.rect[1]; ty <= out.rect[3]; ++ty)
    for (int tx = out.rect[0]; tx <= out.rect[2]; ++tx) out.ntiles += tile_hit(out, opt, tx, ty) ? 1 : 0;
  if (out.ntiles == 0) return;

  // colour: SH evaluated at the unit direction from the camera centre
  double campos[3];
  for (int k = 0; k < 3; ++k) campos[k] = -(cam.R[0 + k] * cam.t[0] + cam.R[3 + k] * cam.t[1] + cam.R[6 + k] * cam.t[2]);
  T dx = th[0] - campos[0], dy = th[1] - campos[1], dz = th[2] - campos[2];
  T dn = sqrt_(dx * dx + dy * dy + dz * dz);
  dx = dx / dn;
  dy = dy / dn;
  dz = dz / dn;
  T Y[16];
  sh_basis(deg, dx, dy, dz, Y);
  int nb = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    T acc(0.0);
    for (int k = 0; k < nb; ++k) acc = acc + th[11 + 3 * k + ch] * Y[k];
    acc = acc + 0.5;
    out.rgb_raw[ch] = val(acc);
    out.rgb[ch] = (val(acc) < 0.0) ? T(0.0) : acc;
  }
  out.visible = true;
}

// alpha of a projected Gaussian at pixel (u,v) before the alpha_max clamp
template <class T>
T alpha_raw(const T& mx, const T& my, const T& A00, const T& A01, const T& A11, const T& o, double u, double v) {
  T dx = u - mx, dy = v - my;
  T power = -0.5 * (A00 * dx * dx + 2.0 * A01 * dx * dy + A11 * dy * dy);
  return o * exp_(power);
}

// alpha inside the footprint (q <= radius_sigmas^2), 0 outside
double alpha_in_footprint(const Proj<double>& g, const Opts& opt, double u, double v) {
  double dx = u - g.mx, dy = v - g.my;
  double q = g.A00 * dx * dx + 2.0 * g.A01 * dx * dy + g.A11 * dy * dy;
  if (q > opt.radius_sigmas * opt.radius_sigmas) return 0.0;
  return alpha_raw(g.mx, g.my, g.A00, g.A01, g.A11, g.o, u, v);
}

// Hessian of alpha w.r.t. the projected mean (Sec. 4.4, App. C.4):
//   alpha * (A d d^T A - A),  d = x - Pi(p)
void alpha_hessian_mu(double mx, double my, double A00, double A01, double A11, double o, double u, double v,
                      double H[3]) {
  double a = alpha_raw(mx, my, A00, A01, A11, o, u, v);
  double dx = u - mx, dy = v - my;
  double Adx = A00 * dx + A01 * dy, Ady = A01 * dx + A11 * dy;
  H[0] = a * (Adx * Adx - A00);
  H[1] = a * (Adx * Ady - A01);
  H[2] = a * (Ady * Ady - A11);
}

// ---------------------------------------------------------------------------
// Second-order forward mode over six variables: value, gradient and the
// upper triangle of the Hessian, propagated by the product and chain rules.
// Used for the splitting matrix over theta = (p, log-scales).

constexpr int kH6 = 21;  // upper triangle of a 6x6, row-major: (0,0) (0,1) .. (0,5) (1,1) .. (5,5)
int h6(int i, int j) {
  if (i > j) std::swap(i, j);
  return i * 6 - i * (i - 1) / 2 + (j - i);
}

struct HD {
  double v = 0.0;
  double g[6] = {0, 0, 0, 0, 0, 0};
  double h[kH6] = {};
  HD() = default;
  HD(double x) : v(x) {}  // NOLINT: constants promote
};

HD operator+(const HD& a, const HD& b) {
  HD r(a.v + b.v);
  for (int k = 0; k < 6; ++k) r.g[k] = a.g[k] + b.g[k];
  for (int k = 0; k < kH6; ++k) r.h[k] = a.h[k] + b.h[k];
  return r;
}
HD operator-(const HD& a, const HD& b) {
  HD r(a.v - b.v);
  for (int k = 0; k < 6; ++k) r.g[k] = a.g[k] - b.g[k];
  for (int k = 0; k < kH6; ++k) r.h[k] = a.h[k] - b.h[k];
  return r;
}
HD operator*(const HD& a, const HD& b) {  // (ab)'' = a'' b + a' b'^T + b' a'^T + a b''
  HD r(a.v * b.v);
  for (int k = 0; k < 6; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k];
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      const int k = h6(i, j);
      r.h[k] = a.h[k] * b.v + a.g[i] * b.g[j] + a.g[j] * b.g[i] + a.v * b.h[k];
    }
  return r;
}
// f(a) for a scalar function with f(a.v), f'(a.v), f''(a.v) given
HD apply(const HD& a, double f0, double f1, double f2) {
  HD r(f0);
  for (int k = 0; k < 6; ++k) r.g[k] = f1 * a.g[k];
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) r.h[h6(i, j)] = f1 * a.h[h6(i, j)] + f2 * a.g[i] * a.g[j];
  return r;
}
HD recip(const HD& a) { return apply(a, 1.0 / a.v, -1.0 / (a.v * a.v), 2.0 / (a.v * a.v * a.v)); }
HD operator/(const HD& a, const HD& b) { return a * recip(b); }
HD hexp(const HD& a) {
  const double e = std::exp(a.v);
  return apply(a, e, e, e);
}
double hexp(double a) { return std::exp(a); }
double recip(double a) { return 1.0 / a; }

// alpha at pixel (u, v) as a function of theta = (p, log-scales) moved by dth
// from the Gaussian's point, with the maps of the projection frozen there (the
// "approximately" of the Hessian in Sec. 4.4, App. C.4): the mean moves along
// the exact Jacobian Pe, the 2D covariance is Pg Sigma(s) Pg^T + dilation with
// Sigma(s) = R diag(exp(2 s)) R^T, R and the opacity fixed.
template <class T>
T alpha_theta6(const Proj<double>& g, double dil, double u, double v, const T dth[6]) {
  T mx = T(g.mx), my = T(g.my);
  for (int c = 0; c < 3; ++c) {
    mx = mx + T(g.Pe[0][c]) * dth[c];
    my = my + T(g.Pe[1][c]) * dth[c];
  }
  T s2[3];
  for (int k = 0; k < 3; ++k) s2[k] = hexp(T(2.0 * g.logs[k]) + T(2.0) * dth[3 + k]);
  T Sig[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      Sig[a][b] = T(0.0);
      for (int k = 0; k < 3; ++k) Sig[a][b] = Sig[a][b] + T(g.Rot[a][k] * g.Rot[b][k]) * s2[k];
    }
  T S2[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      S2[a][b] = T(0.0);
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) S2[a][b] = S2[a][b] + T(g.Pg[a][c] * g.Pg[b][d]) * Sig[c][d];
    }
  S2[0][0] = S2[0][0] + T(dil);
  S2[1][1] = S2[1][1] + T(dil);
  const T idet = recip(S2[0][0] * S2[1][1] - S2[0][1] * S2[1][0]);
  const T A00 = S2[1][1] * idet, A01 = T(0.0) - S2[0][1] * idet, A11 = S2[0][0] * idet;
  const T dx = T(u) - mx, dy = T(v) - my;
  const T q = A00 * dx * dx + T(2.0) * A01 * dx * dy + A11 * dy * dy;
  return T(g.o) * hexp(T(-0.5) * q);
}

// Hessian of alpha over theta = (p, log-scales) at the point, upper triangle
void alpha_hessian_theta6(const Proj<double>& g, double dil, double u, double v, double H[kH6]) {
  HD d[6];
  for (int k = 0; k < 6; ++k) d[k].g[k] = 1.0;
  const HD a = alpha_theta6<HD>(g, dil, u, v, d);
  for (int k = 0; k < kH6; ++k) H[k] = a.h[k];
}

// ---------------------------------------------------------------------------
// one view: projected records and per-tile depth-ordered lists

struct View {
  const Cam* cam;
  const Opts* opt;
  int n;
  std::vector<Proj<double>> rec;
  std::vector<std::vector<int>> tiles;  // Gaussian ids per tile, ordered by (depth_f32 bits, id)
};

uint32_t depth_bits(double z) {
  float f = (float)z;  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

void load_theta(const float* params, int64_t n, int deg, int64_t i, double* th) {
  int F = num_params(deg);
  for (int f = 0; f < F; ++f) th[f] = params[(int64_t)f * n + i];
}

void build_view(const float* params, int64_t n, int deg, const Cam& cam, const Opts& opt, View& view) {
  view.cam = &cam;
  view.opt = &opt;
  view.n = (int)n;
  view.rec.assign(n, Proj<double>());
  double th[59];
  for (int64_t i = 0; i < n; ++i) {
    load_theta(params, n, deg, i, th);
    project(th, deg, cam, opt, view.rec[i]);
  }
  view.tiles.assign((size_t)cam.tiles_x * cam.tiles_y, std::vector<int>());
  for (int64_t i = 0; i < n; ++i) {
    const Proj<double>& p = view.rec[i];
    if (!p.visible) continue;
    for (int ty = p.rect[1]; ty <= p.rect[3]; ++ty)
      for (int tx = p.rect[0]; tx <= p.rect[2]; ++tx) view.tiles[(size_t)ty * cam.tiles_x + tx].push_back((int)i);
  }
  for (auto& lst : view.tiles)
    std::stable_sort(lst.begin(), lst.end(), [&](int a, int b) {
      return depth_bits(view.rec[a].depth) < depth_bits(view.rec[b].depth);
    });
}

// ---------------------------------------------------------------------------
// per-pixel blend (Eq. alpha_blend, front to back)

struct Contrib {
  int g;
  double a, T;
  bool clamped;
};

// A cut-off decision of the blend taken within reach of float32 rounding of
// its threshold: either outcome is a correct result of an implementation
// that evaluates the record in float32.
enum DecisionKind { kDecFootprint = 0, kDecAlphaMax = 1, kDecAlphaMin = 2, kDecTmin = 3 };

struct Pixel {
  double C[3];
  double T_final;
  std::vector<Contrib> list;
  int listed;  // how many entries of the tile list were examined (incl. the stopping one)
  bool ambig;  // a cut-off decision within the ambiguity band, or an uncertain alpha
  std::vector<int> amb_ids;  // entries whose own cut-off decision is within the band
  int ndec;    // decisions within their band (in the order the blend meets them)
  int dec_kind[4];  // kinds of the first four of them
  bool valunc;  // an entry's alpha is uncertain in float32 by more than kAlphaValue
};

constexpr double kAlphaBand = 1e-5;  // relative band around alpha_min / alpha_max
constexpr double kQBand = 1e-5;      // relative band around the footprint cut-off radius_sigmas^2
constexpr double kTBand = 5e-5;      // relative band around t_min (fp32 transmittance after ~400 factors)
// A float32 evaluation of q = d^T A d as a sum of two non-negative terms
// along the footprint ellipse's axes (lambda_1 (e_1 . d)^2 + lambda_2
// (e_2 . d)^2, from float32 axes and eigenvalues) is good to about
// 2^-24 (3 q + 2 sqrt(lambda_max q) e_d) when the projections of d on the
// axes are known to 2^-24 e_d: the larger eigenvalue weighs a change of the
// projections by sqrt(lambda_max q).  The offsets are taken from the float32
// mean, the remainder of its rounding (stored as binary16) folded into the
// projections: e_d = 5 |d| + 2^-11 |mean| + 1/2 covers the float32 roundings
// of the offsets, the axes and the projections, and the remainder's binary16
// rounding.  For a thin Gaussian seen far along its long axis this exceeds
// 2^-24 q by the square root of the ellipse's aspect ratio.  The bands widen
// with that bound, and a pair whose alpha error (alpha * bound / 2) can move
// the colour by more than kAlphaValue marks its pixel as well.
constexpr double kAlphaValue = 1e-5;

// Blend one pixel (Eq. alpha_blend, front to back).  flip >= 0 takes the
// other outcome of the flip-th decision within its band (counted as the
// blend meets them), the alternative result of a float32 implementation.
void blend_pixel(const View& view, int u, int v, Pixel& px, int flip = -1) {
  const Cam& cam = *view.cam;
  const Opts& opt = *view.opt;
  const std::vector<int>& lst = view.tiles[(size_t)(v / opt.th) * cam.tiles_x + (u / opt.tw)];
  double T = 1.0;
  px.C[0] = px.C[1] = px.C[2] = 0.0;
  px.list.clear();
  px.amb_ids.clear();
  px.ambig = false;
  px.valunc = false;
  px.ndec = 0;
  px.listed = (int)lst.size();
  const double k2 = opt.radius_sigmas * opt.radius_sigmas;
  // records a decision within its band; true when this one is to be flipped
  auto decide = [&](int kind, int g) {
    if (px.ndec < 4) px.dec_kind[px.ndec] = kind;
    const bool f = px.ndec == flip;
    ++px.ndec;
    px.ambig = true;
    px.amb_ids.push_back(g);
    return f;
  };
  for (size_t j = 0; j < lst.size(); ++j) {
    const Proj<double>& g = view.rec[lst[j]];
    // footprint: only pixels within radius_sigmas (Mahalanobis) of the mean
    double dxu = u - g.mx, dyv = v - g.my;
    double q = g.A00 * dxu * dxu + 2.0 * g.A01 * dxu * dyv + g.A11 * dyv * dyv;
    const double lmax = 0.5 * (g.A00 + g.A11) + std::sqrt(0.25 * (g.A00 - g.A11) * (g.A00 - g.A11) + g.A01 * g.A01);
    const double e_d = 5.0 * std::sqrt(dxu * dxu + dyv * dyv) + std::ldexp(std::sqrt(g.mx * g.mx + g.my * g.my), -11) +
                       0.5;
    const double err = std::ldexp(3.0 * std::fabs(q) + 2.0 * std::sqrt(lmax * std::max(q, 0.0)) * e_d, -24);
    const double eq = 2.0 * err;  // float32 bound on q, with a factor 2 of margin
    bool outside = q > k2;
    if (std::fabs(q - k2) <= std::max(kQBand * k2, eq) && decide(kDecFootprint, lst[j])) outside = !outside;
    if (outside) continue;
    double a = alpha_raw(g.mx, g.my, g.A00, g.A01, g.A11, g.o, (double)u, (double)v);
    const double aband = std::max(kAlphaBand, 0.5 * eq);  // relative: d alpha / alpha = dq / 2
    bool clamped = a > opt.alpha_max;
    if (opt.alpha_max < 1.0 && std::fabs(a - opt.alpha_max) <= aband * opt.alpha_max &&
        decide(kDecAlphaMax, lst[j]))
      clamped = !clamped;
    if (clamped) a = opt.alpha_max;
    bool skip = a < opt.alpha_min;
    if (opt.alpha_min > 0.0 && std::fabs(a - opt.alpha_min) <= aband * opt.alpha_min &&
        decide(kDecAlphaMin, lst[j]))
      skip = !skip;
    // an alpha error da moves the colour by T da (c_i - mean colour behind
    // the entry, background included): at most T da for colours in [0, 1]
    if (!skip && T * a * 0.5 * err > kAlphaValue) {
      px.valunc = true;
      px.ambig = true;
      px.amb_ids.push_back(lst[j]);
    }
    if (skip) continue;
    double Tn = T * (1.0 - a);
    bool stop = Tn < opt.t_min;
    if (opt.t_min > 0.0 && std::fabs(Tn - opt.t_min) <= kTBand * opt.t_min && decide(kDecTmin, lst[j])) stop = !stop;
    if (stop) {
      px.listed = (int)j + 1;
      break;
    }
    for (int ch = 0; ch < 3; ++ch) px.C[ch] += g.rgb[ch] * a * T;
    px.list.push_back({lst[j], a, T, clamped});
    T = Tn;
  }
  for (int ch = 0; ch < 3; ++ch) px.C[ch] += T * opt.bg[ch];
  px.T_final = T;
}

// per (Gaussian, view) accumulators of the pixel backward
struct Grad2D {
  double g[9];  // dL/d(mx, my, A00, A01, A11, o, r, g, b)
  double H[3];  // sum_x dL/dalpha * Hessian_mu alpha: xx, xy, yy
  double H6[kH6];  // sum_x dL/dalpha * Hessian_theta alpha, theta = (p, log-scales) (when asked)
  // Gross magnitudes of the per-pixel terms whose sums the gradients and S
  // are made of (not part of the method: the scale of the float32 summation
  // error of an implementation that adds them in some order), with
  // g = dL/dalpha, d = pixel - mean, G = alpha / o:
  //   sum |g alpha| |dx|, |g alpha| |dy|, |g alpha| dx^2, |g alpha| |dx dy|,
  //   |g alpha| dy^2, |g| G, alpha T |dL/dC_c| (c = r, g, b), |g alpha|
  double gross[10];
};

// Exact reverse sweep of one pixel given dL/dC.  Accumulates into acc[g]
// for every contributing Gaussian g with want[g] set (want == nullptr: all).
void backward_pixel(const View& view, int u, int v, const Pixel& px, const double dLdC[3],
                    std::vector<Grad2D>& acc, const std::vector<uint8_t>* want, bool hess6 = false) {
  const Opts& opt = *view.opt;
  double R[3];  // sum of the colour behind the current entry, background included
  for (int ch = 0; ch < 3; ++ch) R[ch] = px.T_final * opt.bg[ch];
  for (int k = (int)px.list.size() - 1; k >= 0; --k) {
    const Contrib& c = px.list[k];
    const Proj<double>& g = view.rec[c.g];
    double dLda = 0.0;
    for (int ch = 0; ch < 3; ++ch) dLda += dLdC[ch] * (g.rgb[ch] * c.T - R[ch] / (1.0 - c.a));
    for (int ch = 0; ch < 3; ++ch) R[ch] += g.rgb[ch] * c.a * c.T;
    if (want && !(*want)[c.g]) continue;
    Grad2D& A = acc[c.g];
    for (int ch = 0; ch < 3; ++ch) A.g[6 + ch] += c.a * c.T * dLdC[ch];
    for (int ch = 0; ch < 3; ++ch) A.gross[6 + ch] += c.a * c.T * std::fabs(dLdC[ch]);
    if (c.clamped) continue;  // alpha = alpha_max: constant in (mean, conic, opacity)
    {
      const double ga = std::fabs(dLda) * c.a, dx = u - g.mx, dy = v - g.my;
      A.gross[0] += ga * std::fabs(dx);
      A.gross[1] += ga * std::fabs(dy);
      A.gross[2] += ga * dx * dx;
      A.gross[3] += ga * std::fabs(dx * dy);
      A.gross[4] += ga * dy * dy;
      A.gross[5] += std::fabs(dLda) * c.a / g.o;
      A.gross[9] += ga;
    }
    Dual<6> in[6];
    double vals[6] = {g.mx, g.my, g.A00, g.A01, g.A11, g.o};
    for (int k2 = 0; k2 < 6; ++k2) {
      in[k2] = Dual<6>(vals[k2]);
      in[k2].d[k2] = 1.0;
    }
    Dual<6> a = alpha_raw(in[0], in[1], in[2], in[3], in[4], in[5], (double)u, (double)v);
    for (int k2 = 0; k2 < 6; ++k2) A.g[k2] += dLda * a.d[k2];
    double H[3];
    alpha_hessian_mu(g.mx, g.my, g.A00, g.A01, g.A11, g.o, (double)u, (double)v, H);
    for (int k2 = 0; k2 < 3; ++k2) A.H[k2] += dLda * H[k2];
    if (hess6) {
      double H6[kH6];
      alpha_hessian_theta6(g, opt.dilation, (double)u, (double)v, H6);
      for (int k2 = 0; k2 < kH6; ++k2) A.H6[k2] += dLda * H6[k2];
    }
  }
}

// Jacobian of the 9 projected quantities w.r.t. the F parameters of Gaussian i
template <int F>
bool jacobian(const float* params, int64_t n, int deg, int64_t i, const Cam& cam, const Opts& opt, double J[9][59]) {
  double th[59];
  load_theta(params, n, deg, i, th);
  Dual<F> td[F];
  for (int f = 0; f < F; ++f) {
    td[f] = Dual<F>(th[f]);
    td[f].d[f] = 1.0;
  }
  Proj<Dual<F>> pr;
  project(td, deg, cam, opt, pr);
  if (!pr.visible) return false;
  const Dual<F>* outs[9] = {&pr.mx, &pr.my, &pr.A00, &pr.A01, &pr.A11, &pr.o, &pr.rgb[0], &pr.rgb[1], &pr.rgb[2]};
  for (int r = 0; r < 9; ++r)
    for (int f = 0; f < F; ++f) J[r][f] = outs[r]->d[f];
  return true;
}

bool jacobian_any(const float* params, int64_t n, int deg, int64_t i, const Cam& cam, const Opts& opt, double J[9][59]) {
  switch (deg) {
    case 0: return jacobian<14>(params, n, deg, i, cam, opt, J);
    case 1: return jacobian<23>(params, n, deg, i, cam, opt, J);
    case 2: return jacobian<38>(params, n, deg, i, cam, opt, J);
    default: return jacobian<59>(params, n, deg, i, cam, opt, J);
  }
}

// lift the per-view accumulators of Gaussian i to parameter space:
// grads += J^T g2d, S += P^T H P with P = d Pi(p) / dp (rows 0-1, columns 0-2).
// With rec given, also the gross magnitudes (Grad2D::gross) through the
// absolute Jacobian: gabs += |J|^T (|A| m1, m2 / 2, ..., colour), and
// Sabs += |P|^T (|A| M |A| + m0 |A|) |P| with M, m0 the gross second and
// zeroth moments, |A| the entrywise absolute conic; |S| <= Sabs entrywise.
void lift(const float* params, int64_t n, int deg, int64_t i, const Cam& cam, const Opts& opt, const Grad2D& acc,
          double* grad_i /*[F] stride gstride*/, int64_t gstride, double* S_i /*[9] stride sstride*/, int64_t sstride,
          const Proj<double>* rec = nullptr, double* gabs_i = nullptr, double* Sabs_i = nullptr) {
  double J[9][59];
  if (!jacobian_any(params, n, deg, i, cam, opt, J)) return;
  int F = num_params(deg);
  if (rec && (gabs_i || Sabs_i)) {
    const double* q = acc.gross;
    const double a0 = std::fabs(rec->A00), a1 = std::fabs(rec->A01), a2 = std::fabs(rec->A11);
    const double g2abs[9] = {a0 * q[0] + a1 * q[1], a1 * q[0] + a2 * q[1], 0.5 * q[2], q[3], 0.5 * q[4], q[5],
                             q[6], q[7], q[8]};
    if (gabs_i)
      for (int f = 0; f < F; ++f) {
        double s = 0.0;
        for (int r = 0; r < 9; ++r) s += g2abs[r] * std::fabs(J[r][f]);
        gabs_i[f * gstride] += s;
      }
    if (Sabs_i) {
      const double Aa[2][2] = {{a0, a1}, {a1, a2}}, Ma[2][2] = {{q[2], q[3]}, {q[3], q[4]}};
      double Ha[2][2];
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
          double s = q[9] * Aa[x][y];
          for (int k = 0; k < 2; ++k)
            for (int l = 0; l < 2; ++l) s += Aa[x][k] * Ma[k][l] * Aa[l][y];
          Ha[x][y] = s;
        }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double s = 0.0;
          for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) s += std::fabs(J[x][a]) * Ha[x][y] * std::fabs(J[y][b]);
          Sabs_i[(3 * a + b) * sstride] += s;
        }
    }
  }
  for (int f = 0; f < F; ++f) {
    double s = 0.0;
    for (int r = 0; r < 9; ++r) s += acc.g[r] * J[r][f];
    grad_i[f * gstride] += s;
  }
  double H[2][2] = {{acc.H[0], acc.H[1]}, {acc.H[1], acc.H[2]}};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) s += J[x][a] * H[x][y] * J[y][b];
      S_i[(3 * a + b) * sstride] += s;
    }
}

double sgn(double x) { return (x > 0.0) - (x < 0.0); }

// A flipped decision in a pixel can change the gradient of that pixel's
// contributors and of the entry whose decision flipped; mark those.
void mark_affected(const Pixel& px, uint8_t* flags) {
  for (const Contrib& c : px.list) flags[c.g] = 1;
  for (int g : px.amb_ids) flags[g] = 1;
}

// ---------------------------------------------------------------------------
// symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations

void jacobi_eigh(const double Ain[9], double lam[3], double vec[9] /* columns = eigenvectors */) {
  double A[3][3], Vm[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      A[a][b] = 0.5 * (Ain[3 * a + b] + Ain[3 * b + a]);
      Vm[a][b] = (a == b) ? 1.0 : 0.0;
    }
  double norm = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) norm += A[a][b] * A[a][b];
  norm = std::sqrt(norm);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = std::sqrt(2.0 * (A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2]));
    if (off <= 1e-15 * norm || off == 0.0) break;
    const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (auto& pq : pairs) {
      int p = pq[0], q = pq[1];
      if (A[p][q] == 0.0) continue;
      // rotation angle that zeroes A[p][q]
      double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
      double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
      double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
      double G[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
      G[p][p] = c;
      G[q][q] = c;
      G[p][q] = s;
      G[q][p] = -s;
      double B[3][3], C[3][3];
      for (int a = 0; a < 3; ++a)  // B = G^T A
        for (int b = 0; b < 3; ++b) B[a][b] = G[0][a] * A[0][b] + G[1][a] * A[1][b] + G[2][a] * A[2][b];
      for (int a = 0; a < 3; ++a)  // A = B G
        for (int b = 0; b < 3; ++b) A[a][b] = B[a][0] * G[0][b] + B[a][1] * G[1][b] + B[a][2] * G[2][b];
      for (int a = 0; a < 3; ++a)  // V = V G
        for (int b = 0; b < 3; ++b) C[a][b] = Vm[a][0] * G[0][b] + Vm[a][1] * G[1][b] + Vm[a][2] * G[2][b];
      std::memcpy(Vm, C, sizeof(C));
    }
  }
  int idx[3] = {0, 1, 2};
  std::sort(idx, idx + 3, [&](int a, int b) { return A[a][a] < A[b][b]; });
  for (int k = 0; k < 3; ++k) {
    lam[k] = A[idx[k]][idx[k]];
    double col[3] = {Vm[0][idx[k]], Vm[1][idx[k]], Vm[2][idx[k]]};
    // canonical sign: the largest-magnitude component is positive (ties: lowest index)
    int big = 0;
    for (int r = 1; r < 3; ++r)
      if (std::fabs(col[r]) > std::fabs(col[big])) big = r;
    double sg = col[big] < 0.0 ? -1.0 : 1.0;
    for (int r = 0; r < 3; ++r) vec[3 * r + k] = sg * col[r];
  }
}

// symmetric N x N eigen-decomposition by cyclic Jacobi rotations (N <= 6),
// eigenvalues ascending, eigenvectors in columns with the canonical sign
void jacobi_eigh_n(const double* Ain, int N, double* lam, double* vec) {
  double A[6][6], Vm[6][6];
  double norm = 0.0;
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      A[a][b] = 0.5 * (Ain[N * a + b] + Ain[N * b + a]);
      Vm[a][b] = (a == b) ? 1.0 : 0.0;
      norm += A[a][b] * A[a][b];
    }
  norm = std::sqrt(norm);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int a = 0; a < N; ++a)
      for (int b = a + 1; b < N; ++b) off += 2.0 * A[a][b] * A[a][b];
    off = std::sqrt(off);
    if (off <= 1e-15 * norm || off == 0.0) break;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q) {
        if (A[p][q] == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        // A <- G^T A G, V <- V G with the plane rotation G in (p, q)
        for (int k = 0; k < N; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < N; ++k) {
          const double vkp = Vm[k][p], vkq = Vm[k][q];
          Vm[k][p] = c * vkp - sn * vkq;
          Vm[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  int idx[6] = {0, 1, 2, 3, 4, 5};
  std::sort(idx, idx + N, [&](int a, int b) { return A[a][a] < A[b][b]; });
  for (int k = 0; k < N; ++k) {
    lam[k] = A[idx[k]][idx[k]];
    int big = 0;
    for (int r = 1; r < N; ++r)
      if (std::fabs(Vm[r][idx[k]]) > std::fabs(Vm[big][idx[k]])) big = r;
    const double sg = Vm[big][idx[k]] < 0.0 ? -1.0 : 1.0;
    for (int r = 0; r < N; ++r) vec[N * r + k] = sg * Vm[r][idx[k]];
  }
}

}  // namespace

// ===========================================================================
// C interface (ctypes).  Arrays are plain host memory; shapes in comments.
// cam_f: [V][16] = R(9) t(3) fx fy cx cy; cam_i: [V][3] = W H model;
// opts: [12] = tile_w tile_h near radius_sigmas dilation guard alpha_min
//              alpha_max t_min bg0 bg1 bg2.
// Returns 0 on success, nonzero on bad arguments.

extern "C" {

int orc_num_params(int deg) { return num_params(deg); }

// Per (view, Gaussian) projected record, rows of rec[V*n][12]:
// mx my A00 A01 A11 o r g b depth raw_r raw_g ... (raw_b in rec2)
// rect[V*n][4] (x0 y0 x1 y1 inclusive), tiles[V*n], depth_bits[V*n], visible[V*n]
int orc_project(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                const double* opts, double* rec /*[V*n][13]*/, int32_t* rect /*[V*n][4]*/,
                uint32_t* tiles /*[V*n]*/, uint32_t* dbits /*[V*n]*/, uint8_t* visible /*[V*n]*/) {
  if (n < 0 || V <= 0 || deg < 0 || deg > 3) return 1;
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  double th[59];
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      load_theta(params, n, deg, i, th);
      Proj<double> p;
      project(th, deg, cams[v], opt, p);
      int64_t r = (int64_t)v * n + i;
      double* o = rec + 13 * r;
      o[0] = p.mx; o[1] = p.my; o[2] = p.A00; o[3] = p.A01; o[4] = p.A11; o[5] = p.o;
      o[6] = p.rgb[0]; o[7] = p.rgb[1]; o[8] = p.rgb[2]; o[9] = p.depth;
      o[10] = p.rgb_raw[0]; o[11] = p.rgb_raw[1]; o[12] = p.rgb_raw[2];
      for (int k = 0; k < 4; ++k) rect[4 * r + k] = p.rect[k];
      visible[r] = p.visible ? 1 : 0;
      tiles[r] = p.visible ? (uint32_t)p.ntiles : 0u;
      dbits[r] = p.visible ? depth_bits(p.depth) : 0u;
    }
  return 0;
}

// Instance list: one (key, value) per (visible Gaussian, overlapped tile),
// emitted view by view, Gaussian by Gaussian, tiles row-major;
// key = global_tile << 32 | depth_f32 bits, value = v*n + i; stable sort by
// key; ranges[t] = [begin, end) of tile t (0,0 if empty).
// Call with keys == nullptr to get the count in *count.
int orc_sort(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
             const double* opts, uint64_t* count, uint64_t* keys, uint32_t* vals, uint32_t* ranges /*[Tt][2]*/) {
  if (n < 0 || V <= 0 || deg < 0 || deg > 3) return 1;
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  std::vector<std::pair<uint64_t, uint32_t>> inst;
  double th[59];
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      load_theta(params, n, deg, i, th);
      Proj<double> p;
      project(th, deg, cams[v], opt, p);
      if (!p.visible) continue;
      uint64_t db = depth_bits(p.depth);
      for (int ty = p.rect[1]; ty <= p.rect[3]; ++ty)
        for (int tx = p.rect[0]; tx <= p.rect[2]; ++tx) {
          if (!tile_hit(p, opt, tx, ty)) continue;
          uint64_t tile = (uint64_t)cams[v].tile_offset + (uint64_t)ty * cams[v].tiles_x + tx;
          inst.push_back({(tile << 32) | db, (uint32_t)((int64_t)v * n + i)});
        }
    }
  *count = inst.size();
  if (!keys) return 0;
  std::stable_sort(inst.begin(), inst.end(),
                   [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& b) { return a.first < b.first; });
  int64_t Tt = cams.back().tile_offset + (int64_t)cams.back().tiles_x * cams.back().tiles_y;
  for (int64_t t = 0; t < 2 * Tt; ++t) ranges[t] = 0;
  for (size_t k = 0; k < inst.size(); ++k) {
    keys[k] = inst[k].first;
    vals[k] = inst[k].second;
    uint64_t t = inst[k].first >> 32;
    if (k == 0 || (inst[k - 1].first >> 32) != t) ranges[2 * t] = (uint32_t)k;
    if (k + 1 == inst.size() || (inst[k + 1].first >> 32) != t) ranges[2 * t + 1] = (uint32_t)(k + 1);
  }
  return 0;
}

// Full forward + backward.  Outputs (nullable unless stated):
//   image [packed 3*Px], T_final [Px], n_used [Px] (contributing count),
//   pix_ambig [Px], loss [V] (needs target), grads [F][n] (+=), S [9][n] (+=),
//   g2d [V*n][9] and H2d [V*n][3] per-view accumulators, gauss_ambig [n],
//   grads_abs [F][n] and S_abs [9][n] (+=): the gross magnitudes of the terms
//   the gradients and S are sums of (see lift);
//   pix_ndec [Px]: cut-off decisions within their float32 band, pix_valunc
//   [Px]: an entry's alpha uncertain beyond kAlphaValue, pix_signamb [Px]:
//   bit c set when |C_c - target_c| < sign_band.
// sign_band: |C - target| below it marks the pixel ambiguous.
int orc_forward_backward(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                         const double* opts, const float* target, const double* dLdimage, double sign_band,
                         double* image, double* T_final,
                         int32_t* n_used, uint8_t* pix_ambig, double* loss, double* grads, double* S, double* g2d,
                         double* H2d, uint8_t* gauss_ambig, double* grads_abs, double* S_abs, int32_t* pix_ndec,
                         uint8_t* pix_valunc, uint8_t* pix_signamb) {
  if (n < 0 || V <= 0 || deg < 0 || deg > 3) return 1;
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  int F = num_params(deg);
  if (gauss_ambig)
    for (int64_t i = 0; i < n; ++i) gauss_ambig[i] = 0;
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    View view;
    build_view(params, n, deg, cam, opt, view);
    std::vector<Grad2D> acc(n);
    for (auto& a : acc) std::memset(&a, 0, sizeof(a));
    double inv = 1.0 / (3.0 * cam.W * cam.H);
    double lsum = 0.0;
    Pixel px;
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        int64_t pid = cam.pixel_offset + (int64_t)y * cam.W + x;
        blend_pixel(view, x, y, px);
        if (image)
          for (int ch = 0; ch < 3; ++ch) image[3 * cam.pixel_offset + (int64_t)ch * cam.W * cam.H + (int64_t)y * cam.W + x] = px.C[ch];
        if (T_final) T_final[pid] = px.T_final;
        if (n_used) n_used[pid] = (int32_t)px.list.size();
        if (pix_ndec) pix_ndec[pid] = px.ndec;
        if (pix_valunc) pix_valunc[pid] = px.valunc ? 1 : 0;
        if (pix_signamb) pix_signamb[pid] = 0;
        bool amb = px.ambig;
        if (!target && !dLdimage) {
          if (pix_ambig) pix_ambig[pid] = amb;
          continue;
        }
        double dLdC[3];
        for (int ch = 0; ch < 3; ++ch) {
          const int64_t e = 3 * cam.pixel_offset + (int64_t)ch * cam.W * cam.H + (int64_t)y * cam.W + x;
          if (dLdimage) {  // an upstream loss gradient: no L1 term
            dLdC[ch] = dLdimage[e];
            continue;
          }
          double diff = px.C[ch] - target[e];
          lsum += std::fabs(diff);
          dLdC[ch] = sgn(diff) * inv;
          if (std::fabs(diff) < sign_band) {
            amb = true;
            if (pix_signamb) pix_signamb[pid] |= (uint8_t)(1u << ch);
          }
        }
        if (pix_ambig) pix_ambig[pid] = amb;
        if (amb && gauss_ambig) mark_affected(px, gauss_ambig);
        backward_pixel(view, x, y, px, dLdC, acc, nullptr);
      }
    if (!target && !dLdimage) continue;
    if (loss) loss[v] = dLdimage ? 0.0 : lsum * inv;
    for (int64_t i = 0; i < n; ++i) {
      int64_t r = (int64_t)v * n + i;
      if (g2d)
        for (int k = 0; k < 9; ++k) g2d[9 * r + k] = acc[i].g[k];
      if (H2d)
        for (int k = 0; k < 3; ++k) H2d[3 * r + k] = acc[i].H[k];
      if (!view.rec[i].visible) continue;
      bool any = false;
      for (int k = 0; k < 9; ++k) any |= acc[i].g[k] != 0.0;
      if (!any || (!grads && !S)) continue;
      static thread_local std::vector<double> gtmp, stmp, gatmp, satmp;
      gtmp.assign(F, 0.0);
      stmp.assign(9, 0.0);
      gatmp.assign(F, 0.0);
      satmp.assign(9, 0.0);
      lift(params, n, deg, i, cam, opt, acc[i], gtmp.data(), 1, stmp.data(), 1, &view.rec[i], gatmp.data(),
           satmp.data());
      if (grads)
        for (int f = 0; f < F; ++f) grads[(int64_t)f * n + i] += gtmp[f];
      if (S)
        for (int k = 0; k < 9; ++k) S[(int64_t)k * n + i] += stmp[k];
      if (grads_abs)
        for (int f = 0; f < F; ++f) grads_abs[(int64_t)f * n + i] += gatmp[f];
      if (S_abs)
        for (int k = 0; k < 9; ++k) S_abs[(int64_t)k * n + i] += satmp[k];
    }
  }
  (void)F;
  return 0;
}

// The contribution of single pixels to the gradients and splitting matrices,
// under a chosen outcome of their in-band decisions and a chosen loss sign:
// variant k is pixel pix[k] (global packed id), blended with decision
// flip[k] flipped (-1: none), with dL/dC_c = sgnv[3k+c] / (3 H W) where
// sgnv[3k+c] is -1, 0 or 1, or (2) the sign of C_c - target_c of the
// variant's own colour; with dLdimage (packed image layout) dL/dC comes from
// there instead.  Out: rgb [nv][3], T_final [nv], used [nv] (entries
// blended), ndec [nv], valunc [nv] (nullable: an entry's alpha uncertain in
// float32 beyond kAlphaValue), and the Gaussians whose gradient or S the pixel
// changes, in CSR form: count [nv]; with gid != nullptr also gid [sum count]
// (Gaussian index), grad [sum count][F], S [sum count][9] (the pixel's term
// of Theorem 1's sum, lifted with the Gaussian's own Jacobian) and, when
// non-null, S6 [sum count][21] (its term of the dim-6 S).  Call once with
// gid == nullptr for the counts.
int orc_pixel_variants(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                       const double* opts, const float* target, const double* dLdimage, int64_t nv,
                       const int64_t* pix, const int32_t* flip, const int32_t* sgnv, double* rgb, double* T_final,
                       int32_t* used, int32_t* ndec, uint8_t* valunc, int64_t* count, int64_t* gid, double* grad,
                       double* S, double* S6) {
  if (n < 0 || V <= 0 || deg < 0 || deg > 3 || (!target && !dLdimage)) return 1;
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  const int F = num_params(deg);
  std::vector<int64_t> start(nv + 1, 0);
  if (gid) {
    for (int64_t k = 0; k < nv; ++k) start[k + 1] = start[k] + count[k];
  }
  // views are independent (every variant belongs to one view and writes only
  // its own outputs): processed on their own, in parallel with OpenMP
#pragma omp parallel for schedule(dynamic, 1)
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    bool any = false;
    for (int64_t k = 0; k < nv; ++k)
      any |= (pix[k] >= cam.pixel_offset && pix[k] < cam.pixel_offset + (int64_t)cam.W * cam.H);
    if (!any) continue;
    View view;
    build_view(params, n, deg, cam, opt, view);
    std::vector<Grad2D> acc(n);
    for (auto& a : acc) std::memset(&a, 0, sizeof(a));
    const double inv = 1.0 / (3.0 * cam.W * cam.H);
    Pixel px;
    for (int64_t k = 0; k < nv; ++k) {
      const int64_t local = pix[k] - cam.pixel_offset;
      if (local < 0 || local >= (int64_t)cam.W * cam.H) continue;
      const int x = (int)(local % cam.W), y = (int)(local / cam.W);
      blend_pixel(view, x, y, px, flip[k]);
      for (int ch = 0; ch < 3; ++ch) rgb[3 * k + ch] = px.C[ch];
      T_final[k] = px.T_final;
      used[k] = (int32_t)px.list.size();
      ndec[k] = px.ndec;
      if (valunc) valunc[k] = px.valunc ? 1 : 0;
      double dLdC[3];
      for (int ch = 0; ch < 3; ++ch) {
        const int64_t e = 3 * cam.pixel_offset + (int64_t)ch * cam.W * cam.H + (int64_t)y * cam.W + x;
        const int sg = sgnv[3 * k + ch];
        dLdC[ch] = dLdimage ? dLdimage[e] : (sg == 2 ? sgn(px.C[ch] - target[e]) : (double)sg) * inv;
      }
      backward_pixel(view, x, y, px, dLdC, acc, nullptr, S6 != nullptr);
      // the contributors, in blend order (each once)
      int64_t c = 0;
      for (const Contrib& ct : px.list) {
        const int g = ct.g;
        if (gid) {
          const int64_t o = start[k] + c;
          gid[o] = g;
          for (int f = 0; f < F; ++f) grad[o * F + f] = 0.0;
          for (int q = 0; q < 9; ++q) S[o * 9 + q] = 0.0;
          lift(params, n, deg, g, cam, opt, acc[g], grad + o * F, 1, S + o * 9, 1);
          if (S6)
            for (int q = 0; q < kH6; ++q) S6[o * kH6 + q] = acc[g].H6[q];
        }
        ++c;
      }
      for (const Contrib& ct : px.list) std::memset(&acc[ct.g], 0, sizeof(Grad2D));
      if (!gid) count[k] = c;
    }
  }
  return 0;
}

// Splitting matrices over theta = (p, log-scales) (dim 6; the paper's theta
// generalised beyond position, Sec. 4.4): S6[21][n] += sum over views and
// contributing unclamped pixels of dL/dalpha * Hessian_theta alpha, upper
// triangle row-major, theta order (p_x, p_y, p_z, s_x, s_y, s_z).  The
// loss is the fused L1 against target (or the upstream dLdimage).
int orc_split6(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
               const double* opts, const float* target, const double* dLdimage, double* S6) {
  if (n < 0 || V <= 0 || deg < 0 || deg > 3 || (!target && !dLdimage)) return 1;
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    View view;
    build_view(params, n, deg, cam, opt, view);
    std::vector<Grad2D> acc(n);
    for (auto& a : acc) std::memset(&a, 0, sizeof(a));
    const double inv = 1.0 / (3.0 * cam.W * cam.H);
    Pixel px;
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        blend_pixel(view, x, y, px);
        double dLdC[3];
        for (int ch = 0; ch < 3; ++ch) {
          const int64_t e = 3 * cam.pixel_offset + (int64_t)ch * cam.W * cam.H + (int64_t)y * cam.W + x;
          dLdC[ch] = dLdimage ? dLdimage[e] : sgn(px.C[ch] - target[e]) * inv;
        }
        backward_pixel(view, x, y, px, dLdC, acc, nullptr, true);
      }
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < kH6; ++k) S6[(int64_t)k * n + i] += acc[i].H6[k];
  }
  return 0;
}

// alpha at (u, v) of a Gaussian (its projected record in `params`-space:
// view 0 of `cam`) moved by dth in theta = (p, log-scales), maps frozen; and
// its Hessian there.  For the pins.
int orc_alpha_theta6(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i,
                     const double* opts, int64_t i, double u, double v, const double* dth, double* alpha,
                     double* H6) {
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, 1, opt);
  double th[59];
  load_theta(params, n, deg, i, th);
  Proj<double> g;
  project(th, deg, cams[0], opt, g);
  if (g.depth <= opt.near_z) return 1;
  *alpha = alpha_theta6<double>(g, opt.dilation, u, v, dth);
  if (H6) alpha_hessian_theta6(g, opt.dilation, u, v, H6);
  return 0;
}

// Loss only (sum over views of the per-view mean L1), for finite differences.
double orc_loss(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                const double* opts, const float* target) {
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  double total = 0.0;
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    View view;
    build_view(params, n, deg, cam, opt, view);
    Pixel px;
    double lsum = 0.0;
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        blend_pixel(view, x, y, px);
        for (int ch = 0; ch < 3; ++ch)
          lsum += std::fabs(px.C[ch] - target[3 * cam.pixel_offset + (int64_t)ch * cam.W * cam.H + (int64_t)y * cam.W + x]);
      }
    total += lsum / (3.0 * cam.W * cam.H);
  }
  return total;
}

// Colour and final transmittance of sampled pixels (global packed pixel ids).
int orc_render_pixels(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                      const double* opts, const int64_t* pix, int64_t npix, double* rgb /*[npix][3]*/,
                      double* T_final, uint8_t* ambig) {
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    bool any = false;
    for (int64_t k = 0; k < npix; ++k) any |= (pix[k] >= cam.pixel_offset && pix[k] < cam.pixel_offset + (int64_t)cam.W * cam.H);
    if (!any) continue;
    View view;
    build_view(params, n, deg, cam, opt, view);
    Pixel px;
    for (int64_t k = 0; k < npix; ++k) {
      int64_t local = pix[k] - cam.pixel_offset;
      if (local < 0 || local >= (int64_t)cam.W * cam.H) continue;
      int x = (int)(local % cam.W), y = (int)(local / cam.W);
      blend_pixel(view, x, y, px);
      for (int ch = 0; ch < 3; ++ch) rgb[3 * k + ch] = px.C[ch];
      if (T_final) T_final[k] = px.T_final;
      if (ambig) ambig[k] = px.ambig;
    }
  }
  return 0;
}

// Gradients and splitting matrices of sampled Gaussians only: every pixel of
// every tile the sampled Gaussian touches is blended in full, its L1
// gradient formed, and the reverse sweep credited to the sampled Gaussians.
// grads [ns][F], S [ns][9], ambig [ns]; flagged (nullable, capacity
// flag_cap): the global ids of the pixels with an in-band decision, an
// uncertain alpha or an L1 sign within sign_band of zero that touch a sampled
// Gaussian, their number in *nflagged (returns 2 when they do not fit).
int orc_grads_sampled(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                      const double* opts, const float* target, double sign_band, const int64_t* gids, int64_t ns,
                      double* grads, double* S, uint8_t* ambig, int64_t* flagged, int64_t flag_cap,
                      int64_t* nflagged) {
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  int F = num_params(deg);
  std::vector<uint8_t> want(n, 0);
  for (int64_t k = 0; k < ns; ++k) want[gids[k]] = 1;
  // views are independent: each is processed on its own (in parallel when
  // the library is built with OpenMP) into its own buffers, and the buffers
  // are summed in view order afterwards, so the result does not depend on
  // the number of threads
  std::vector<std::vector<double>> vg(V, std::vector<double>(ns * F, 0.0)), vS(V, std::vector<double>(ns * 9, 0.0));
  std::vector<std::vector<int64_t>> vflag(V);
  std::vector<std::vector<uint8_t>> vamb(V);
#pragma omp parallel for schedule(dynamic, 1)
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    View view;
    build_view(params, n, deg, cam, opt, view);
    std::vector<uint8_t> tile_needed((size_t)cam.tiles_x * cam.tiles_y, 0);
    for (int64_t k = 0; k < ns; ++k) {
      const Proj<double>& p = view.rec[gids[k]];
      if (!p.visible) continue;
      for (int ty = p.rect[1]; ty <= p.rect[3]; ++ty)
        for (int tx = p.rect[0]; tx <= p.rect[2]; ++tx) tile_needed[(size_t)ty * cam.tiles_x + tx] = 1;
    }
    std::vector<Grad2D> acc(n);
    for (auto& a : acc) std::memset(&a, 0, sizeof(a));
    std::vector<uint8_t> gamb(n, 0);
    double inv = 1.0 / (3.0 * cam.W * cam.H);
    Pixel px;
    for (int ty = 0; ty < cam.tiles_y; ++ty)
      for (int tx = 0; tx < cam.tiles_x; ++tx) {
        if (!tile_needed[(size_t)ty * cam.tiles_x + tx]) continue;
        for (int y = ty * opt.th; y < std::min(cam.H, (ty + 1) * opt.th); ++y)
          for (int x = tx * opt.tw; x < std::min(cam.W, (tx + 1) * opt.tw); ++x) {
            blend_pixel(view, x, y, px);
            double dLdC[3];
            bool amb = px.ambig;
            for (int ch = 0; ch < 3; ++ch) {
              double tg = target[3 * cam.pixel_offset + (int64_t)ch * cam.W * cam.H + (int64_t)y * cam.W + x];
              double diff = px.C[ch] - tg;
              dLdC[ch] = sgn(diff) * inv;
              if (std::fabs(diff) < sign_band) amb = true;
            }
            if (amb) {
              mark_affected(px, gamb.data());
              bool touches = false;
              for (const Contrib& c : px.list) touches |= want[c.g] != 0;
              for (int g : px.amb_ids) touches |= want[g] != 0;
              if (touches) vflag[v].push_back(cam.pixel_offset + (int64_t)y * cam.W + x);
            }
            backward_pixel(view, x, y, px, dLdC, acc, &want);
          }
      }
    for (int64_t k = 0; k < ns; ++k) {
      int64_t i = gids[k];
      if (!view.rec[i].visible) continue;
      lift(params, n, deg, i, cam, opt, acc[i], vg[v].data() + k * F, 1, vS[v].data() + k * 9, 1);
    }
    vamb[v].assign(ns, 0);
    for (int64_t k = 0; k < ns; ++k) vamb[v][k] = gamb[gids[k]];
  }
  for (int64_t k = 0; k < ns; ++k) {
    ambig[k] = 0;
    for (int f = 0; f < F; ++f) grads[k * F + f] = 0.0;
    for (int q = 0; q < 9; ++q) S[k * 9 + q] = 0.0;
  }
  int64_t nf = 0;
  for (int v = 0; v < V; ++v) {
    for (int64_t k = 0; k < ns * F; ++k) grads[k] += vg[v][k];
    for (int64_t k = 0; k < ns * 9; ++k) S[k] += vS[v][k];
    for (int64_t k = 0; k < ns; ++k) ambig[k] |= vamb[v][k];
    for (int64_t p : vflag[v]) {
      if (flagged && nf < flag_cap) flagged[nf] = p;
      ++nf;
    }
  }
  if (nflagged) *nflagged = nf;
  return (nflagged && nf > flag_cap) ? 2 : 0;
}

// Loss after splitting Gaussian i into two offspring at p +/- eps*delta with
// weights 1/2 that share the parent's slot in every blend (the replacement of
// sigma_i by sum_j w_j sigma_j of Sec. 4.1); other parameters unchanged.
double orc_loss_merged_split(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                             const double* opts, const float* target, int64_t gi, const double* delta, double eps) {
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  double total = 0.0;
  double th[59], thp[59], thm[59];
  load_theta(params, n, deg, gi, th);
  std::memcpy(thp, th, sizeof(th));
  std::memcpy(thm, th, sizeof(th));
  for (int k = 0; k < 3; ++k) {
    thp[k] = th[k] + eps * delta[k];
    thm[k] = th[k] - eps * delta[k];
  }
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    View view;
    build_view(params, n, deg, cam, opt, view);
    Proj<double> cp, cm;
    project(thp, deg, cam, opt, cp);
    project(thm, deg, cam, opt, cm);
    double lsum = 0.0;
    for (int y = 0; y < cam.H; ++y)
      for (int x = 0; x < cam.W; ++x) {
        const std::vector<int>& lst = view.tiles[(size_t)(y / opt.th) * cam.tiles_x + (x / opt.tw)];
        double T = 1.0, C[3] = {0, 0, 0};
        for (size_t j = 0; j < lst.size(); ++j) {
          const Proj<double>& g = view.rec[lst[j]];
          double a, rgb[3];
          if (lst[j] == gi) {
            a = 0.0;
            for (int ch = 0; ch < 3; ++ch) rgb[ch] = g.rgb[ch];
            if (cp.visible) a += 0.5 * alpha_in_footprint(cp, opt, (double)x, (double)y);
            if (cm.visible) a += 0.5 * alpha_in_footprint(cm, opt, (double)x, (double)y);
          } else {
            a = alpha_in_footprint(g, opt, (double)x, (double)y);
            for (int ch = 0; ch < 3; ++ch) rgb[ch] = g.rgb[ch];
          }
          if (a > opt.alpha_max) a = opt.alpha_max;
          if (a < opt.alpha_min) continue;
          double Tn = T * (1.0 - a);
          if (Tn < opt.t_min) break;
          for (int ch = 0; ch < 3; ++ch) C[ch] += rgb[ch] * a * T;
          T = Tn;
        }
        for (int ch = 0; ch < 3; ++ch) {
          C[ch] += T * opt.bg[ch];
          lsum += std::fabs(C[ch] - target[3 * cam.pixel_offset + (int64_t)ch * cam.W * cam.H + (int64_t)y * cam.W + x]);
        }
      }
    total += lsum / (3.0 * cam.W * cam.H);
  }
  return total;
}

// Real SH basis at m unit directions: out[m][(deg+1)^2]
void orc_sh_basis(int deg, const double* dirs, int64_t m, double* out) {
  int nb = (deg + 1) * (deg + 1);
  for (int64_t k = 0; k < m; ++k) sh_basis(deg, dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2], out + k * nb);
}

// alpha (before clamping) and its mean-Hessian at a pixel
double orc_alpha(const double* g6, double u, double v) { return alpha_raw(g6[0], g6[1], g6[2], g6[3], g6[4], g6[5], u, v); }
void orc_alpha_hessian(const double* g6, double u, double v, double* H3) {
  alpha_hessian_mu(g6[0], g6[1], g6[2], g6[3], g6[4], g6[5], u, v, H3);
}

// Symmetric eigen-decomposition of m matrices S[m][9] (row-major 3x3):
// lam[m][3] ascending, vec[m][9] with eigenvectors in columns (canonical sign).
void orc_eigh(const double* S, int64_t m, double* lam, double* vec) {
  for (int64_t k = 0; k < m; ++k) jacobi_eigh(S + 9 * k, lam + 3 * k, vec + 9 * k);
}

// Steepest Density Control over all Gaussians.  S is [9][n] (row-major 3x3 per
// Gaussian, any scale); s_scale multiplies it first (Algorithm 1 averages the
// accumulated matrix over the densification interval).  out_params is
// [F][out_cap] doubles; returns n_out (or -1 if out_cap is too small, with
// *needed set).  lam_min [n], vmin [3][n], split [n].
// Steepest Density Control (Theorem 2, Algorithm 1) with the two variants of
// the paper's "Variants" section:
//  - compactest splitting: a Gaussian is a candidate only if, besides
//    lambda_min < eps_split, its averaged position gradient G (Algorithm 1's
//    accumulator, times g_scale) has norm <= eps_grad (G == nullptr or
//    eps_grad <= 0: no gradient condition);
//  - ADC-style gate (Algorithm 1's "condition on G" in the form of the
//    adaptive density control the Variants section compares with): a
//    candidate only if also the averaged per-step norm of the position
//    gradient, g_scale * Gabs, is >= adc_tau (Gabs == nullptr or
//    adc_tau <= 0: off);
//  - increment budget: when more than `budget` Gaussians are candidates
//    (budget > 0), only the `budget` candidates with the smallest lambda_min
//    split (ties: lower index first), since the loss decrease of a split is
//    proportional to lambda_min / 2 (Theorem 2).
int64_t orc_densify(const float* params, int64_t n, int deg, const double* S, double s_scale, double eps,
                    double eps_split, const float* G, double g_scale, double eps_grad, const float* Gabs,
                    double adc_tau, int64_t budget, double* out_params, int64_t out_cap, double* lam_min, double* vmin, uint8_t* split,
                    int64_t* needed) {
  int F = num_params(deg);
  std::vector<int64_t> cand;
  for (int64_t i = 0; i < n; ++i) {
    double M[9], lam[3], vec[9];
    for (int k = 0; k < 9; ++k) M[k] = s_scale * S[(int64_t)k * n + i];
    jacobi_eigh(M, lam, vec);
    lam_min[i] = lam[0];
    for (int r = 0; r < 3; ++r) vmin[(int64_t)r * n + i] = vec[3 * r + 0];
    bool c = lam[0] < eps_split;
    if (c && G && eps_grad > 0.0) {
      double g2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        double g = g_scale * (double)G[(int64_t)k * n + i];
        g2 = g2 + g * g;
      }
      c = g2 <= eps_grad * eps_grad;
    }
    if (c && Gabs && adc_tau > 0.0) c = g_scale * (double)Gabs[i] >= adc_tau;
    split[i] = 0;
    if (c) cand.push_back(i);
  }
  if (budget > 0 && (int64_t)cand.size() > budget) {
    std::stable_sort(cand.begin(), cand.end(), [&](int64_t a, int64_t b) { return lam_min[a] < lam_min[b]; });
    cand.resize(budget);
  }
  for (int64_t i : cand) split[i] = 1;
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + 1 + split[i];
  *needed = off[n];
  if (off[n] > out_cap) return -1;
  for (int64_t i = 0; i < n; ++i) {
    int64_t o = off[i];
    for (int f = 0; f < F; ++f) {
      double x = params[(int64_t)f * n + i];
      out_params[(int64_t)f * out_cap + o] = x;
      if (split[i]) out_params[(int64_t)f * out_cap + o + 1] = x;
    }
    if (!split[i]) continue;
    for (int k = 0; k < 3; ++k) {
      double p = params[(int64_t)k * n + i], d = vmin[(int64_t)k * n + i];
      out_params[(int64_t)k * out_cap + o] = p + eps * d;
      out_params[(int64_t)k * out_cap + o + 1] = p - eps * d;
    }
    double op = 1.0 / (1.0 + std::exp(-(double)params[(int64_t)10 * n + i]));
    double oh = 0.5 * op;
    double logit = std::log(oh / (1.0 - oh));
    out_params[(int64_t)10 * out_cap + o] = logit;
    out_params[(int64_t)10 * out_cap + o + 1] = logit;
  }
  return off[n];
}

// Steepest Density Control over theta = (p, log-scales): S6 [21][n] (upper
// triangle of the 6x6 splitting matrix, any scale) times s_scale; split iff
// lambda_min < eps_split; the offspring move by +-eps v_min in theta (both the
// position and the log-scales) and take o/2; other rows copied.  Same layout
// as orc_densify; vmin [6][n].
int64_t orc_densify6(const float* params, int64_t n, int deg, const double* S6, double s_scale, double eps,
                     double eps_split, double* out_params, int64_t out_cap, double* lam_min, double* vmin,
                     uint8_t* split, int64_t* needed) {
  const int F = num_params(deg);
  for (int64_t i = 0; i < n; ++i) {
    double M[36], lam[6], vec[36];
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) M[6 * a + b] = s_scale * S6[(int64_t)h6(a, b) * n + i];
    jacobi_eigh_n(M, 6, lam, vec);
    lam_min[i] = lam[0];
    for (int r = 0; r < 6; ++r) vmin[(int64_t)r * n + i] = vec[6 * r + 0];
    split[i] = lam[0] < eps_split ? 1 : 0;
  }
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + 1 + split[i];
  *needed = off[n];
  if (off[n] > out_cap) return -1;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = off[i];
    for (int f = 0; f < F; ++f) {
      const double x = params[(int64_t)f * n + i];
      out_params[(int64_t)f * out_cap + o] = x;
      if (split[i]) out_params[(int64_t)f * out_cap + o + 1] = x;
    }
    if (!split[i]) continue;
    for (int k = 0; k < 6; ++k) {  // rows 0-2 position, 3-5 log-scales
      const double x = params[(int64_t)k * n + i], d = vmin[(int64_t)k * n + i];
      out_params[(int64_t)k * out_cap + o] = x + eps * d;
      out_params[(int64_t)k * out_cap + o + 1] = x - eps * d;
    }
    const double op = 1.0 / (1.0 + std::exp(-(double)params[(int64_t)10 * n + i]));
    const double oh = 0.5 * op;
    const double logit = std::log(oh / (1.0 - oh));
    out_params[(int64_t)10 * out_cap + o] = logit;
    out_params[(int64_t)10 * out_cap + o + 1] = logit;
  }
  return off[n];
}

// eigen-decomposition of m symmetric N x N matrices (N <= 6) S[m][N*N]
void orc_eigh_n(const double* S, int64_t m, int N, double* lam, double* vec) {
  for (int64_t k = 0; k < m; ++k) jacobi_eigh_n(S + (int64_t)N * N * k, N, lam + N * k, vec + (int64_t)N * N * k);
}

}  // extern "C"

extern "C" {

// Instance lists of selected global tiles (the values a sorted instance list
// holds in each tile's range): records r = v*n + i whose footprint holds the
// tile, ordered by (depth float bits, r).  counts[k] = list length of tile k;
// lists is filled back to back when non-null (call once with nullptr for the
// counts).
int orc_tile_lists(const float* params, int64_t n, int deg, const float* cam_f, const int32_t* cam_i, int V,
                   const double* opts, const int64_t* tiles, int64_t nt, int64_t* counts, uint32_t* lists) {
  Opts opt = read_opts(opts);
  std::vector<Cam> cams = read_cams(cam_f, cam_i, V, opt);
  std::vector<std::vector<uint32_t>> out(nt);
  double th[59];
  for (int v = 0; v < V; ++v) {
    const Cam& cam = cams[v];
    int64_t first = cam.tile_offset, last = cam.tile_offset + (int64_t)cam.tiles_x * cam.tiles_y;
    bool any = false;
    for (int64_t k = 0; k < nt; ++k) any |= tiles[k] >= first && tiles[k] < last;
    if (!any) continue;
    std::vector<Proj<double>> rec(n);
    for (int64_t i = 0; i < n; ++i) {
      load_theta(params, n, deg, i, th);
      project(th, deg, cam, opt, rec[i]);
    }
    for (int64_t k = 0; k < nt; ++k) {
      if (tiles[k] < first || tiles[k] >= last) continue;
      int tx = (int)((tiles[k] - first) % cam.tiles_x), ty = (int)((tiles[k] - first) / cam.tiles_x);
      std::vector<std::pair<uint32_t, uint32_t>> items;
      for (int64_t i = 0; i < n; ++i) {
        const Proj<double>& p = rec[i];
        if (!p.visible || tx < p.rect[0] || tx > p.rect[2] || ty < p.rect[1] || ty > p.rect[3]) continue;
        if (!tile_hit(p, opt, tx, ty)) continue;
        items.push_back({depth_bits(p.depth), (uint32_t)((int64_t)v * n + i)});
      }
      std::sort(items.begin(), items.end());
      for (auto& it : items) out[k].push_back(it.second);
    }
  }
  int64_t pos = 0;
  for (int64_t k = 0; k < nt; ++k) {
    counts[k] = (int64_t)out[k].size();
    if (lists)
      for (uint32_t r : out[k]) lists[pos++] = r;
  }
  return 0;
}

}  // extern "C"
