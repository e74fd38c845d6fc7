// Stage 5: Steepest Density Control (Theorem 2, Algorithm 1) with the
// closed-form 3x3 eigensolve of App. A.3.
//
// Kernel 1, one thread per Gaussian: S' = s_scale * S, smallest eigenpair by
// the trigonometric root formula (fp64), split flag lambda_min < eps_split
// (and the optional gradient gate); an optional budget then keeps only the
// candidates with the smallest lambda_min (radix select).
// An exclusive scan of the flags places the output: Gaussian i lands at
// i + (#splits before i), a split one occupies two slots.  Kernel 2 scatters
// the parent, or the two offspring p +/- eps v_min with opacity o/2 (the
// logit re-derived) and every other attribute copied.
#include <algorithm>

#include "common.h"
#include "scan.h"

namespace sg {

// smallest eigenpair of a symmetric 3x3 matrix given as xx xy xz yy yz zz
SG_DEV void eig3_min(const double s[6], double& lam_min, double v[3]) {
  const double a00 = s[0], a01 = s[1], a02 = s[2], a11 = s[3], a12 = s[4], a22 = s[5];
  const double q = (a00 + a11 + a22) / 3.0;
  const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * (a01 * a01 + a02 * a02 + a12 * a12);
  v[0] = 1.0;
  v[1] = 0.0;
  v[2] = 0.0;
  if (!(p2 > 0.0)) {  // A = q I: every vector is an eigenvector
    lam_min = q;
    return;
  }
  const double p = sqrt(p2 / 6.0);
  const double ip = 1.0 / p;
  // B = (A - q I) / p;  det(B) / 2 = cos(3 theta)
  const double c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip, c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
  const double detB = c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02);
  double r = 0.5 * detB;
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  const double phi = acos(r) / 3.0;
  // roots q + 2 p cos(phi + 2 k pi / 3); k = 1 is the smallest
  lam_min = q + 2.0 * p * cos(phi + 2.0943951023931957);  // 2 pi / 3
  // eigenvector: null direction of A - lambda I from the largest row cross product
  const double r0[3] = {a00 - lam_min, a01, a02};
  const double r1[3] = {a01, a11 - lam_min, a12};
  const double r2[3] = {a02, a12, a22 - lam_min};
  // (the best candidate is kept by value: indexing arrays with a run-time
  // choice would place them in scratch memory)
  const double* rows[3][2] = {{r0, r1}, {r0, r2}, {r1, r2}};
  double best = -1.0, cb0 = 0.0, cb1 = 0.0, cb2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double* u = rows[k][0];
    const double* w = rows[k][1];
    const double x = u[1] * w[2] - u[2] * w[1];
    const double y = u[2] * w[0] - u[0] * w[2];
    const double z = u[0] * w[1] - u[1] * w[0];
    const double nn = x * x + y * y + z * z;
    if (nn > best) {
      best = nn;
      cb0 = x;
      cb1 = y;
      cb2 = z;
    }
  }
  const double scale2 = p2 * p2;  // |A - q I|^4 sets the scale of a cross product's square norm
  if (best > 1e-24 * scale2) {
    const double inv = 1.0 / sqrt(best);
    v[0] = cb0 * inv;
    v[1] = cb1 * inv;
    v[2] = cb2 * inv;
  } else {
    // lambda_min repeated: A - lambda I has rank <= 1; any unit vector
    // orthogonal to its largest row is an eigenvector
    const double* rr[3] = {r0, r1, r2};
    double bn = -1.0, u0 = 0.0, u1 = 0.0, u2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double nn = rr[k][0] * rr[k][0] + rr[k][1] * rr[k][1] + rr[k][2] * rr[k][2];
      if (nn > bn) {
        bn = nn;
        u0 = rr[k][0];
        u1 = rr[k][1];
        u2 = rr[k][2];
      }
    }
    if (bn > 1e-24 * p2) {
      int ax = 0;  // axis least aligned with u
      if (fabs(u1) < fabs(u0)) ax = 1;
      if (fabs(u2) < fabs(ax == 0 ? u0 : u1)) ax = 2;
      const double e0 = ax == 0 ? 1.0 : 0.0, e1 = ax == 1 ? 1.0 : 0.0, e2 = ax == 2 ? 1.0 : 0.0;
      const double t0 = u1 * e2 - u2 * e1, t1 = u2 * e0 - u0 * e2, t2 = u0 * e1 - u1 * e0;
      const double inv = 1.0 / sqrt(t0 * t0 + t1 * t1 + t2 * t2);
      v[0] = t0 * inv;
      v[1] = t1 * inv;
      v[2] = t2 * inv;
    }
  }
  // canonical sign: largest-magnitude component positive (ties: lowest index)
  int big = 0;
  if (fabs(v[1]) > fabs(v[big])) big = 1;
  if (fabs(v[2]) > fabs(v[big])) big = 2;
  if (v[big] < 0.0) {
    v[0] = -v[0];
    v[1] = -v[1];
    v[2] = -v[2];
  }
}

// order-preserving map of a float to an unsigned key
SG_DEV uint32_t float_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ void __launch_bounds__(256) k_densify_eig(const float* __restrict__ S, int64_t n, float s_scale,
                                                     float eps_split, const float* __restrict__ G, float g_scale,
                                                     float eps_grad, const float* __restrict__ Gabs, float adc_tau,
                                                     float* __restrict__ lam_out,
                                                     float* __restrict__ v_out, uint32_t* __restrict__ flag,
                                                     uint32_t* __restrict__ key) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s[6];
  for (int k = 0; k < 6; ++k) s[k] = (double)s_scale * (double)S[k * n + i];
  double lam, v[3];
  eig3_min(s, lam, v);
  const float lam32 = (float)lam;
  lam_out[i] = lam32;
  for (int k = 0; k < 3; ++k) v_out[k * n + i] = (float)v[k];
  bool cand = lam < (double)eps_split;
  if (cand && G && eps_grad > 0.f) {  // compactest gate on the averaged position gradient
    double g2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double g = (double)g_scale * (double)G[k * n + i];
      g2 = g2 + g * g;
    }
    cand = g2 <= (double)eps_grad * (double)eps_grad;
  }
  // ADC-style gate on the averaged per-step norm of the position gradient
  if (cand && Gabs && adc_tau > 0.f) cand = (double)g_scale * (double)Gabs[i] >= (double)adc_tau;
  flag[i] = cand ? 1u : 0u;
  if (key) key[i] = float_key(lam32);
}

// ---------------------------------------------------------------------------
// increment budget: the `budget` candidates with the smallest float32
// lambda_min (ties: lower index).  A four-pass radix select (8 bits per pass,
// most significant first) finds the key of the budget-th smallest candidate;
// state lives in device memory so the stage stays graph-capturable.

struct SelectState {
  uint32_t prefix;   // key bits fixed so far
  uint32_t remain;   // how many still to take among keys matching the prefix
  uint32_t all;      // 1: the budget does not bind, every candidate splits
  uint32_t pad;
};

__global__ void k_select_init(SelectState* st, uint32_t* __restrict__ hist, int64_t budget) {
  const int t = threadIdx.x;
  for (int k = t; k < 4 * 256; k += blockDim.x) hist[k] = 0u;
  if (t == 0) {
    st->prefix = 0u;
    st->remain = (uint32_t)budget;
    st->all = 0u;
  }
}

__global__ void __launch_bounds__(256) k_select_hist(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ key,
                                                     int64_t n, int pass, const SelectState* __restrict__ st,
                                                     uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int shift = 24 - 8 * pass;
  const uint32_t hmask = pass == 0 ? 0u : (0xFFFFFFFFu << (32 - 8 * pass));
  const uint32_t prefix = st->prefix;
  const bool live = st->all == 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; live && i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    const uint32_t k = key[i];
    if ((k & hmask) == (prefix & hmask)) atomicAdd(&h[(k >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  const uint32_t c = h[threadIdx.x];
  if (c) atomicAdd(&hist[pass * 256 + threadIdx.x], c);
}

__global__ void k_select_pick(SelectState* st, const uint32_t* __restrict__ hist, int pass) {
  if (threadIdx.x != 0 || st->all) return;
  const uint32_t* h = hist + pass * 256;
  if (pass == 0) {
    uint64_t total = 0;
    for (int d = 0; d < 256; ++d) total += h[d];
    if (total <= st->remain) {
      st->all = 1u;
      return;
    }
  }
  uint32_t below = 0;
  int d = 0;
  for (; d < 255; ++d) {
    if (below + h[d] >= st->remain) break;
    below += h[d];
  }
  st->prefix |= (uint32_t)d << (24 - 8 * pass);
  st->remain -= below;
}

// candidates whose key equals the selected key, in index order (for the tie rule)
struct LoadTies {
  const uint32_t* flag;
  const uint32_t* key;
  const SelectState* st;
  SG_DEV uint32_t operator()(int64_t i) const {
    return (st->all == 0u && flag[i] && key[i] == st->prefix) ? 1u : 0u;
  }
};

__global__ void __launch_bounds__(256) k_select_apply(uint32_t* __restrict__ flag, const uint32_t* __restrict__ key,
                                                      const uint32_t* __restrict__ tie_rank, int64_t n,
                                                      const SelectState* __restrict__ st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || st->all || !flag[i]) return;
  const uint32_t k = key[i];
  const bool take = k < st->prefix || (k == st->prefix && tie_rank[i] < st->remain);
  if (!take) flag[i] = 0u;
}

struct LoadFlags {
  const uint32_t* f;
  SG_DEV uint32_t operator()(int64_t i) const { return f[i]; }
};

__global__ void k_densify_total(const uint32_t* __restrict__ total, int64_t n, int64_t cap, int64_t* __restrict__ n_out,
                                int32_t* __restrict__ status) {
  const int64_t need = n + (int64_t)*total;
  *n_out = need;
  *status = need > cap ? (int32_t)STEEPGS_ERR_CAPACITY : (int32_t)STEEPGS_OK;
}

// rows: the leading parameter rows the offspring move along +-eps v_min (3:
// the position; 6: the position and the log-scales)
__global__ void __launch_bounds__(256) k_densify_scatter(const float* __restrict__ params, int64_t n, int F,
                                                         const uint32_t* __restrict__ flag,
                                                         const uint32_t* __restrict__ before,
                                                         const float* __restrict__ vmin, int rows, float eps,
                                                         float* __restrict__ out, int64_t cap,
                                                         const int32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || *status != STEEPGS_OK) return;
  const int64_t o = i + (int64_t)before[i];
  const bool split = flag[i] != 0u;
  for (int f = 0; f < F; ++f) {
    const float x = params[(int64_t)f * n + i];
    out[(int64_t)f * cap + o] = x;
    if (split) out[(int64_t)f * cap + o + 1] = x;
  }
  if (!split) return;
  for (int k = 0; k < rows; ++k) {
    const double p = params[(int64_t)k * n + i];
    const double d = (double)eps * (double)vmin[k * n + i];
    out[(int64_t)k * cap + o] = (float)(p + d);
    out[(int64_t)k * cap + o + 1] = (float)(p - d);
  }
  // opacity halved in [0, 1]; stored as a logit
  const double op = 1.0 / (1.0 + exp(-(double)params[(int64_t)STEEPGS_ROW_OPACITY * n + i]));
  const double half = 0.5 * op;
  const float logit = (float)log(half / (1.0 - half));
  out[(int64_t)STEEPGS_ROW_OPACITY * cap + o] = logit;
  out[(int64_t)STEEPGS_ROW_OPACITY * cap + o + 1] = logit;
}

struct DensWs {
  float* lam;
  float* vmin;
  uint32_t* flag;
  uint32_t* before;
  uint32_t* partials;
  uint32_t* key;
  uint32_t* hist;
  SelectState* state;
};

static size_t densify_layout(void* base, int64_t n, DensWs& w) {
  Carver c(base);
  w.lam = c.take<float>(n);
  w.vmin = c.take<float>(6 * n);  // room for the dim-6 eigenvectors
  w.flag = c.take<uint32_t>(n);
  w.before = c.take<uint32_t>(n);
  w.partials = c.take<uint32_t>(scan_partials_count(n) + 1);
  w.key = c.take<uint32_t>(n);
  w.hist = c.take<uint32_t>(4 * 256);
  w.state = c.take<SelectState>(1);
  return c.used + 256;
}

size_t densify_workspace(int64_t n) {
  DensWs w;
  return densify_layout(nullptr, n, w);
}

__global__ void k_copy_f32(const float* __restrict__ a, float* __restrict__ b, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = a[i];
}

__global__ void k_flag_u8(const uint32_t* __restrict__ f, uint8_t* __restrict__ o, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) o[i] = (uint8_t)f[i];
}

__global__ void k_densify_empty(int64_t* n_out, int32_t* status) {
  *n_out = 0;
  *status = STEEPGS_OK;
}

// ---------------------------------------------------------------------------
// splitting matrix over theta = (p, log-scales): smallest eigenpair of a
// symmetric 6x6 by cyclic Jacobi rotations in fp64 (no closed form beyond 4x4)

SG_DEV int h6_index(int i, int j) { return i <= j ? i * 6 - i * (i - 1) / 2 + (j - i) : j * 6 - j * (j - 1) / 2 + (i - j); }

SG_DEV void eig6_min(const double s[21], double& lam_min, double v[6]) {
  // the symmetric matrix as its upper triangle (h6_index; every index below
  // is a compile-time constant once the loops are unrolled) and the
  // accumulated rotations
  double A[21], Q[6][6];
  double norm2 = 0.0;
#pragma unroll
  for (int k = 0; k < 21; ++k) A[k] = s[k];
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      norm2 += A[h6_index(a, b)] * A[h6_index(a, b)];
      Q[a][b] = a == b ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a + 1; b < 6; ++b) off += A[h6_index(a, b)] * A[h6_index(a, b)];
    if (!(2.0 * off > 1e-30 * norm2)) break;
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int q = p + 1; q < 6; ++q) {
        const double apq = A[h6_index(p, q)];
        if (apq == 0.0) continue;
        // the plane rotation (p, q) that zeroes A[p][q]: t = tan of its
        // angle, the smaller root of t^2 + 2 th t - 1 = 0
        const double th = (A[h6_index(q, q)] - A[h6_index(p, p)]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        // J^T A J touches rows and columns p and q only
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          if (k == p || k == q) continue;
          const double akp = A[h6_index(k, p)], akq = A[h6_index(k, q)];
          A[h6_index(k, p)] = c * akp - sn * akq;
          A[h6_index(k, q)] = sn * akp + c * akq;
        }
        A[h6_index(p, p)] -= t * apq;
        A[h6_index(q, q)] += t * apq;
        A[h6_index(p, q)] = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const double qkp = Q[k][p], qkq = Q[k][q];
          Q[k][p] = c * qkp - sn * qkq;
          Q[k][q] = sn * qkp + c * qkq;
        }
      }
  }
  // the smallest diagonal entry, tracked by value (indexing A with the
  // run-time m would place the matrix in scratch memory)
  int m = 0;
  lam_min = A[h6_index(0, 0)];
#pragma unroll
  for (int k = 1; k < 6; ++k)
    if (A[h6_index(k, k)] < lam_min) {
      lam_min = A[h6_index(k, k)];
      m = k;
    }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int r = 0; r < 6; ++r)
      if (k == m) v[r] = Q[r][k];
  }
  // canonical sign: largest-magnitude component positive (ties: lowest index)
  int big = 0;
#pragma unroll
  for (int r = 1; r < 6; ++r)
    if (fabs(v[r]) > fabs(v[big])) big = r;
  const double sg = v[big] < 0.0 ? -1.0 : 1.0;
#pragma unroll
  for (int r = 0; r < 6; ++r) v[r] *= sg;
}

__global__ void __launch_bounds__(128) k_densify6_eig(const float* __restrict__ S6, int64_t n, float s_scale,
                                                      float eps_split, float* __restrict__ lam_out,
                                                      float* __restrict__ v_out, uint32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) s[k] = (double)s_scale * (double)S6[k * n + i];
  double lam, v[6];
  eig6_min(s, lam, v);
  lam_out[i] = (float)lam;
#pragma unroll
  for (int k = 0; k < 6; ++k) v_out[k * n + i] = (float)v[k];
  flag[i] = lam < (double)eps_split ? 1u : 0u;
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_densify(const float* d_params, int64_t n, int32_t sh_degree, const float* d_S,
                                          float s_scale, float eps, float eps_split,
                                          const steepgs_split_select* select, float* d_out,
                                          int64_t out_capacity, int64_t* d_n_out, float* d_lambda_min, float* d_vmin,
                                          uint8_t* d_split, int32_t* d_status, void* d_ws, size_t ws_bytes,
                                          void* stream) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || out_capacity < 0 || !d_n_out || !d_status)
    return STEEPGS_ERR_INVALID_ARG;
  if (n >= (int64_t)1 << 31) return STEEPGS_ERR_INVALID_ARG;
  hipStream_t st = as_stream(stream);
  if (n == 0) {
    hipLaunchKernelGGL(k_densify_empty, dim3(1), dim3(1), 0, st, d_n_out, d_status);
    SG_TRY_LAUNCH();
    return STEEPGS_OK;
  }
  if (!d_params || !d_S || (out_capacity > 0 && !d_out)) return STEEPGS_ERR_INVALID_ARG;
  DensWs w;
  const size_t need = densify_layout(nullptr, n, w);
  if (!d_ws || ws_bytes < need) return STEEPGS_ERR_WORKSPACE;
  densify_layout(d_ws, n, w);
  const int F = STEEPGS_NUM_PARAMS(sh_degree);
  const unsigned nb = (unsigned)ceil_div(n, 256);
  const float* G = select ? select->d_G : nullptr;
  const float g_scale = select ? select->g_scale : 1.f;
  const float eps_grad = select ? select->eps_grad : 0.f;
  const int64_t budget = select ? select->budget : 0;
  const float* Gabs = select ? select->d_Gabs : nullptr;
  const float adc_tau = select ? select->adc_tau : 0.f;
  if (budget >= (int64_t)1 << 32) return STEEPGS_ERR_INVALID_ARG;
  timer_begin(STEEPGS_TIMER_DENSIFY, st);
  hipLaunchKernelGGL(k_densify_eig, dim3(nb), dim3(256), 0, st, d_S, n, s_scale, eps_split, G, g_scale, eps_grad,
                     Gabs, adc_tau, w.lam, w.vmin, w.flag, budget > 0 ? w.key : nullptr);
  if (budget > 0) {
    const unsigned hb = (unsigned)std::min<int64_t>(ceil_div(n, 256), 2048);
    hipLaunchKernelGGL(k_select_init, dim3(1), dim3(256), 0, st, w.state, w.hist, budget);
    for (int pass = 0; pass < 4; ++pass) {
      hipLaunchKernelGGL(k_select_hist, dim3(hb), dim3(256), 0, st, w.flag, w.key, n, pass, w.state, w.hist);
      hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(64), 0, st, w.state, w.hist, pass);
    }
    if (exclusive_scan<LoadTies, uint32_t, uint32_t>(LoadTies{w.flag, w.key, w.state}, n, w.before, w.partials, st) !=
        hipSuccess)
      return STEEPGS_ERR_HIP;
    hipLaunchKernelGGL(k_select_apply, dim3(nb), dim3(256), 0, st, w.flag, w.key, w.before, n, w.state);
  }
  if (exclusive_scan<LoadFlags, uint32_t, uint32_t>(LoadFlags{w.flag}, n, w.before, w.partials, st) != hipSuccess)
    return STEEPGS_ERR_HIP;
  hipLaunchKernelGGL(k_densify_total, dim3(1), dim3(1), 0, st, w.partials + scan_partials_count(n), n, out_capacity,
                     d_n_out, d_status);
  if (out_capacity > 0)
    hipLaunchKernelGGL(k_densify_scatter, dim3(nb), dim3(256), 0, st, d_params, n, F, w.flag, w.before, w.vmin, 3, eps,
                       d_out, out_capacity, d_status);
  if (d_lambda_min) hipLaunchKernelGGL(k_copy_f32, dim3(nb), dim3(256), 0, st, w.lam, d_lambda_min, n);
  if (d_vmin) hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)ceil_div(3 * n, 256)), dim3(256), 0, st, w.vmin, d_vmin, 3 * n);
  if (d_split) hipLaunchKernelGGL(k_flag_u8, dim3(nb), dim3(256), 0, st, w.flag, d_split, n);
  timer_end(STEEPGS_TIMER_DENSIFY, st);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}

extern "C" steepgs_status steepgs_densify6(const float* d_params, int64_t n, int32_t sh_degree, const float* d_S6,
                                           float s_scale, float eps, float eps_split, float* d_out,
                                           int64_t out_capacity, int64_t* d_n_out, float* d_lambda_min,
                                           float* d_vmin, uint8_t* d_split, int32_t* d_status, void* d_ws,
                                           size_t ws_bytes, void* stream) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || out_capacity < 0 || !d_n_out || !d_status)
    return STEEPGS_ERR_INVALID_ARG;
  if (n >= (int64_t)1 << 31) return STEEPGS_ERR_INVALID_ARG;
  hipStream_t st = as_stream(stream);
  if (n == 0) {
    hipLaunchKernelGGL(k_densify_empty, dim3(1), dim3(1), 0, st, d_n_out, d_status);
    SG_TRY_LAUNCH();
    return STEEPGS_OK;
  }
  if (!d_params || !d_S6 || (out_capacity > 0 && !d_out)) return STEEPGS_ERR_INVALID_ARG;
  DensWs w;
  const size_t need = densify_layout(nullptr, n, w);
  if (!d_ws || ws_bytes < need) return STEEPGS_ERR_WORKSPACE;
  densify_layout(d_ws, n, w);
  const int F = STEEPGS_NUM_PARAMS(sh_degree);
  const unsigned nb = (unsigned)ceil_div(n, 256);
  timer_begin(STEEPGS_TIMER_DENSIFY, st);
  hipLaunchKernelGGL(k_densify6_eig, dim3((unsigned)ceil_div(n, 128)), dim3(128), 0, st, d_S6, n, s_scale, eps_split,
                     w.lam, w.vmin, w.flag);
  if (exclusive_scan<LoadFlags, uint32_t, uint32_t>(LoadFlags{w.flag}, n, w.before, w.partials, st) != hipSuccess)
    return STEEPGS_ERR_HIP;
  hipLaunchKernelGGL(k_densify_total, dim3(1), dim3(1), 0, st, w.partials + scan_partials_count(n), n, out_capacity,
                     d_n_out, d_status);
  if (out_capacity > 0)
    hipLaunchKernelGGL(k_densify_scatter, dim3(nb), dim3(256), 0, st, d_params, n, F, w.flag, w.before, w.vmin, 6, eps,
                       d_out, out_capacity, d_status);
  if (d_lambda_min) hipLaunchKernelGGL(k_copy_f32, dim3(nb), dim3(256), 0, st, w.lam, d_lambda_min, n);
  if (d_vmin) hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)ceil_div(6 * n, 256)), dim3(256), 0, st, w.vmin, d_vmin, 6 * n);
  if (d_split) hipLaunchKernelGGL(k_flag_u8, dim3(nb), dim3(256), 0, st, w.flag, d_split, n);
  timer_end(STEEPGS_TIMER_DENSIFY, st);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
