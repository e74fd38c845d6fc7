// Stage 4: backward of the blend and of the projection, with the splitting
// matrices of Theorem 1 accumulated on the way (Sec. 4.4).
//
// Kernel 1 (raster backward, persistent over tiles): every pixel walks its
// contributors back to front, recomputing alpha with the forward's own
// routine and the transmittance T_i = T_{i+1} / (1 - alpha_i) from the stored
// final value (no per-pixel lists are stored).  Per contributor it forms
//   g = dL/dalpha_i = sum_c dL/dC_c (c_i T_i - R_c / (1 - alpha_i)),
// R = colour of everything behind i (background included), and the
// gradients w.r.t. the 2D mean, conic, opacity and colour.  A wavefront sums
// them over its 64 pixels and issues one atomic per quantity.
//
// Kernel 2 (one thread per Gaussian, all views): chain rule from the 2D
// quantities to the 3D parameters, and the splitting matrix.  With
// g(x) = dL/dalpha_i(x), the per-view sum
//   sum_x g alpha (A d d^T A - A) = A M A - m0 A,
//   M = sum_x g alpha d d^T = -2 dL/dA,  m0 = sum_x g alpha = o dL/do,
// so the 2x2 matrix comes from the conic and opacity gradients the raster
// backward already produced: S_i += P^T (A M A - m0 A) P at no per-pixel cost
// (P = Jacobian of the projected mean w.r.t. p, App. C.4).
#include "projection.h"

namespace sg {

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) k_render_bwd(const steepgs_splat* __restrict__ splats,
                                                      const uint32_t* __restrict__ vals,
                                                      const uint32_t* __restrict__ ranges,
                                                      const steepgs_camera* __restrict__ cams, int V,
                                                      steepgs_opts opt, int total_tiles,
                                                      const float* __restrict__ image,
                                                      const float* __restrict__ T_final,
                                                      const uint32_t* __restrict__ n_contrib,
                                                      const float* __restrict__ dL_dimage,
                                                      const float* __restrict__ target, float* __restrict__ g2d,
                                                      int64_t m, uint32_t* __restrict__ queue) {
  constexpr int NT = TW * TH;
  __shared__ float s_mx[NT], s_my[NT], s_a[NT], s_b[NT], s_c[NT], s_o[NT], s_r[NT], s_g[NT], s_bl[NT];
  __shared__ uint32_t s_id[NT];
  __shared__ int s_tile;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (;;) {
    // The barrier closes the previous tile before lane 0 fetches the next one,
    // so no lane-0-only region can span the loop's back edge (the compiler
    // would otherwise merge them and let the other lanes re-enter the tile
    // loop without the fetch).
    __syncthreads();
    if (tid == 0) s_tile = (int)atomicAdd(queue, 1u);
    __syncthreads();
    // scalar (wave-uniform) copy: the loop exit below must be a uniform branch,
    // or the compiler may move the queue atomic out of the per-tile loop
    const int tile = __builtin_amdgcn_readfirstlane(s_tile);
    __syncthreads();
    if (tile >= total_tiles) break;
    const int v = view_of_tile(cams, V, tile);
    const int W = cams[v].width, H = cams[v].height, tiles_x = cams[v].tiles_x;
    const int64_t pix_off = cams[v].pixel_offset;
    const int lt = tile - cams[v].tile_offset;
    const int px = (lt % tiles_x) * TW + tid % TW;
    const int py = (lt / tiles_x) * TH + tid / TW;
    const bool inside = px < W && py < H;
    const uint32_t begin = ranges[2 * tile], end = ranges[2 * tile + 1];
    const float fx = (float)px, fy = (float)py;
    float T = 1.f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f, R0 = 0.f, R1 = 0.f, R2 = 0.f;
    uint32_t last = 0;
    if (inside) {
      const int64_t p = pix_off + (int64_t)py * W + px;
      const int64_t plane = (int64_t)W * H;
      const int64_t q = 3 * pix_off + (int64_t)py * W + px;
      T = T_final[p];
      last = n_contrib[p];
      if (dL_dimage) {
        dC0 = dL_dimage[q];
        dC1 = dL_dimage[q + plane];
        dC2 = dL_dimage[q + 2 * plane];
      } else {
        const float inv = 1.f / (3.f * (float)W * (float)H);
        const float e0 = image[q] - target[q], e1 = image[q + plane] - target[q + plane];
        const float e2 = image[q + 2 * plane] - target[q + 2 * plane];
        dC0 = (e0 > 0.f) ? inv : ((e0 < 0.f) ? -inv : 0.f);
        dC1 = (e1 > 0.f) ? inv : ((e1 < 0.f) ? -inv : 0.f);
        dC2 = (e2 > 0.f) ? inv : ((e2 < 0.f) ? -inv : 0.f);
      }
      R0 = T * opt.bg[0];
      R1 = T * opt.bg[1];
      R2 = T * opt.bg[2];
    }
    const int count = (int)(end - begin);
    for (int b_end = count; b_end > 0; b_end -= NT) {
      const int b_start = b_end > NT ? b_end - NT : 0;
      __syncthreads();
      if (b_start + tid < b_end) {
        const uint32_t id = vals[begin + b_start + tid];
        const steepgs_splat s = splats[id];
        s_id[tid] = id;
        s_mx[tid] = s.mean_x;
        s_my[tid] = s.mean_y;
        s_a[tid] = s.conic_a;
        s_b[tid] = s.conic_b;
        s_c[tid] = s.conic_c;
        s_o[tid] = s.opacity;
        s_r[tid] = s.rgb[0];
        s_g[tid] = s.rgb[1];
        s_bl[tid] = s.rgb[2];
      }
      __syncthreads();
      for (int j = b_end - b_start - 1; j >= 0; --j) {
        const uint32_t pos = (uint32_t)(b_start + j);
        bool contrib = pos < last;  // false for pixels outside the image (last = 0)
        float gmx = 0.f, gmy = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f;
        if (contrib) {
          const float dx = fx - s_mx[j], dy = fy - s_my[j];
          const float a = s_a[j], b = s_b[j], c = s_c[j];
          const float G = __expf(splat_power(dx, dy, a, b, c));
          const float raw = s_o[j] * G;
          const bool clamped = raw > opt.alpha_max;
          const float alpha = clamped ? opt.alpha_max : raw;
          contrib = alpha >= opt.alpha_min;
          if (contrib) {
            const float om = 1.f - alpha;
            T = T / om;  // transmittance in front of this entry
            const float w = alpha * T;
            const float inv_om = 1.f / om;
            const float g = dC0 * (s_r[j] * T - R0 * inv_om) + dC1 * (s_g[j] * T - R1 * inv_om) +
                            dC2 * (s_bl[j] * T - R2 * inv_om);
            R0 += s_r[j] * w;
            R1 += s_g[j] * w;
            R2 += s_bl[j] * w;
            gr = w * dC0;
            gg = w * dC1;
            gbl = w * dC2;
            if (!clamped) {
              const float gaw = g * alpha;
              gmx = gaw * (a * dx + b * dy);
              gmy = gaw * (b * dx + c * dy);
              ga = -0.5f * gaw * dx * dx;
              gb = -gaw * dx * dy;
              gc = -0.5f * gaw * dy * dy;
              go = g * G;
            }
          }
        }
        if (ballot(contrib)) {
          gmx = wave_sum(gmx);
          gmy = wave_sum(gmy);
          ga = wave_sum(ga);
          gb = wave_sum(gb);
          gc = wave_sum(gc);
          go = wave_sum(go);
          gr = wave_sum(gr);
          gg = wave_sum(gg);
          gbl = wave_sum(gbl);
          if (lane == 0) {
            const int64_t id = s_id[j];
            unsafeAtomicAdd(&g2d[0 * m + id], gmx);
            unsafeAtomicAdd(&g2d[1 * m + id], gmy);
            unsafeAtomicAdd(&g2d[2 * m + id], ga);
            unsafeAtomicAdd(&g2d[3 * m + id], gb);
            unsafeAtomicAdd(&g2d[4 * m + id], gc);
            unsafeAtomicAdd(&g2d[5 * m + id], go);
            unsafeAtomicAdd(&g2d[6 * m + id], gr);
            unsafeAtomicAdd(&g2d[7 * m + id], gg);
            unsafeAtomicAdd(&g2d[8 * m + id], gbl);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// kernel 2: projection backward and the splitting-matrix lift

__global__ void __launch_bounds__(128) k_proj_bwd(const float* __restrict__ params, int64_t n, int deg,
                                                  const steepgs_camera* __restrict__ cams, int V, steepgs_opts opt,
                                                  const uint32_t* __restrict__ tiles, const float* __restrict__ g2d,
                                                  float* __restrict__ grads, float* __restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t m = (int64_t)V * n;
  const int nb = (deg + 1) * (deg + 1);
  Gauss g;
  load_gauss(params, n, i, g);
  double dp[3] = {0, 0, 0}, dSig[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, dop = 0.0;
  double S3[6] = {0, 0, 0, 0, 0, 0};
  float dsh[48];
  for (int k = 0; k < 3 * nb; ++k) dsh[k] = 0.f;
  bool any = false;
  for (int v = 0; v < V; ++v) {
    const int64_t r = (int64_t)v * n + i;
    if (tiles[r] == 0) continue;
    double G9[9];
    bool nz = false;
    for (int q = 0; q < 9; ++q) {
      G9[q] = g2d[q * m + r];
      nz |= G9[q] != 0.0;
    }
    if (!nz) continue;
    CamD cam;
    load_cam(cams[v], cam);
    ViewProj pv;
    if (!project_view(g, params, n, i, deg, cam, opt, pv, true)) continue;
    any = true;
    const double gmx = G9[0], gmy = G9[1], ga = G9[2], gb = G9[3], gc = G9[4], go = G9[5];

    // colour: rgb = max(0, sum_k sh_k Y_k(dir) + 1/2)
    double dcol[3];
    for (int ch = 0; ch < 3; ++ch) dcol[ch] = pv.raw[ch] < 0.0 ? 0.0 : G9[6 + ch];
    double dY[16];
    for (int k = 0; k < nb; ++k) {
      double s = 0.0;
      for (int ch = 0; ch < 3; ++ch) {
        dsh[3 * k + ch] += (float)(pv.Y[k] * dcol[ch]);
        s += (double)params[(STEEPGS_ROW_SH + 3 * k + ch) * n + i] * dcol[ch];
      }
      dY[k] = s;
    }
    if (deg > 0) {
      double gd[3] = {0, 0, 0};
      sh_grad(deg, pv.dir[0], pv.dir[1], pv.dir[2], dY, gd);
      const double dot = gd[0] * pv.dir[0] + gd[1] * pv.dir[1] + gd[2] * pv.dir[2];
      for (int k = 0; k < 3; ++k) dp[k] += (gd[k] - pv.dir[k] * dot) / pv.dlen;
    }

    // conic -> Pi(Sigma): dL/dS2 = -A G_A A with G_A = [[ga, gb/2], [gb/2, gc]]
    const double A[2][2] = {{pv.A00, pv.A01}, {pv.A01, pv.A11}};
    const double GA[2][2] = {{ga, 0.5 * gb}, {0.5 * gb, gc}};
    double AG[2][2], GS2[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) AG[a][b] = A[a][0] * GA[0][b] + A[a][1] * GA[1][b];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) GS2[a][b] = -(AG[a][0] * A[0][b] + AG[a][1] * A[1][b]);
    // Pi(Sigma) = P Sigma P^T (+dilation): dL/dSigma += P^T GS2 P, dL/dP = 2 GS2 P Sigma
    double GSP[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) GSP[a][c] = GS2[a][0] * pv.P[0][c] + GS2[a][1] * pv.P[1][c];
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) dSig[c][d] += pv.P[0][c] * GSP[0][d] + pv.P[1][c] * GSP[1][d];
    double GP[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c)
        GP[a][c] = 2.0 * (GSP[a][0] * g.Sig[0][c] + GSP[a][1] * g.Sig[1][c] + GSP[a][2] * g.Sig[2][c]);
    // P = J W: dL/dJ = dL/dP W^T
    double GJ[2][3];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b)
        GJ[a][b] = GP[a][0] * cam.R[3 * b + 0] + GP[a][1] * cam.R[3 * b + 1] + GP[a][2] * cam.R[3 * b + 2];
    // camera-space position gradient from the mean and from J
    double dpc[3] = {0, 0, 0};
    const double x = pv.pc[0], y = pv.pc[1], z = pv.pc[2];
    double Pe[2][3];  // Jacobian of the projected mean w.r.t. p (exact, unguarded)
    if (cam.model == 0) {
      const double iz = 1.0 / z, iz2 = iz * iz;
      dpc[0] += gmx * cam.fx * iz;
      dpc[1] += gmy * cam.fy * iz;
      dpc[2] -= (gmx * cam.fx * x + gmy * cam.fy * y) * iz2;
      dpc[2] -= (GJ[0][0] * cam.fx + GJ[1][1] * cam.fy) * iz2;
      // J02 = -fx gx / z, J12 = -fy gy / z, gx = x/z unless clamped
      dpc[2] += GJ[0][2] * cam.fx * pv.gx * iz2 + GJ[1][2] * cam.fy * pv.gy * iz2;
      if (pv.gx_free) {
        dpc[0] -= GJ[0][2] * cam.fx * iz2;
        dpc[2] += GJ[0][2] * cam.fx * x * iz2 * iz;
      }
      if (pv.gy_free) {
        dpc[1] -= GJ[1][2] * cam.fy * iz2;
        dpc[2] += GJ[1][2] * cam.fy * y * iz2 * iz;
      }
      const double Je[2][3] = {{cam.fx * iz, 0.0, -cam.fx * x * iz2}, {0.0, cam.fy * iz, -cam.fy * y * iz2}};
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) Pe[a][c] = Je[a][0] * cam.R[c] + Je[a][1] * cam.R[3 + c] + Je[a][2] * cam.R[6 + c];
    } else {
      dpc[0] += gmx * cam.fx;
      dpc[1] += gmy * cam.fy;
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) Pe[a][c] = pv.P[a][c];
    }
    for (int c = 0; c < 3; ++c) dp[c] += cam.R[c] * dpc[0] + cam.R[3 + c] * dpc[1] + cam.R[6 + c] * dpc[2];
    dop += go;

    // splitting matrix: S2D = A M A - m0 A, M = [[-2ga, -gb], [-gb, -2gc]], m0 = o * go
    const double M[2][2] = {{-2.0 * ga, -gb}, {-gb, -2.0 * gc}};
    double AM[2][2], S2D[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) AM[a][b] = A[a][0] * M[0][b] + A[a][1] * M[1][b];
    const double m0 = g.o * go;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) S2D[a][b] = AM[a][0] * A[0][b] + AM[a][1] * A[1][b] - m0 * A[a][b];
    double SP[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) SP[a][c] = S2D[a][0] * Pe[0][c] + S2D[a][1] * Pe[1][c];
    const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int k = 0; k < 6; ++k) {
      const int a = ij[k][0], b = ij[k][1];
      S3[k] += Pe[0][a] * SP[0][b] + Pe[1][a] * SP[1][b];
    }
  }
  if (!any) return;

  // Sigma = M M^T, M = R diag(s): dL/dM = 2 dSig M
  double GM[3][3];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k)
      GM[a][k] = 2.0 * (dSig[a][0] * g.R[0][k] + dSig[a][1] * g.R[1][k] + dSig[a][2] * g.R[2][k]) * g.s[k];
  double dls[3], GR[3][3];
  for (int k = 0; k < 3; ++k) {
    dls[k] = (GM[0][k] * g.R[0][k] + GM[1][k] * g.R[1][k] + GM[2][k] * g.R[2][k]) * g.s[k];
    for (int a = 0; a < 3; ++a) GR[a][k] = GM[a][k] * g.s[k];
  }
  const double w = g.qw, x = g.qx, y = g.qy, z = g.qz;
  double dq[4];
  dq[0] = 2.0 * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
  dq[1] = 2.0 * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2.0 * x * GR[1][1] - w * GR[1][2] + z * GR[2][0] +
                 w * GR[2][1] - 2.0 * x * GR[2][2]);
  dq[2] = 2.0 * (-2.0 * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + z * GR[1][2] - w * GR[2][0] +
                 z * GR[2][1] - 2.0 * y * GR[2][2]);
  dq[3] = 2.0 * (-2.0 * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - 2.0 * z * GR[1][1] +
                 y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
  // through the normalisation q_hat = q / |q|
  const double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  const double qh[4] = {w, x, y, z};
  for (int k = 0; k < 4; ++k) dq[k] = (dq[k] - qh[k] * qd) / g.qn;

  float* gp = grads + i;
  for (int k = 0; k < 3; ++k) gp[(STEEPGS_ROW_MEAN + k) * n] += (float)dp[k];
  for (int k = 0; k < 3; ++k) gp[(STEEPGS_ROW_LOG_SCALE + k) * n] += (float)dls[k];
  for (int k = 0; k < 4; ++k) gp[(STEEPGS_ROW_QUAT + k) * n] += (float)dq[k];
  gp[STEEPGS_ROW_OPACITY * n] += (float)(dop * g.o * (1.0 - g.o));
  for (int k = 0; k < 3 * nb; ++k) gp[(STEEPGS_ROW_SH + k) * n] += dsh[k];
  for (int k = 0; k < 6; ++k) S[k * n + i] += (float)S3[k];
}

__global__ void k_zero(float* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

static size_t bwd_layout(void* base, int64_t m, float** g2d, uint32_t** queue) {
  Carver c(base);
  *queue = c.take<uint32_t>(64);
  *g2d = c.take<float>((size_t)9 * m);
  return c.used + 256;
}

size_t render_bwd_workspace(int64_t m) {
  float* g;
  uint32_t* q;
  return bwd_layout(nullptr, m, &g, &q);
}

template <int TW, int TH>
static void launch_bwd(int grid, hipStream_t st, const steepgs_splat* splats, const uint32_t* vals,
                       const uint32_t* ranges, const steepgs_camera* cams, int V, const steepgs_opts& opt,
                       int total_tiles, const float* image, const float* T_final, const uint32_t* n_contrib,
                       const float* dL_dimage, const float* target, float* g2d, int64_t m, uint32_t* queue) {
  hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3(grid), dim3(TW * TH), 0, st, splats, vals, ranges, cams, V, opt,
                     total_tiles, image, T_final, n_contrib, dL_dimage, target, g2d, m, queue);
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_render_bwd_split(const float* d_params, int64_t n, int32_t sh_degree,
                                                   const steepgs_camera* d_cams, int32_t V, const steepgs_opts* opts,
                                                   const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                                                   const uint32_t* d_vals, const uint32_t* d_tile_ranges,
                                                   int32_t total_tiles, int64_t total_pixels, const float* d_image,
                                                   const float* d_T_final, const uint32_t* d_n_contrib,
                                                   const float* d_dL_dimage, const float* d_target, float* d_grads,
                                                   float* d_S, float* d_grad2d, void* d_ws, size_t ws_bytes,
                                                   void* stream) {
  if (n < 0 || V <= 0 || sh_degree < 0 || sh_degree > 3 || total_tiles <= 0 || total_pixels <= 0 || !opts_ok(opts))
    return STEEPGS_ERR_INVALID_ARG;
  if (!d_cams || !d_tile_ranges || !d_T_final || !d_n_contrib || !d_grads || !d_S) return STEEPGS_ERR_INVALID_ARG;
  if (!d_dL_dimage && (!d_target || !d_image)) return STEEPGS_ERR_INVALID_ARG;
  if (n == 0) return STEEPGS_OK;
  if (!d_params || !d_splats || !d_tiles_touched) return STEEPGS_ERR_INVALID_ARG;
  const int64_t m = (int64_t)V * n;
  float* g2d;
  uint32_t* queue;
  const size_t need = bwd_layout(nullptr, m, &g2d, &queue);
  if (!d_ws || ws_bytes < need) return STEEPGS_ERR_WORKSPACE;
  bwd_layout(d_ws, m, &g2d, &queue);
  if (d_grad2d) g2d = d_grad2d;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, reinterpret_cast<float*>(queue), (int64_t)1);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>(ceil_div(9 * m, 256), 65536)), dim3(256), 0, st, g2d,
                     9 * m);
  const int grid = (int)std::min<int64_t>(total_tiles, (int64_t)device_cu_count() * 8);
  const steepgs_opts& o = *opts;
  timer_begin(STEEPGS_TIMER_RENDER_BWD, st);
  if (o.tile_w == 16 && o.tile_h == 16)
    launch_bwd<16, 16>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_image, d_T_final,
                       d_n_contrib, d_dL_dimage, d_target, g2d, m, queue);
  else if (o.tile_w == 16 && o.tile_h == 8)
    launch_bwd<16, 8>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_image, d_T_final,
                      d_n_contrib, d_dL_dimage, d_target, g2d, m, queue);
  else
    launch_bwd<8, 8>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_image, d_T_final,
                     d_n_contrib, d_dL_dimage, d_target, g2d, m, queue);
  timer_end(STEEPGS_TIMER_RENDER_BWD, st);
  timer_begin(STEEPGS_TIMER_PROJ_BWD, st);
  hipLaunchKernelGGL(k_proj_bwd, dim3((unsigned)ceil_div(n, 128)), dim3(128), 0, st, d_params, n, sh_degree, d_cams, V,
                     o, d_tiles_touched, g2d, d_grads, d_S);
  timer_end(STEEPGS_TIMER_PROJ_BWD, st);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
