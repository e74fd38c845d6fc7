// Stage 4: backward of the blend and of the projection, with the splitting
// matrices of Theorem 1 accumulated on the way (Sec. 4.4).
//
// Kernel 1 (raster backward, persistent over tiles): every pixel walks its
// contributors back to front, recomputing alpha with the forward's own
// routine and the transmittance T_i = T_{i+1} / (1 - alpha_i) from the stored
// final value (no per-pixel lists are stored).  The walk starts at the last
// contributor of the workgroup (of the wavefront, per wave); the thread that
// stages an entry tests its alpha >= alpha_min box against every 8x8
// quadrant, and each wavefront walks only the entries that reach its own.
// Per contributor it forms
//   g = dL/dalpha_i = sum_c dL/dC_c (c_i T_i - R_c / (1 - alpha_i)),
// R = colour of everything behind i (background included), and the
// gradients w.r.t. the 2D mean, conic, opacity and colour.  A wavefront sums
// them over its 64 pixels with DPP row operations and issues one atomic per
// quantity.
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
  constexpr int NW = NT / 64;           // wavefronts per workgroup = 64-entry chunks per batch
  constexpr int WX = TW / 8;            // each wavefront owns an 8x8 pixel quadrant of the tile
  __shared__ float4 s_a[NT];            // mean x, mean y, conic a, conic b
  __shared__ float4 s_c[NT];            // conic c, opacity, red, green
  __shared__ float2 s_e[NT];            // blue, record id (bits)
  __shared__ uint64_t s_bits[NW][NW];   // [wave][chunk]: entries of the chunk that reach the wave's quadrant
  __shared__ uint32_t s_last[NW];
  __shared__ int s_tile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int qx = (wave % WX) * 8 + (lane & 7), qy = (wave / WX) * 8 + (lane >> 3);
  const float cut = footprint_power_cut(opt);
  for (;;) {
    // The barrier closes the previous tile before lane 0 fetches the next one,
    // so no lane-0-only region can span the loop's back edge.
    __syncthreads();
    if (tid == 0) s_tile = (int)atomicAdd(queue, 1u);
    __syncthreads();
    // scalar (wave-uniform) copy: the loop exit below must be a uniform branch
    const int tile = __builtin_amdgcn_readfirstlane(s_tile);
    if (tile >= total_tiles) break;
    const int v = view_of_tile(cams, V, tile);
    const int W = cams[v].width, H = cams[v].height, tiles_x = cams[v].tiles_x;
    const int64_t pix_off = cams[v].pixel_offset;
    const int lt = tile - cams[v].tile_offset;
    const int tx0 = (lt % tiles_x) * TW, ty0 = (lt / tiles_x) * TH;
    const int px = tx0 + qx, py = ty0 + qy;
    const bool inside = px < W && py < H;
    const uint32_t begin = ranges[2 * tile];
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
    // entries at or past a wavefront's last contributor need no work from it;
    // the workgroup walks back from the largest last contributor
    const int wlast = (int)__builtin_amdgcn_readfirstlane(wave_max_u32(last));
    if (lane == 0) s_last[wave] = (uint32_t)wlast;
    __syncthreads();
    int count = 0;
    for (int w = 0; w < NW; ++w) count = max(count, (int)s_last[w]);
    count = __builtin_amdgcn_readfirstlane(count);
    for (int b_end = count; b_end > 0; b_end -= NT) {
      const int b_start = b_end > NT ? b_end - NT : 0;
      __syncthreads();
      // stage one batch; the loading thread tests the entry's cut-off box
      // against the quadrant of every wavefront
      uint32_t qmask = 0;
      if (b_start + tid < b_end) {
        const uint32_t id = vals[begin + b_start + tid];
        const steepgs_splat s = splats[id];
        float ex, ey;
        cutoff_extent(s.conic_a, s.conic_b, s.conic_c, s.opacity, opt, ex, ey);
        s_a[tid] = make_float4(s.mean_x, s.mean_y, s.conic_a, s.conic_b);
        s_c[tid] = make_float4(s.conic_c, s.opacity, s.rgb[0], s.rgb[1]);
        s_e[tid] = make_float2(s.rgb[2], __uint_as_float(id));
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const float x0 = (float)(tx0 + (w % WX) * 8), y0 = (float)(ty0 + (w / WX) * 8);
          const bool hit = (s.mean_x + ex >= x0) && (s.mean_x - ex <= x0 + 7.f) && (s.mean_y + ey >= y0) &&
                           (s.mean_y - ey <= y0 + 7.f);
          qmask |= hit ? (1u << w) : 0u;
        }
      }
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint64_t b = ballot((qmask >> w) & 1u);
        if (lane == 0) s_bits[w][wave] = b;
      }
      __syncthreads();
      // this wavefront's entries of the batch below its last contributor, back to front
      const int jtop = min(b_end, wlast) - b_start - 1;
      for (int c = NW - 1; c >= 0; --c) {
        if (jtop < c * 64) continue;
        uint64_t bits = uniform_u64(s_bits[wave][c]);
        if (jtop - c * 64 < 63) bits &= (2ull << (jtop - c * 64)) - 1ull;
        while (bits) {
          const int hb = 63 - (int)__builtin_clzll(bits);
          bits &= ~(1ull << hb);
          const int j = c * 64 + hb;
          const float4 a = s_a[j];
          const float4 qq = s_c[j];
          const uint32_t pos = (uint32_t)(b_start + j);
          bool contrib = pos < last;  // false for pixels outside the image (last = 0)
          float gmx = 0.f, gmy = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f;
          if (contrib) {
            const float dx = fx - a.x, dy = fy - a.y;
            const float ca = a.z, cb = a.w, cc = qq.x;
            const float power = splat_power(dx, dy, ca, cb, cc);
            const float G = __expf(power);
            const float raw_a = qq.y * G;
            const bool clamped = raw_a > opt.alpha_max;
            const float alpha = clamped ? opt.alpha_max : raw_a;
            contrib = power >= cut && alpha >= opt.alpha_min;
            if (contrib) {
              const float blue = s_e[j].x;
              const float om = 1.f - alpha;
              T = T / om;  // transmittance in front of this entry
              const float w = alpha * T;
              const float inv_om = 1.f / om;
              const float g = dC0 * (qq.z * T - R0 * inv_om) + dC1 * (qq.w * T - R1 * inv_om) +
                              dC2 * (blue * T - R2 * inv_om);
              R0 += qq.z * w;
              R1 += qq.w * w;
              R2 += blue * w;
              gr = w * dC0;
              gg = w * dC1;
              gbl = w * dC2;
              if (!clamped) {
                const float gaw = g * alpha;
                gmx = gaw * (ca * dx + cb * dy);
                gmy = gaw * (cb * dx + cc * dy);
                ga = -0.5f * gaw * dx * dx;
                gb = -gaw * dx * dy;
                gc = -0.5f * gaw * dy * dy;
                go = g * G;
              }
            }
          }
          if (ballot(contrib)) {
            gmx = wave_sum_dpp(gmx);
            gmy = wave_sum_dpp(gmy);
            ga = wave_sum_dpp(ga);
            gb = wave_sum_dpp(gb);
            gc = wave_sum_dpp(gc);
            go = wave_sum_dpp(go);
            gr = wave_sum_dpp(gr);
            gg = wave_sum_dpp(gg);
            gbl = wave_sum_dpp(gbl);
            if (lane == 0) {
              const int64_t id = __float_as_uint(s_e[j].y);
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
}

// ---------------------------------------------------------------------------
// kernel 2: projection backward and the splitting-matrix lift.
// One thread per Gaussian loops over the views.  The two discrete decisions
// the forward took in fp64 are re-taken identically: the frustum-guard clamp
// (fp64 camera-space position, same operation order) and the colour clamp
// (fp32 value, re-evaluated in fp64 when within 1e-5 of zero).  The chain
// rule itself runs in fp32.

// fp64 colour of one channel, for a clamp decision too close to call in fp32
__device__ __noinline__ bool colour_clamped_fp64(const float* __restrict__ params, int64_t n, int64_t i, int deg,
                                                  const steepgs_camera& cam, int ch) {
#pragma clang fp contract(off)
  double R[9], t[3];
  for (int k = 0; k < 9; ++k) R[k] = cam.R[k];
  for (int k = 0; k < 3; ++k) t[k] = cam.t[k];
  double campos[3], d[3];
  for (int k = 0; k < 3; ++k) campos[k] = -(R[0 + k] * t[0] + R[3 + k] * t[1] + R[6 + k] * t[2]);
  for (int k = 0; k < 3; ++k) d[k] = (double)params[(STEEPGS_ROW_MEAN + k) * n + i] - campos[k];
  const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double Y[16];
  sh_eval<double>(deg, d[0] / len, d[1] / len, d[2] / len, Y);
  double acc = 0.0;
  for (int k = 0; k < (deg + 1) * (deg + 1); ++k) acc = acc + (double)params[(STEEPGS_ROW_SH + 3 * k + ch) * n + i] * Y[k];
  acc = acc + 0.5;
  return acc < 0.0;
}

template <int D>
__global__ void __launch_bounds__(128) k_proj_bwd(const float* __restrict__ params, int64_t n,
                                                  const steepgs_camera* __restrict__ cams, int V, steepgs_opts opt,
                                                  const uint32_t* __restrict__ tiles, const float* __restrict__ g2d,
                                                  float* __restrict__ grads, float* __restrict__ S) {
  constexpr int NB = (D + 1) * (D + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t m = (int64_t)V * n;
  float p[3];
  for (int k = 0; k < 3; ++k) p[k] = params[(STEEPGS_ROW_MEAN + k) * n + i];
  float sh[3 * NB];
#pragma unroll
  for (int k = 0; k < 3 * NB; ++k) sh[k] = params[(STEEPGS_ROW_SH + k) * n + i];
  // covariance R diag(s^2) R^T (fp32), opacity
  float q[4];
  for (int k = 0; k < 4; ++k) q[k] = params[(STEEPGS_ROW_QUAT + k) * n + i];
  const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  const float Rq[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                          {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                          {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  float sc[3];
  for (int k = 0; k < 3; ++k) sc[k] = expf(params[(STEEPGS_ROW_LOG_SCALE + k) * n + i]);
  float Sig[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Sig[a][b] = Rq[a][0] * sc[0] * sc[0] * Rq[b][0] + Rq[a][1] * sc[1] * sc[1] * Rq[b][1] +
                  Rq[a][2] * sc[2] * sc[2] * Rq[b][2];
  const float o = 1.f / (1.f + expf(-params[STEEPGS_ROW_OPACITY * n + i]));

  float dp[3] = {0.f, 0.f, 0.f}, dSig[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, dop = 0.f;
  float S3[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float dsh[3 * NB];
#pragma unroll
  for (int k = 0; k < 3 * NB; ++k) dsh[k] = 0.f;
  bool any = false;
  for (int v = 0; v < V; ++v) {
    const int64_t r = (int64_t)v * n + i;
    if (tiles[r] == 0) continue;
    float G9[9];
    bool nz = false;
    for (int k = 0; k < 9; ++k) {
      G9[k] = g2d[k * m + r];
      nz |= G9[k] != 0.f;
    }
    if (!nz) continue;
    any = true;
    const steepgs_camera& cam = cams[v];
    float W[9];
    for (int k = 0; k < 9; ++k) W[k] = cam.R[k];
    const float fx = cam.fx, fy = cam.fy;
    const float gmx = G9[0], gmy = G9[1], ga = G9[2], gb = G9[3], gc = G9[4], go = G9[5];

    // camera-space position: fp64 in the forward's operation order for the guard decision
    double pcd[3];
    {
#pragma clang fp contract(off)
      for (int k = 0; k < 3; ++k)
        pcd[k] = (double)cam.R[3 * k + 0] * (double)p[0] + (double)cam.R[3 * k + 1] * (double)p[1] +
                 (double)cam.R[3 * k + 2] * (double)p[2] + (double)cam.t[k];
    }
    const float pcx = (float)pcd[0], pcy = (float)pcd[1], pcz = (float)pcd[2];
    float J[2][3];
    float gx = 0.f, gy = 0.f;
    bool gx_free = false, gy_free = false;
    if (cam.model == 0) {
      double gxd = pcd[0] / pcd[2], gyd = pcd[1] / pcd[2];
      gx_free = gy_free = true;
      if (opt.frustum_guard > 0.f) {
        const double limx = (double)opt.frustum_guard * (0.5 * cam.width / (double)cam.fx);
        const double limy = (double)opt.frustum_guard * (0.5 * cam.height / (double)cam.fy);
        if (gxd < -limx) { gxd = -limx; gx_free = false; }
        if (gxd > limx) { gxd = limx; gx_free = false; }
        if (gyd < -limy) { gyd = -limy; gy_free = false; }
        if (gyd > limy) { gyd = limy; gy_free = false; }
      }
      gx = (float)gxd;
      gy = (float)gyd;
      const float iz = 1.f / pcz;
      J[0][0] = fx * iz; J[0][1] = 0.f; J[0][2] = -fx * gx * iz;
      J[1][0] = 0.f; J[1][1] = fy * iz; J[1][2] = -fy * gy * iz;
    } else {
      J[0][0] = fx; J[0][1] = 0.f; J[0][2] = 0.f;
      J[1][0] = 0.f; J[1][1] = fy; J[1][2] = 0.f;
    }
    float P[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) P[a][c] = J[a][0] * W[c] + J[a][1] * W[3 + c] + J[a][2] * W[6 + c];
    // Pi(Sigma) and its inverse (the conic)
    float PS[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) PS[a][c] = P[a][0] * Sig[0][c] + P[a][1] * Sig[1][c] + P[a][2] * Sig[2][c];
    const float s00 = PS[0][0] * P[0][0] + PS[0][1] * P[0][1] + PS[0][2] * P[0][2] + opt.dilation;
    const float s01 = PS[0][0] * P[1][0] + PS[0][1] * P[1][1] + PS[0][2] * P[1][2];
    const float s11 = PS[1][0] * P[1][0] + PS[1][1] * P[1][1] + PS[1][2] * P[1][2] + opt.dilation;
    const float idet = 1.f / (s00 * s11 - s01 * s01);
    const float A[2][2] = {{s11 * idet, -s01 * idet}, {-s01 * idet, s00 * idet}};

    // colour: rgb = max(0, sum_k sh_k Y_k(dir) + 1/2)
    float campos[3];
    for (int k = 0; k < 3; ++k) campos[k] = -(W[0 + k] * cam.t[0] + W[3 + k] * cam.t[1] + W[6 + k] * cam.t[2]);
    float dv[3] = {p[0] - campos[0], p[1] - campos[1], p[2] - campos[2]};
    const float dlen = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const float idl = 1.f / dlen;
    const float dir[3] = {dv[0] * idl, dv[1] * idl, dv[2] * idl};
    float Y[NB];
    sh_eval<float>(D, dir[0], dir[1], dir[2], Y);
    float dcol[3];
    for (int ch = 0; ch < 3; ++ch) {
      float raw = 0.5f;
#pragma unroll
      for (int k = 0; k < NB; ++k) raw += sh[3 * k + ch] * Y[k];
      bool clamped = raw < 0.f;
      if (fabsf(raw) < 1e-5f) clamped = colour_clamped_fp64(params, n, i, D, cam, ch);
      dcol[ch] = clamped ? 0.f : G9[6 + ch];
    }
    float dY[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      dY[k] = sh[3 * k] * dcol[0] + sh[3 * k + 1] * dcol[1] + sh[3 * k + 2] * dcol[2];
      dsh[3 * k] += Y[k] * dcol[0];
      dsh[3 * k + 1] += Y[k] * dcol[1];
      dsh[3 * k + 2] += Y[k] * dcol[2];
    }
    if (D > 0) {
      float gd[3] = {0.f, 0.f, 0.f};
      sh_grad<float>(D, dir[0], dir[1], dir[2], dY, gd);
      const float dot = gd[0] * dir[0] + gd[1] * dir[1] + gd[2] * dir[2];
      for (int k = 0; k < 3; ++k) dp[k] += (gd[k] - dir[k] * dot) * idl;
    }

    // conic -> Pi(Sigma): dL/dS2 = -A G_A A, G_A = [[ga, gb/2], [gb/2, gc]]
    const float GA[2][2] = {{ga, 0.5f * gb}, {0.5f * gb, gc}};
    float AG[2][2], GS2[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) AG[a][b] = A[a][0] * GA[0][b] + A[a][1] * GA[1][b];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) GS2[a][b] = -(AG[a][0] * A[0][b] + AG[a][1] * A[1][b]);
    // Pi(Sigma) = P Sigma P^T + dilation: dL/dSigma += P^T GS2 P; dL/dP = 2 GS2 P Sigma
    float GSP[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) GSP[a][c] = GS2[a][0] * P[0][c] + GS2[a][1] * P[1][c];
    const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int c = ij[k][0], d = ij[k][1];
      dSig[k] += P[0][c] * GSP[0][d] + P[1][c] * GSP[1][d];
    }
    float GJ[2][3];
    for (int a = 0; a < 2; ++a) {
      float GP[3];
      for (int c = 0; c < 3; ++c)
        GP[c] = 2.f * (GSP[a][0] * Sig[0][c] + GSP[a][1] * Sig[1][c] + GSP[a][2] * Sig[2][c]);
      // P = J W: dL/dJ = dL/dP W^T
      for (int b = 0; b < 3; ++b) GJ[a][b] = GP[0] * W[3 * b + 0] + GP[1] * W[3 * b + 1] + GP[2] * W[3 * b + 2];
    }
    // camera-space position gradient from the mean and from J
    float dpc[3] = {0.f, 0.f, 0.f};
    float Pe[2][3];  // Jacobian of the projected mean w.r.t. p (exact, unguarded)
    if (cam.model == 0) {
      const float iz = 1.f / pcz, iz2 = iz * iz;
      dpc[0] += gmx * fx * iz;
      dpc[1] += gmy * fy * iz;
      dpc[2] -= (gmx * fx * pcx + gmy * fy * pcy) * iz2;
      dpc[2] -= (GJ[0][0] * fx + GJ[1][1] * fy) * iz2;
      // J02 = -fx gx / z, J12 = -fy gy / z with gx = x/z unless clamped
      dpc[2] += (GJ[0][2] * fx * gx + GJ[1][2] * fy * gy) * iz2;
      if (gx_free) {
        dpc[0] -= GJ[0][2] * fx * iz2;
        dpc[2] += GJ[0][2] * fx * pcx * iz2 * iz;
      }
      if (gy_free) {
        dpc[1] -= GJ[1][2] * fy * iz2;
        dpc[2] += GJ[1][2] * fy * pcy * iz2 * iz;
      }
      const float Je[2][3] = {{fx * iz, 0.f, -fx * pcx * iz2}, {0.f, fy * iz, -fy * pcy * iz2}};
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) Pe[a][c] = Je[a][0] * W[c] + Je[a][2] * W[6 + c] + Je[a][1] * W[3 + c];
    } else {
      dpc[0] += gmx * fx;
      dpc[1] += gmy * fy;
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) Pe[a][c] = P[a][c];
    }
    for (int c = 0; c < 3; ++c) dp[c] += W[c] * dpc[0] + W[3 + c] * dpc[1] + W[6 + c] * dpc[2];
    dop += go;

    // splitting matrix: S2D = A M A - m0 A, M = [[-2ga, -gb], [-gb, -2gc]], m0 = o * go
    const float M[2][2] = {{-2.f * ga, -gb}, {-gb, -2.f * gc}};
    float AM[2][2], S2D[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) AM[a][b] = A[a][0] * M[0][b] + A[a][1] * M[1][b];
    const float m0 = o * go;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) S2D[a][b] = AM[a][0] * A[0][b] + AM[a][1] * A[1][b] - m0 * A[a][b];
    float SP[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) SP[a][c] = S2D[a][0] * Pe[0][c] + S2D[a][1] * Pe[1][c];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = ij[k][0], b = ij[k][1];
      S3[k] += Pe[0][a] * SP[0][b] + Pe[1][a] * SP[1][b];
    }
  }
  if (!any) return;

  // Sigma = M M^T, M = R diag(s): dL/dM = 2 dSig M (dSig symmetric)
  const float G[3][3] = {{dSig[0], dSig[1], dSig[2]}, {dSig[1], dSig[3], dSig[4]}, {dSig[2], dSig[4], dSig[5]}};
  float GR[3][3], dls[3];
  for (int k = 0; k < 3; ++k) {
    float acc = 0.f;
    for (int a = 0; a < 3; ++a) {
      const float gm = 2.f * (G[a][0] * Rq[0][k] + G[a][1] * Rq[1][k] + G[a][2] * Rq[2][k]) * sc[k];
      acc += gm * Rq[a][k];
      GR[a][k] = gm * sc[k];
    }
    dls[k] = acc * sc[k];
  }
  float dq[4];
  dq[0] = 2.f * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
  dq[1] = 2.f * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2.f * x * GR[1][1] - w * GR[1][2] + z * GR[2][0] +
                 w * GR[2][1] - 2.f * x * GR[2][2]);
  dq[2] = 2.f * (-2.f * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + z * GR[1][2] - w * GR[2][0] +
                 z * GR[2][1] - 2.f * y * GR[2][2]);
  dq[3] = 2.f * (-2.f * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - 2.f * z * GR[1][1] +
                 y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
  // through the normalisation q_hat = q / |q|
  const float qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  const float qh[4] = {w, x, y, z};
  float* gp = grads + i;
  for (int k = 0; k < 3; ++k) gp[(STEEPGS_ROW_MEAN + k) * n] += dp[k];
  for (int k = 0; k < 3; ++k) gp[(STEEPGS_ROW_LOG_SCALE + k) * n] += dls[k];
  for (int k = 0; k < 4; ++k) gp[(STEEPGS_ROW_QUAT + k) * n] += (dq[k] - qh[k] * qd) / qn;
  gp[STEEPGS_ROW_OPACITY * n] += dop * o * (1.f - o);
#pragma unroll
  for (int k = 0; k < 3 * NB; ++k) gp[(STEEPGS_ROW_SH + k) * n] += dsh[k];
  for (int k = 0; k < 6; ++k) S[k * n + i] += S3[k];
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
  const dim3 pg((unsigned)ceil_div(n, 128));
  switch (sh_degree) {
    case 0: hipLaunchKernelGGL(k_proj_bwd<0>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, g2d, d_grads, d_S); break;
    case 1: hipLaunchKernelGGL(k_proj_bwd<1>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, g2d, d_grads, d_S); break;
    case 2: hipLaunchKernelGGL(k_proj_bwd<2>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, g2d, d_grads, d_S); break;
    default: hipLaunchKernelGGL(k_proj_bwd<3>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, g2d, d_grads, d_S); break;
  }
  timer_end(STEEPGS_TIMER_PROJ_BWD, st);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
