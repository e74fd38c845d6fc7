// Stage 4: backward of the blend and of the projection, with the splitting
// matrices of Theorem 1 accumulated on the way (Sec. 4.4).
//
// Kernel 1 (raster backward, persistent over tiles, one wavefront per tile):
// each lane owns one pixel in every 8x8 quadrant of the tile; every pixel
// walks its contributors back to front, recomputing alpha with the forward's
// own routine and the transmittance T_i = T_{i+1} / (1 - alpha_i) from the
// stored final value (no per-pixel lists are stored).  The walk starts at the
// tile's last contributor; the lane that stages an entry tests its
// alpha >= alpha_min region (bounding box, then the ellipse) against every
// quadrant, and a quadrant whose pixels
// the entry cannot reach (or whose last contributor lies before it) is
// skipped for the whole wave.  Per contributor it forms
//   g = dL/dalpha_i = sum_c dL/dC_c (c_i T_i - R_c / (1 - alpha_i)),
// R = colour of everything behind i (background included; a pixel carries
// only the scalar dL/dC . R), and accumulates the opacity and colour
// gradients and the moments m1 = sum g alpha d, m2 = sum g alpha d d^T
// (d = pixel - mean, unclamped pixels): the 2D mean and conic gradients are
// linear in them, dL/dmean = A m1 and dL/d(a, b, c) = -(m2_xx / 2, m2_xy,
// m2_yy / 2).  A lane adds up its pixels' contributions, the wavefront sums
// them over its lanes with DPP row operations and issues one atomic per
// quantity and entry for the whole tile.
//
// Kernel 2 (one thread per Gaussian, all views): chain rule from the 2D
// quantities to the 3D parameters, and the splitting matrix.  With
// g(x) = dL/dalpha_i(x), the per-view sum
//   sum_x g alpha (A d d^T A - A) = A M A - m0 A,
//   M = sum_x g alpha d d^T = m2,  m0 = sum_x g alpha = o dL/do,
// so the 2x2 matrix comes from the conic and opacity gradients the raster
// backward already produced: S_i += P^T (A M A - m0 A) P at no per-pixel cost
// (P = Jacobian of the projected mean w.r.t. p, App. C.4).
#include "projection.h"

namespace sg {

// The backward's per-record accumulators (fp64 sums of the per-tile float32
// partials): slot [m][9] = (m1_l, m1_s, m2_ll, m2_ls, m2_ss, m0, dL/dr,
// dL/dg, dL/db) -- the first moments and second moments of g alpha d in the
// frame of the footprint's axis (l along it, s across), m0 = sum g alpha
// = o dL/do over the unclamped pixels -- one 72-byte block per record so that the nine atomics of a
// (tile, entry) touch one or two cache lines (planar geometry and colour
// arrays were measured 0.1 ms slower in the raster backward on the 16-view
// workload).  With the splitting matrix over theta = (p, log-scales) a
// second array h6 [m][9] holds the third and fourth moments in the same
// frame (m3_lll, m3_lls, m3_lss, m3_sss, m4_llll, m4_llls, m4_llss, m4_lsss,
// m4_ssss).
struct Slots {
  double* slot;
  double* h6;
};
constexpr int kSlot = 9, kH6 = 9;
// floats per record of the caller's optional 2D-gradient output
constexpr int kGrad2dOut = 12;

// H6: also the moments the dim-6 splitting matrix needs (third and fourth
// order in d), summed like the others; WAVES wavefronts per workgroup, each
// on a tile of its own
// Occupancy target of the blend kernel without the split6 moments
// (wavefronts per SIMD; a build option, it sets the register budget)
#ifndef SG_BWD_WAVES_PER_EU
#define SG_BWD_WAVES_PER_EU 6
#endif

template <int TW, int TH, bool H6, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(H6 ? 4 : SG_BWD_WAVES_PER_EU))) k_render_bwd(const steepgs_splat* __restrict__ splats,
                                                               const uint32_t* __restrict__ vals,
                                                               const uint32_t* __restrict__ ranges,
                                                               const steepgs_camera* __restrict__ cams, int V,
                                                               steepgs_opts opt, int total_tiles,
                                                               const float* __restrict__ image,
                                                               const float* __restrict__ T_final,
                                                               const uint32_t* __restrict__ n_contrib,
                                                               const float* __restrict__ dL_dimage,
                                                               const float* __restrict__ target,
                                                               Slots g2d, int64_t m,
                                                               uint32_t* __restrict__ queue) {
  constexpr int NQ = TW * TH / 64;  // 8x8 quadrants of the tile = pixels per lane
  constexpr int QX = TW / 8;
  __shared__ float4 s_a[WAVES][64];  // float32 mean x, y, long axis x, y
  __shared__ float4 s_c[WAVES][64];  // e_long, e_short, opacity, red
  __shared__ float4 s_e[WAVES][64];  // green, blue, remainder constants cl, cs
  __shared__ float s_t[WAVES][64];   // smallest power2 taken (entry_power2_min)
  __shared__ uint32_t s_id[WAVES][64];  // record id
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 7, ly = lane >> 3;
  const int red_idx = reduce9_index(lane);
  float4* const A = s_a[wave];
  float4* const Cq = s_c[wave];
  float4* const E = s_e[wave];
  uint32_t* const Id = s_id[wave];
  float* const Th = s_t[wave];
  const float cut = footprint_power2_cut(opt);
  for (;;) {
    // the wave barrier keeps the lane-0 fetch inside the loop
    __builtin_amdgcn_wave_barrier();
    uint32_t ticket = 0;
    if (lane == 0) ticket = atomicAdd(queue, 1u);
    const int tile = (int)__builtin_amdgcn_readfirstlane(ticket);
    if (tile >= total_tiles) break;
    const int v = view_of_tile(cams, V, tile);
    const int W = cams[v].width, H = cams[v].height, tiles_x = cams[v].tiles_x;
    const int64_t pix_off = cams[v].pixel_offset;
    const int lt = tile - cams[v].tile_offset;
    const int tx0 = (lt % tiles_x) * TW, ty0 = (lt / tiles_x) * TH;
    const uint32_t begin = ranges[2 * tile];
    const int64_t plane = (int64_t)W * H;
    const float inv = 1.f / (3.f * (float)W * (float)H);
    // per-pixel state of the lane's pixel in every quadrant; D = dL/dC . R with
    // R the colour of everything behind the current entry (background included)
    float T[NQ], dC[NQ][3], D[NQ];
    uint32_t last[NQ], qlast[NQ];
    int count = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int px = tx0 + (q % QX) * 8 + lx, py = ty0 + (q / QX) * 8 + ly;
      T[q] = 1.f;
      last[q] = 0;
      dC[q][0] = dC[q][1] = dC[q][2] = 0.f;
      D[q] = 0.f;
      if (px < W && py < H) {
        const int64_t pp = pix_off + (int64_t)py * W + px;
        const int64_t e = 3 * pix_off + (int64_t)py * W + px;
        T[q] = T_final[pp];
        last[q] = n_contrib[pp];
        if (dL_dimage) {
          dC[q][0] = dL_dimage[e];
          dC[q][1] = dL_dimage[e + plane];
          dC[q][2] = dL_dimage[e + 2 * plane];
        } else {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            const float d = image[e + ch * plane] - target[e + ch * plane];
            dC[q][ch] = (d > 0.f) ? inv : ((d < 0.f) ? -inv : 0.f);
          }
        }
        D[q] = T[q] * (dC[q][0] * opt.bg[0] + dC[q][1] * opt.bg[1] + dC[q][2] * opt.bg[2]);
      }
      // entries at or past a quadrant's last contributor need no work for it
      qlast[q] = (uint32_t)__builtin_amdgcn_readfirstlane(wave_max_u32(last[q]));
      count = max(count, (int)qlast[q]);
    }
    for (int b_end = count; b_end > 0; b_end -= 64) {
      const int b_start = b_end > 64 ? b_end - 64 : 0;
      // stage one batch of 64 entries in the wave's LDS slice; the loading
      // lane tests the entry's cut-off region (bounding box, then the
      // ellipse) against every quadrant
      const bool have = b_start + lane < b_end;
      bool hitq[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) hitq[q] = false;
      __builtin_amdgcn_wave_barrier();
      if (have) {
        const uint32_t id = vals[begin + b_start + lane];
        const steepgs_splat sp = splats[id];
        float ex, ey;
        cutoff_extent(sp.conic_a, sp.conic_b, sp.conic_c, sp.opacity, opt, ex, ey);
        const float lev = cutoff_level(sp.opacity, opt);
        const float ia = __builtin_amdgcn_rcpf(sp.conic_a), ic = __builtin_amdgcn_rcpf(sp.conic_c);
        const float2 rc = rem_axes(sp);
        A[lane] = make_float4(sp.mean_x, sp.mean_y, sp.axis_x, sp.axis_y);
        Cq[lane] = make_float4(sp.e_long, sp.e_short, sp.opacity, sp.rgb[0]);
        E[lane] = make_float4(sp.rgb[1], sp.rgb[2], rc.x, rc.y);
        Th[lane] = entry_power2_min(sp.opacity, cut, opt);
        Id[lane] = id;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const float x0 = (float)(tx0 + (q % QX) * 8), y0 = (float)(ty0 + (q / QX) * 8);
          hitq[q] = (sp.mean_x + ex >= x0) && (sp.mean_x - ex <= x0 + 7.f) && (sp.mean_y + ey >= y0) &&
                    (sp.mean_y - ey <= y0 + 7.f) &&
                    block_reach(sp.mean_x, sp.mean_y, sp.conic_a, sp.conic_b, sp.conic_c, ia, ic, lev, x0, y0,
                                x0 + 7.f, y0 + 7.f);
        }
      }
      uint64_t qm[NQ], any_q = 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        qm[q] = uniform_u64(ballot(hitq[q]));
        // only entries below the quadrant's last contributor
        const int lim = (int)qlast[q] - b_start;
        if (lim <= 0) qm[q] = 0;
        else if (lim < 64) qm[q] &= (1ull << lim) - 1ull;
        any_q |= qm[q];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // back to front over the batch
      while (any_q) {
        const int j = 63 - (int)__builtin_clzll(any_q);
        any_q &= ~(1ull << j);
        const float4 a = A[j];
        const float4 cq = Cq[j];
        const uint32_t pos = (uint32_t)(b_start + j);
        const float4 ej = E[j];  // green, blue, cl, cs
        const float pmin = Th[j];
        // moments of g alpha d over the tile's pixels, in the frame of the
        // footprint's axes (pl = axis . d, ps = axis_perp . d, d the offset
        // from the exact mean: for a thin footprint the moments across it
        // would cancel to nothing in pixel coordinates; the lift turns them
        // into pixel coordinates in fp64; the mean and conic gradients are
        // linear in them), sum of g alpha (the opacity gradient times o) and
        // colour gradients.  The
        // per-pixel work is predicated (selects, no divergent branch), so the
        // sums are updated in place; a quadrant is skipped as a whole when
        // the entry is outside its reach or no pixel of it takes the entry.
        float mx = 0.f, my = 0.f, mxx = 0.f, mxy = 0.f, myy = 0.f, s0 = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f;
        float h3[4] = {0.f, 0.f, 0.f, 0.f}, h4[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        uint64_t took = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (!((qm[q] >> j) & 1ull)) continue;  // wave-uniform
          const float dx = (float)(tx0 + (q % QX) * 8 + lx) - a.x;
          const float dy = (float)(ty0 + (q / QX) * 8 + ly) - a.y;
          // offsets from the exact mean along and across the footprint's axis
          float pl, ps;
          const float power = splat_power2_axes(dx, dy, a.z, a.w, ej.z, ej.w, cq.x, cq.y, pl, ps);
          const float raw = cq.z * __builtin_amdgcn_exp2f(power);
          const bool clamped = raw > opt.alpha_max;
          const float alpha = clamped ? opt.alpha_max : raw;  // min(alpha_max, raw): raw is finite
          // entries at or past the pixel's last contributor (or outside the
          // image) and those below the cut-offs were skipped by the forward
          const uint64_t cm = ballot(pos < last[q]) & ballot(power >= pmin);
          if (!cm) continue;
          took |= cm;
          // the rest runs under the taking lanes' mask
          if (!__builtin_amdgcn_inverse_ballot_w64(cm)) continue;
          // transmittance in front of this entry, T_i = T_{i+1} / (1 - alpha_i),
          // with the hardware reciprocal (within 1 ulp); alpha <= 1 - 2^-24
          // (the host caps alpha_max below one)
          const float inv_om = __builtin_amdgcn_rcpf(1.f - alpha);
          const float Ti = T[q] * inv_om;
          // g = dL/dalpha_i = sum_c dL/dC_c (c_c T_i - R_c / (1 - alpha_i))
          const float x = dC[q][0] * cq.w + dC[q][1] * ej.x + dC[q][2] * ej.y;
          const float g = Ti * x - D[q] * inv_om;
          const float w = alpha * Ti;
          T[q] = Ti;
          D[q] += x * w;
          gr += w * dC[q][0];
          gg += w * dC[q][1];
          gbl += w * dC[q][2];
          // the clamped alpha does not depend on the mean, conic or opacity
          const float gaw = clamped ? 0.f : g * alpha;
          const float tx = gaw * pl, ty = gaw * ps;
          mx += tx;
          my += ty;
          mxx += tx * pl;
          mxy += tx * ps;
          myy += ty * ps;
          s0 += gaw;  // dL/do = sum g G = s0 / o
          if (H6) {
            const float txx = tx * pl, tyy = ty * ps;
            h3[0] += txx * pl;
            h3[1] += txx * ps;
            h3[2] += tyy * pl;
            h3[3] += tyy * ps;
            const float dxx = pl * pl, dxy = pl * ps, dyy = ps * ps;
            h4[0] += txx * dxx;
            h4[1] += txx * dxy;
            h4[2] += txx * dyy;
            h4[3] += tyy * dxy;
            h4[4] += tyy * dyy;
          }
        }
        if (took) {
          // per-entry sums over the tile, one quantity per lane, and one
          // nine-lane fp64 atomic into the record's slot: the sums over the
          // tiles of a footprint are exact up to fp64 rounding, so their
          // hardware-chosen order leaves the float32 results unchanged
          const float part[9] = {mx, my, mxx, mxy, myy, s0, gr, gg, gbl};
          const float tot = reduce9(part);
          const int64_t rid = (int64_t)Id[j];
          if (red_idx >= 0) unsafeAtomicAdd(g2d.slot + rid * kSlot + red_idx, (double)tot);
          if (H6) {
            const float part2[9] = {h3[0], h3[1], h3[2], h3[3], h4[0], h4[1], h4[2], h4[3], h4[4]};
            const float tot2 = reduce9(part2);
            if (red_idx >= 0) unsafeAtomicAdd(g2d.h6 + rid * kH6 + red_idx, (double)tot2);
          }
        }
      }
    }
  }
}

// The blend takes its moments in the frame of the footprint's float32 axis
// a (pl = a . d, ps = a_perp . d, a_perp = (-a_y, a_x)); with
// d = (pl a + ps a_perp) / |a|^2 they become moments of the pixel offsets:
// mom[i][j] = sum w pl^i ps^j on entry, sum w dx^i dy^j on return (i + j <= K),
// expanded in fp64 (a thin footprint's moments across its axis survive the
// cancellation there)
template <int K>
SG_DEV void axis_to_pixel_moments(double (&mom)[K + 1][K + 1], float axf, float ayf) {
  const double ax = axf, ay = ayf, n2 = ax * ax + ay * ay;
  // dx = xl pl + xs ps, dy = yl pl + ys ps
  const double xl = ax / n2, xs = -ay / n2, yl = ay / n2, ys = ax / n2;
  double out[K + 1][K + 1];
#pragma unroll
  for (int a = 0; a <= K; ++a)
#pragma unroll
    for (int b = 0; b <= K - a; ++b) {
      // coefficients of pl^(a+b-k) ps^k in (xl pl + xs ps)^a (yl pl + ys ps)^b
      double c[K + 1];
      c[0] = 1.0;
#pragma unroll
      for (int k = 1; k <= K; ++k) c[k] = 0.0;
#pragma unroll
      for (int t = 0; t < a + b; ++t) {
        const double u = t < a ? xl : yl, v = t < a ? xs : ys;
#pragma unroll
        for (int k = K; k >= 1; --k) c[k] = c[k] * u + c[k - 1] * v;
        c[0] *= u;
      }
      double s = 0.0;
#pragma unroll
      for (int k = 0; k <= a + b; ++k) s += c[k] * mom[a + b - k][k];
      out[a][b] = s;
    }
#pragma unroll
  for (int a = 0; a <= K; ++a)
#pragma unroll
    for (int b = 0; b <= K - a; ++b) mom[a][b] = out[a][b];
}

// The second-order case written out (m1 and m2 of the lift):
// m1 = (m1l, m1s), m2 = (m2ll, m2ls, m2ss) in the axis frame on entry,
// (x, y) and (xx, xy, yy) on return
SG_DEV void axis_to_pixel_moments2(double& m1l, double& m1s, double& m2ll, double& m2ls, double& m2ss, float axf,
                                   float ayf) {
  const double ax = axf, ay = ayf, n2 = ax * ax + ay * ay;
  const double xl = ax / n2, xs = -ay / n2, yl = ay / n2, ys = ax / n2;
  const double x = xl * m1l + xs * m1s, y = yl * m1l + ys * m1s;
  const double xx = xl * xl * m2ll + 2.0 * xl * xs * m2ls + xs * xs * m2ss;
  const double xy = xl * yl * m2ll + (xl * ys + xs * yl) * m2ls + xs * ys * m2ss;
  const double yy = yl * yl * m2ll + 2.0 * yl * ys * m2ls + ys * ys * m2ss;
  m1l = x;
  m1s = y;
  m2ll = xx;
  m2ls = xy;
  m2ss = yy;
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
  double campos[3];
  camera_centre(cam, campos);
  return colour_channel_fp64(params, n, i, deg, campos, ch) < 0.0;
}

// lane k's double, for every lane of the wavefront (k uniform)
SG_DEV double lane_double(double x, int k) {
  const uint64_t b = __double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), k);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// fp64 rotation of the normalised quaternion qh = q / |q| and the scales
// exp(log_scale) of Gaussian i
SG_DEV void rotation_scales(const float* __restrict__ params, int64_t n, int64_t i, double Rq[3][3], double sc[3],
                            double qh[4], double& qn) {
  double q[4];
  for (int k = 0; k < 4; ++k) q[k] = (double)params[(STEEPGS_ROW_QUAT + k) * n + i];
  qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) qh[k] = q[k] / qn;
  const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  Rq[0][0] = 1.0 - 2.0 * (y * y + z * z); Rq[0][1] = 2.0 * (x * y - w * z); Rq[0][2] = 2.0 * (x * z + w * y);
  Rq[1][0] = 2.0 * (x * y + w * z); Rq[1][1] = 1.0 - 2.0 * (x * x + z * z); Rq[1][2] = 2.0 * (y * z - w * x);
  Rq[2][0] = 2.0 * (x * z - w * y); Rq[2][1] = 2.0 * (y * z + w * x); Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
  for (int k = 0; k < 3; ++k) sc[k] = exp((double)params[(STEEPGS_ROW_LOG_SCALE + k) * n + i]);
}

// bit v - v0 set when view v of [v0, v0 + 32) sees Gaussian i (eight flags in
// flight at a time)
SG_DEV uint32_t visible_views(const uint32_t* __restrict__ tiles, int64_t n, int64_t i, int v0, int nv) {
  uint32_t vis = 0;
  for (int k0 = 0; k0 < nv; k0 += 8) {
    uint32_t f[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) f[k] = (k0 + k < nv) ? tiles[(int64_t)(v0 + k0 + k) * n + i] : 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) vis |= (f[k] != 0u ? 1u : 0u) << (k0 + k);
  }
  return vis;
}

// One thread per Gaussian, two passes over the views: the colour (SH) part
// in fp32, then the geometric chain -- camera map, Pi(Sigma), its inverse,
// (quaternion, scale) -- and the splitting-matrix lift in fp64 (the conic of a
// thin footprint, condition number kappa, loses ~kappa ulps when inverted or
// differentiated in fp32).  The passes keep the SH coefficients and the
// fp64 geometry out of each other's live range (as two kernels they ran
// slower than as one).  The view index stays uniform over the wavefront, so
// camera data are scalar loads; each pass loads the next view's slot while
// it processes the current one.
template <int D>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) k_proj_bwd(const float* __restrict__ params, int64_t n,
                                                  const steepgs_camera* __restrict__ cams, int V, steepgs_opts opt,
                                                  const uint32_t* __restrict__ tiles,
                                                  const steepgs_splat* __restrict__ splats,
                                                  const double* __restrict__ g2d,
                                                  float* __restrict__ grads, float* __restrict__ S) {
  constexpr int NB = (D + 1) * (D + 1);
  // threads past n stay (with no visible view) so that every lane of a
  // wavefront takes part in the per-view lane tables below
  const int64_t i_raw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i_raw < n;
  const int64_t i = live ? i_raw : n - 1;
  const int lane = threadIdx.x & 63;
  float pf[3];
  for (int k = 0; k < 3; ++k) pf[k] = params[(STEEPGS_ROW_MEAN + k) * n + i];
  double dp[3] = {0.0, 0.0, 0.0};
  bool any = false;

  // pass 1: colour, rgb = max(0, sum_k sh_k Y_k(dir) + 1/2) (the clamp decision
  // re-taken in fp64 when within 1e-5 of zero)
  {
    float sh[3 * NB];
#pragma unroll
    for (int k = 0; k < 3 * NB; ++k) sh[k] = params[(STEEPGS_ROW_SH + k) * n + i];
    float dsh[3 * NB];
#pragma unroll
    for (int k = 0; k < 3 * NB; ++k) dsh[k] = 0.f;
    for (int v0 = 0; v0 < V; v0 += 32) {
      const int nv = min(32, V - v0);
      const uint32_t vis = live ? visible_views(tiles, n, i, v0, nv) : 0u;
      // lane k holds the camera centre of view v0 + k (read per view by readlane)
      float centre_k[3];
      {
        const steepgs_camera& ck = cams[v0 + (lane < nv ? lane : 0)];
        for (int e = 0; e < 3; ++e)
          centre_k[e] = -(ck.R[0 + e] * ck.t[0] + ck.R[3 + e] * ck.t[1] + ck.R[6 + e] * ck.t[2]);
      }
      // the next view's colour gradient is loaded while this one is processed
      double nc[3] = {0.0, 0.0, 0.0};
      auto fetch = [&](int k) {
        if ((vis >> k) & 1u) {
          const double* slot = g2d + ((int64_t)(v0 + k) * n + i) * kSlot;
          for (int e = 0; e < 3; ++e) nc[e] = slot[6 + e];
        }
      };
      fetch(0);
      for (int k = 0; k < nv; ++k) {
        const float gcol[3] = {(float)nc[0], (float)nc[1], (float)nc[2]};
        if (k + 1 < nv) fetch(k + 1);
        if (!((vis >> k) & 1u)) continue;
        const int v = v0 + k;
        if (gcol[0] == 0.f && gcol[1] == 0.f && gcol[2] == 0.f) continue;
        any = true;
        const steepgs_camera& cam = cams[v];
        float campos[3];
        for (int e = 0; e < 3; ++e) campos[e] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(centre_k[e]), k));
        const float dv[3] = {pf[0] - campos[0], pf[1] - campos[1], pf[2] - campos[2]};
        // 1 / |p - c| by the hardware reciprocal square root (1 ulp): the
        // direction enters the gradients only
        const float idl = __builtin_amdgcn_rsqf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        const float dir[3] = {dv[0] * idl, dv[1] * idl, dv[2] * idl};
        float Y[NB];
        sh_eval<float>(D, dir[0], dir[1], dir[2], Y);
        float dcol[3];
        for (int ch = 0; ch < 3; ++ch) {
          float raw = 0.5f;
#pragma unroll
          for (int e = 0; e < NB; ++e) raw += sh[3 * e + ch] * Y[e];
          bool clamped = raw < 0.f;
          if (fabsf(raw) < 1e-5f) clamped = colour_clamped_fp64(params, n, i, D, cam, ch);
          dcol[ch] = clamped ? 0.f : gcol[ch];
        }
        float dY[NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) {
          dY[e] = sh[3 * e] * dcol[0] + sh[3 * e + 1] * dcol[1] + sh[3 * e + 2] * dcol[2];
          dsh[3 * e] += Y[e] * dcol[0];
          dsh[3 * e + 1] += Y[e] * dcol[1];
          dsh[3 * e + 2] += Y[e] * dcol[2];
        }
        if (D > 0) {
          float gd[3] = {0.f, 0.f, 0.f};
          sh_grad<float>(D, dir[0], dir[1], dir[2], dY, gd);
          const float dot = gd[0] * dir[0] + gd[1] * dir[1] + gd[2] * dir[2];
          for (int e = 0; e < 3; ++e) dp[e] += (double)((gd[e] - dir[e] * dot) * idl);
        }
      }
    }
    if (any) {
#pragma unroll
      for (int k = 0; k < 3 * NB; ++k) grads[(STEEPGS_ROW_SH + k) * n + i] += dsh[k];
    }
  }

  // pass 2: geometry.  Covariance R diag(s^2) R^T and opacity in fp64; the
  // rotation is formed again after the loop rather than kept live across it.
  const int ij[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  double Sg[6];  // unique entries xx xy xz yy yz zz
  {
    double Rq[3][3], sc[3], qh[4], qn;
    rotation_scales(params, n, i, Rq, sc, qh, qn);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = ij[k][0], b = ij[k][1];
      Sg[k] = Rq[a][0] * sc[0] * sc[0] * Rq[b][0] + Rq[a][1] * sc[1] * sc[1] * Rq[b][1] +
              Rq[a][2] * sc[2] * sc[2] * Rq[b][2];
    }
  }
  const double o = 1.0 / (1.0 + exp(-(double)params[STEEPGS_ROW_OPACITY * n + i]));
  double dSig[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, dop = 0.0;
  double S3[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int v0 = 0; v0 < V; v0 += 32) {
    const int nv = min(32, V - v0);
    const uint32_t vis = live ? visible_views(tiles, n, i, v0, nv) : 0u;
    // lane k holds the frustum-guard limits of view v0 + k (the projection's
    // expression, so the clamp decisions match); read per view by readlane
    double lim_k[2] = {0.0, 0.0};
    if (opt.frustum_guard > 0.f) {
      const steepgs_camera& ck = cams[v0 + (lane < nv ? lane : 0)];
      lim_k[0] = (double)opt.frustum_guard * (0.5 * ck.width / (double)ck.fx);
      lim_k[1] = (double)opt.frustum_guard * (0.5 * ck.height / (double)ck.fy);
    }
    // the next view's moments and footprint axis are loaded while this one
    // is processed
    double nm[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    float nax = 1.f, nay = 0.f;
    auto fetch = [&](int k) {
      if ((vis >> k) & 1u) {
        const int64_t r = (int64_t)(v0 + k) * n + i;
        const double* slot = g2d + r * kSlot;
        for (int e = 0; e < 6; ++e) nm[e] = slot[e];
        nax = splats[r].axis_x;
        nay = splats[r].axis_y;
      }
    };
    fetch(0);
    for (int k = 0; k < nv; ++k) {
      double cm[6];
      for (int e = 0; e < 6; ++e) cm[e] = nm[e];
      const float cax = nax, cay = nay;
      if (k + 1 < nv) fetch(k + 1);
      if (!((vis >> k) & 1u)) continue;
      const int v = v0 + k;
      const double m0 = cm[5];  // sum g alpha = o dL/do
      double m1x = cm[0], m1y = cm[1], m2xx = cm[2], m2xy = cm[3], m2yy = cm[4];
      if (m1x == 0.0 && m1y == 0.0 && m2xx == 0.0 && m2xy == 0.0 && m2yy == 0.0 && m0 == 0.0) continue;
      any = true;
      axis_to_pixel_moments2(m1x, m1y, m2xx, m2xy, m2yy, cax, cay);
      const steepgs_camera& cam = cams[v];
      double W[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) W[e] = (double)cam.R[e];
      const double fx = cam.fx, fy = cam.fy;

      // camera-space position: fp64 in the forward's operation order for the guard decision
      double pcd[3];
      {
#pragma clang fp contract(off)
        for (int e = 0; e < 3; ++e)
          pcd[e] = (double)cam.R[3 * e + 0] * (double)pf[0] + (double)cam.R[3 * e + 1] * (double)pf[1] +
                   (double)cam.R[3 * e + 2] * (double)pf[2] + (double)cam.t[e];
      }
      double J[2][3];
      double gx = 0.0, gy = 0.0;
      bool gx_free = false, gy_free = false;
      if (cam.model == 0) {
        gx = pcd[0] / pcd[2];
        gy = pcd[1] / pcd[2];
        gx_free = gy_free = true;
        if (opt.frustum_guard > 0.f) {
          const double limx = lane_double(lim_k[0], k), limy = lane_double(lim_k[1], k);
          if (gx < -limx) { gx = -limx; gx_free = false; }
          if (gx > limx) { gx = limx; gx_free = false; }
          if (gy < -limy) { gy = -limy; gy_free = false; }
          if (gy > limy) { gy = limy; gy_free = false; }
        }
        const double iz = 1.0 / pcd[2];
        J[0][0] = fx * iz; J[0][1] = 0.0; J[0][2] = -fx * gx * iz;
        J[1][0] = 0.0; J[1][1] = fy * iz; J[1][2] = -fy * gy * iz;
      } else {
        J[0][0] = fx; J[0][1] = 0.0; J[0][2] = 0.0;
        J[1][0] = 0.0; J[1][1] = fy; J[1][2] = 0.0;
      }
      double P[2][3];
      // P = J W without the products by J's structural zeros (J01 = J10 = 0)
      for (int c = 0; c < 3; ++c) {
        P[0][c] = J[0][0] * W[c] + J[0][2] * W[6 + c];
        P[1][c] = J[1][1] * W[3 + c] + J[1][2] * W[6 + c];
      }
      const double Sig[3][3] = {{Sg[0], Sg[1], Sg[2]}, {Sg[1], Sg[3], Sg[4]}, {Sg[2], Sg[4], Sg[5]}};
      // Pi(Sigma) and its inverse (the conic)
      double PS[2][3];
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) PS[a][c] = P[a][0] * Sig[0][c] + P[a][1] * Sig[1][c] + P[a][2] * Sig[2][c];
      const double s00 = PS[0][0] * P[0][0] + PS[0][1] * P[0][1] + PS[0][2] * P[0][2] + (double)opt.dilation;
      const double s01 = PS[0][0] * P[1][0] + PS[0][1] * P[1][1] + PS[0][2] * P[1][2];
      const double s11 = PS[1][0] * P[1][0] + PS[1][1] * P[1][1] + PS[1][2] * P[1][2] + (double)opt.dilation;
      const double idet = 1.0 / (s00 * s11 - s01 * s01);
      const double A[2][2] = {{s11 * idet, -s01 * idet}, {-s01 * idet, s00 * idet}};
      // 2D mean and conic gradients from the moments
      const double gmx = A[0][0] * m1x + A[0][1] * m1y, gmy = A[1][0] * m1x + A[1][1] * m1y;
      const double ga = -0.5 * m2xx, gb = -m2xy, gc = -0.5 * m2yy;

      // conic -> Pi(Sigma): dL/dS2 = -A G_A A, G_A = [[ga, gb/2], [gb/2, gc]]
      const double GA[2][2] = {{ga, 0.5 * gb}, {0.5 * gb, gc}};
      double AG[2][2], GS2[2][2];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) AG[a][b] = A[a][0] * GA[0][b] + A[a][1] * GA[1][b];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) GS2[a][b] = -(AG[a][0] * A[0][b] + AG[a][1] * A[1][b]);
      // Pi(Sigma) = P Sigma P^T + dilation: dL/dSigma += P^T GS2 P; dL/dP = 2 GS2 P Sigma
      double GSP[2][3];
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) GSP[a][c] = GS2[a][0] * P[0][c] + GS2[a][1] * P[1][c];
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const int c = ij[e][0], d = ij[e][1];
        dSig[e] += P[0][c] * GSP[0][d] + P[1][c] * GSP[1][d];
      }
      double GJ[2][3];
      for (int a = 0; a < 2; ++a) {
        double GP[3];
        for (int c = 0; c < 3; ++c)
          GP[c] = 2.0 * (GSP[a][0] * Sig[0][c] + GSP[a][1] * Sig[1][c] + GSP[a][2] * Sig[2][c]);
        // P = J W: dL/dJ = dL/dP W^T
        for (int b = 0; b < 3; ++b) GJ[a][b] = GP[0] * W[3 * b + 0] + GP[1] * W[3 * b + 1] + GP[2] * W[3 * b + 2];
      }
      // camera-space position gradient from the mean and from J
      double dpc[3] = {0.0, 0.0, 0.0};
      double Pe[2][3];  // Jacobian of the projected mean w.r.t. p (exact, unguarded)
      if (cam.model == 0) {
        const double pcx = pcd[0], pcy = pcd[1];
        const double iz = 1.0 / pcd[2], iz2 = iz * iz;
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
        // exact Jacobian of the projected mean times W (its zeros left out)
        const double je00 = fx * iz, je02 = -fx * pcx * iz2, je11 = fy * iz, je12 = -fy * pcy * iz2;
        for (int c = 0; c < 3; ++c) {
          Pe[0][c] = je00 * W[c] + je02 * W[6 + c];
          Pe[1][c] = je11 * W[3 + c] + je12 * W[6 + c];
        }
      } else {
        dpc[0] += gmx * fx;
        dpc[1] += gmy * fy;
        for (int a = 0; a < 2; ++a)
          for (int c = 0; c < 3; ++c) Pe[a][c] = P[a][c];
      }
      for (int c = 0; c < 3; ++c) dp[c] += W[c] * dpc[0] + W[3 + c] * dpc[1] + W[6 + c] * dpc[2];
      dop += m0;  // sum over views of o dL/do, divided by o once

      // splitting matrix: S2D = A M A - m0 A, M = m2
      const double M[2][2] = {{m2xx, m2xy}, {m2xy, m2yy}};
      double AM[2][2], S2D[2][2];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) AM[a][b] = A[a][0] * M[0][b] + A[a][1] * M[1][b];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) S2D[a][b] = AM[a][0] * A[0][b] + AM[a][1] * A[1][b] - m0 * A[a][b];
      double SP[2][3];
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) SP[a][c] = S2D[a][0] * Pe[0][c] + S2D[a][1] * Pe[1][c];
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const int a = ij[e][0], b = ij[e][1];
        S3[e] += Pe[0][a] * SP[0][b] + Pe[1][a] * SP[1][b];
      }
    }
  }
  if (!any) return;

  // Sigma = M M^T, M = R diag(s): dL/dM = 2 dSig M (dSig symmetric)
  double Rq[3][3], sc[3], qh[4], qn;
  rotation_scales(params, n, i, Rq, sc, qh, qn);
  const double w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  const double G[3][3] = {{dSig[0], dSig[1], dSig[2]}, {dSig[1], dSig[3], dSig[4]}, {dSig[2], dSig[4], dSig[5]}};
  double GR[3][3], dls[3];
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double gm = 2.0 * (G[a][0] * Rq[0][k] + G[a][1] * Rq[1][k] + G[a][2] * Rq[2][k]) * sc[k];
      acc += gm * Rq[a][k];
      GR[a][k] = gm * sc[k];
    }
    dls[k] = acc * sc[k];
  }
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
  float* gp = grads + i;
  for (int k = 0; k < 3; ++k) gp[(STEEPGS_ROW_MEAN + k) * n] += (float)dp[k];
  for (int k = 0; k < 3; ++k) gp[(STEEPGS_ROW_LOG_SCALE + k) * n] += (float)dls[k];
  for (int k = 0; k < 4; ++k) gp[(STEEPGS_ROW_QUAT + k) * n] += (float)((dq[k] - qh[k] * qd) / qn);
  gp[STEEPGS_ROW_OPACITY * n] += (float)(dop * (1.0 - o));  // dL/do o (1 - o), dL/do = dop / o
  if (S)
    for (int k = 0; k < 6; ++k) S[k * n + i] += (float)S3[k];
}

// ---------------------------------------------------------------------------
// kernel 3 (dim 6): the splitting matrix over theta = (p, log-scales), from the
// pixel moments of every view.  With the projection's maps frozen at the point
// (the mean moves along the exact Jacobian Pe, the 2D covariance is
// Pg Sigma(s) Pg^T + dilation, Pg = J W with J at the guarded point), per
// pixel q = d^T A d has
//   dq/dp = -2 Pe^T A d,  dq/ds_k = -2 sig_k^2 z_k^2,  z_k = a_k . d,
//   a_k = A w_k, w_k = Pg r_k (r_k the k-th axis of the rotation, sig_k^2 =
//   exp(2 s_k)), d2q/dp2 = 2 Pe^T A Pe, d2q/dp ds_k = 4 sig_k^2 z_k Pe^T a_k,
//   d2q/ds_j ds_k = -4 sig_k^2 [j = k] z_k^2 + 8 sig_j^2 sig_k^2 M_jk z_j z_k,
//   M_jk = w_j^T A w_k,
// and Hess alpha = alpha (dq dq^T / 4 - d2q / 2).  Summed with g = dL/dalpha
// over a view's pixels, every block is a contraction of the moments
// m0 = sum g alpha, m1 = sum g alpha d, m2 (second), m3 (third), m4 (fourth):
//   S_pp = Pe^T (A m2 A - m0 A) Pe,
//   S_ps[:, k] = sig_k^2 Pe^T (A T3(a_k) - 2 (a_k . m1) a_k),
//   S_ss[j][k] = sig_j^2 sig_k^2 T4(a_j, a_k) + 2 sig_k^2 [j = k] T2(a_k, a_k)
//                - 4 sig_j^2 sig_k^2 M_jk T2(a_j, a_k),
// T2(a, b) = a^T m2 b, T3(a) = sum g alpha d (a . d)^2, T4(a, b) =
// sum g alpha (a . d)^2 (b . d)^2.  S6 [21][n] accumulates the upper triangle,
// row-major over (p_x, p_y, p_z, s_x, s_y, s_z).

SG_DEV int h6_slot(int i, int j) { return i <= j ? i * 6 - i * (i - 1) / 2 + (j - i) : j * 6 - j * (j - 1) / 2 + (i - j); }

// coefficients of (a . d)^2 in (dx^2, dx dy, dy^2)
SG_DEV void sq_coef(const double a[2], double c[3]) {
  c[0] = a[0] * a[0];
  c[1] = 2.0 * a[0] * a[1];
  c[2] = a[1] * a[1];
}

__global__ void __launch_bounds__(128) k_split6_lift(const float* __restrict__ params, int64_t n,
                                                     const steepgs_camera* __restrict__ cams, int V, steepgs_opts opt,
                                                     const uint32_t* __restrict__ tiles,
                                                     const steepgs_splat* __restrict__ splats,
                                                     const double* __restrict__ g2d,
                                                     const double* __restrict__ h6, float* __restrict__ S6) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double p[3], q[4], s2[3];
  for (int k = 0; k < 3; ++k) p[k] = params[(STEEPGS_ROW_MEAN + k) * n + i];
  for (int k = 0; k < 4; ++k) q[k] = params[(STEEPGS_ROW_QUAT + k) * n + i];
  for (int k = 0; k < 3; ++k) s2[k] = exp(2.0 * params[(STEEPGS_ROW_LOG_SCALE + k) * n + i]);
  const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  const double Rq[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                          {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                          {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  const double o = 1.0 / (1.0 + exp(-params[STEEPGS_ROW_OPACITY * n + i]));
  double acc[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) acc[k] = 0.0;
  for (int v = 0; v < V; ++v) {
    const int64_t r = (int64_t)v * n + i;
    if (tiles[r] == 0) continue;
    const double* slot = g2d + r * kSlot;
    const double* hs = h6 + r * kH6;
    const double m0 = slot[5];  // sum g alpha
    if (slot[0] == 0.0 && slot[1] == 0.0 && slot[2] == 0.0 && slot[3] == 0.0 && slot[4] == 0.0 && m0 == 0.0) continue;
    // mom[a][b] = sum g alpha dx^a dy^b, from the moments along and across the axis
    double mom[5][5] = {{m0, slot[1], slot[4], hs[3], hs[8]},
                        {slot[0], slot[3], hs[2], hs[7], 0.0},
                        {slot[2], hs[1], hs[6], 0.0, 0.0},
                        {hs[0], hs[5], 0.0, 0.0, 0.0},
                        {hs[4], 0.0, 0.0, 0.0, 0.0}};
    axis_to_pixel_moments<4>(mom, splats[r].axis_x, splats[r].axis_y);
    const double m1[2] = {mom[1][0], mom[0][1]};
    const double m2[3] = {mom[2][0], mom[1][1], mom[0][2]};  // xx, xy, yy
    const double m3[4] = {mom[3][0], mom[2][1], mom[1][2], mom[0][3]};  // xxx, xxy, xyy, yyy
    const double m4[5] = {mom[4][0], mom[3][1], mom[2][2], mom[1][3], mom[0][4]};  // xxxx .. yyyy
    const steepgs_camera& cam = cams[v];
    // camera space (fp64 for the guard decision, as the forward)
    double pcd[3];
    {
#pragma clang fp contract(off)
      for (int k = 0; k < 3; ++k)
        pcd[k] = (double)cam.R[3 * k + 0] * (double)p[0] + (double)cam.R[3 * k + 1] * (double)p[1] +
                 (double)cam.R[3 * k + 2] * (double)p[2] + (double)cam.t[k];
    }
    double Jg[2][3], Je[2][3];
    if (cam.model == 0) {
      double gxd = pcd[0] / pcd[2], gyd = pcd[1] / pcd[2];
      const double exd = gxd, eyd = gyd;
      if (opt.frustum_guard > 0.0) {
        const double limx = (double)opt.frustum_guard * (0.5 * cam.width / (double)cam.fx);
        const double limy = (double)opt.frustum_guard * (0.5 * cam.height / (double)cam.fy);
        gxd = gxd < -limx ? -limx : (gxd > limx ? limx : gxd);
        gyd = gyd < -limy ? -limy : (gyd > limy ? limy : gyd);
      }
      const double iz = 1.0 / pcd[2];
      Jg[0][0] = cam.fx * iz; Jg[0][1] = 0.0; Jg[0][2] = -cam.fx * (double)gxd * iz;
      Jg[1][0] = 0.0; Jg[1][1] = cam.fy * iz; Jg[1][2] = -cam.fy * (double)gyd * iz;
      Je[0][0] = Jg[0][0]; Je[0][1] = 0.0; Je[0][2] = -cam.fx * (double)exd * iz;
      Je[1][0] = 0.0; Je[1][1] = Jg[1][1]; Je[1][2] = -cam.fy * (double)eyd * iz;
    } else {
      Jg[0][0] = cam.fx; Jg[0][1] = 0.0; Jg[0][2] = 0.0;
      Jg[1][0] = 0.0; Jg[1][1] = cam.fy; Jg[1][2] = 0.0;
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) Je[a][c] = Jg[a][c];
    }
    double Pg[2][3], Pe[2][3];
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 3; ++c) {
        Pg[a][c] = Jg[a][0] * cam.R[c] + Jg[a][1] * cam.R[3 + c] + Jg[a][2] * cam.R[6 + c];
        Pe[a][c] = Je[a][0] * cam.R[c] + Je[a][1] * cam.R[3 + c] + Je[a][2] * cam.R[6 + c];
      }
    // w_k = Pg r_k; Sigma_2D = sum_k sig_k^2 w_k w_k^T + dilation; A its inverse
    double wv[3][2];
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 2; ++a) wv[k][a] = Pg[a][0] * Rq[0][k] + Pg[a][1] * Rq[1][k] + Pg[a][2] * Rq[2][k];
    double c00 = opt.dilation, c01 = 0.0, c11 = opt.dilation;
    for (int k = 0; k < 3; ++k) {
      c00 += s2[k] * wv[k][0] * wv[k][0];
      c01 += s2[k] * wv[k][0] * wv[k][1];
      c11 += s2[k] * wv[k][1] * wv[k][1];
    }
    const double idet = 1.0 / (c00 * c11 - c01 * c01);
    const double A[2][2] = {{c11 * idet, -c01 * idet}, {-c01 * idet, c00 * idet}};
    double ak[3][2];
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 2; ++a) ak[k][a] = A[a][0] * wv[k][0] + A[a][1] * wv[k][1];
    const double M2[2][2] = {{m2[0], m2[1]}, {m2[1], m2[2]}};
    // position block: Pe^T (A m2 A - m0 A) Pe
    double AM[2][2], K[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) AM[a][b] = A[a][0] * M2[0][b] + A[a][1] * M2[1][b];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) K[a][b] = AM[a][0] * A[0][b] + AM[a][1] * A[1][b] - m0 * A[a][b];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        double t = 0.0;
        for (int x2 = 0; x2 < 2; ++x2)
          for (int y2 = 0; y2 < 2; ++y2) t += Pe[x2][a] * K[x2][y2] * Pe[y2][b];
        acc[h6_slot(a, b)] += t;
      }
    // mixed block
    double cf[3][3];
    for (int k = 0; k < 3; ++k) sq_coef(ak[k], cf[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double t3x = cf[k][0] * m3[0] + cf[k][1] * m3[1] + cf[k][2] * m3[2];
      const double t3y = cf[k][0] * m3[1] + cf[k][1] * m3[2] + cf[k][2] * m3[3];
      const double c1 = ak[k][0] * m1[0] + ak[k][1] * m1[1];
      const double vx = A[0][0] * t3x + A[0][1] * t3y - 2.0 * c1 * ak[k][0];
      const double vy = A[1][0] * t3x + A[1][1] * t3y - 2.0 * c1 * ak[k][1];
#pragma unroll
      for (int a = 0; a < 3; ++a) acc[h6_slot(a, 3 + k)] += s2[k] * (Pe[0][a] * vx + Pe[1][a] * vy);
    }
    // scale block
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = j; k < 3; ++k) {
        const double* aj = cf[j];
        const double* bk = cf[k];
        const double t4 = aj[0] * bk[0] * m4[0] + (aj[0] * bk[1] + aj[1] * bk[0]) * m4[1] +
                         (aj[0] * bk[2] + aj[1] * bk[1] + aj[2] * bk[0]) * m4[2] +
                         (aj[1] * bk[2] + aj[2] * bk[1]) * m4[3] + aj[2] * bk[2] * m4[4];
        const double t2 = ak[j][0] * (M2[0][0] * ak[k][0] + M2[0][1] * ak[k][1]) +
                         ak[j][1] * (M2[1][0] * ak[k][0] + M2[1][1] * ak[k][1]);
        const double Mjk = wv[j][0] * ak[k][0] + wv[j][1] * ak[k][1];
        double t = s2[j] * s2[k] * (t4 - 4.0 * Mjk * t2);
        if (j == k) t += 2.0 * s2[k] * t2;
        acc[h6_slot(3 + j, 3 + k)] += t;
      }
  }
#pragma unroll
  for (int k = 0; k < 21; ++k) S6[k * n + i] += (float)acc[k];
}

// the caller's 2D-gradient buffer: moments -> mean and conic gradients, with
// the conic the raster kernels used (the projected record's)
__global__ void k_export2d(const steepgs_splat* __restrict__ splats, const uint32_t* __restrict__ tiles, int64_t m,
                           const double* __restrict__ g2d, float* __restrict__ out) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    float* o = out + r * kGrad2dOut;
    float v[kGrad2dOut];
#pragma unroll
    for (int k = 0; k < kGrad2dOut; ++k) v[k] = 0.f;
    if (tiles[r] != 0) {
      const double* slot = g2d + r * kSlot;
      double m1x = slot[0], m1y = slot[1], m2xx = slot[2], m2xy = slot[3], m2yy = slot[4];
      axis_to_pixel_moments2(m1x, m1y, m2xx, m2xy, m2yy, splats[r].axis_x, splats[r].axis_y);
      const double a = splats[r].conic_a, b = splats[r].conic_b, c = splats[r].conic_c;
      v[0] = (float)(a * m1x + b * m1y);
      v[1] = (float)(b * m1x + c * m1y);
      v[2] = (float)(-0.5 * m2xx);
      v[3] = (float)(-m2xy);
      v[4] = (float)(-0.5 * m2yy);
      // slot[5] = sum g alpha = o dL/do
      const double o = splats[r].opacity;
      v[5] = o > 0.0 ? (float)(slot[5] / o) : 0.f;
#pragma unroll
      for (int k = 6; k < 9; ++k) v[k] = (float)slot[k];
    }
#pragma unroll
    for (int k = 0; k < kGrad2dOut; ++k) o[k] = v[k];
  }
}

__global__ void k_zero(float* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

__global__ void k_zero64(double* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// the slot arrays are carved back to back, so one fill clears them
static size_t bwd_layout(void* base, int64_t m, bool h6, Slots* g2d, uint32_t** queue) {
  Carver c(base);
  *queue = c.take<uint32_t>(64);
  double* all = c.take<double>((size_t)(kSlot + (h6 ? kH6 : 0)) * m);
  g2d->slot = all;
  g2d->h6 = (all && h6) ? all + (size_t)kSlot * m : nullptr;
  return c.used + 256;
}

size_t render_bwd_workspace(int64_t m) {
  Slots g;
  uint32_t* q;
  return bwd_layout(nullptr, m, false, &g, &q);
}

size_t render_bwd6_workspace(int64_t m) {
  Slots g;
  uint32_t* q;
  return bwd_layout(nullptr, m, true, &g, &q);
}

template <int TW, int TH, bool H6>
static void launch_bwd(int grid, hipStream_t st, const steepgs_splat* splats, const uint32_t* vals,
                       const uint32_t* ranges, const steepgs_camera* cams, int V, const steepgs_opts& opt,
                       int total_tiles, const float* image, const float* T_final, const uint32_t* n_contrib,
                       const float* dL_dimage, const float* target, Slots g2d, int64_t m, uint32_t* queue) {
#define SG_BWD(WAVES)                                                                                              \
  hipLaunchKernelGGL((k_render_bwd<TW, TH, H6, WAVES>), dim3(grid), dim3(64 * WAVES), 0, st, splats, vals, ranges,  \
                     cams, V, opt, total_tiles, image, T_final, n_contrib, dL_dimage, target, g2d, m, queue)
  const int w = raster_waves(opt);
  if (w == 2) SG_BWD(2); else if (w == 8) SG_BWD(8); else SG_BWD(4);
#undef SG_BWD
}

}  // namespace sg

using namespace sg;

static steepgs_status bwd_impl(const float* d_params, int64_t n, int32_t sh_degree, const steepgs_camera* d_cams,
                               int32_t V, const steepgs_opts* opts, const steepgs_splat* d_splats,
                               const uint32_t* d_tiles_touched, const uint32_t* d_vals,
                               const uint32_t* d_tile_ranges, int32_t total_tiles, int64_t total_pixels,
                               const float* d_image, const float* d_T_final, const uint32_t* d_n_contrib,
                               const float* d_dL_dimage, const float* d_target, float* d_grads, float* d_S,
                               float* d_S6, float* d_grad2d, void* d_ws, size_t ws_bytes, void* stream,
                               bool clear = true) {
  const bool h6 = d_S6 != nullptr;
  if (n < 0 || V <= 0 || sh_degree < 0 || sh_degree > 3 || total_tiles <= 0 || total_pixels <= 0 || !opts_ok(opts))
    return STEEPGS_ERR_INVALID_ARG;
  if (!d_cams || !d_tile_ranges || !d_T_final || !d_n_contrib) return STEEPGS_ERR_INVALID_ARG;
  if (!d_dL_dimage && (!d_target || !d_image)) return STEEPGS_ERR_INVALID_ARG;
  if (n == 0) return STEEPGS_OK;  // nothing to accumulate; the per-Gaussian buffers may be empty
  if (!d_params || !d_splats || !d_tiles_touched || !d_grads || (!d_S && !h6)) return STEEPGS_ERR_INVALID_ARG;
  const int64_t m = (int64_t)V * n;
  const int per_record = kSlot + (h6 ? kH6 : 0);
  Slots g2d;
  uint32_t* queue;
  const size_t need = bwd_layout(nullptr, m, h6, &g2d, &queue);
  if (!d_ws || ws_bytes < need) return STEEPGS_ERR_WORKSPACE;
  bwd_layout(d_ws, m, h6, &g2d, &queue);
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, reinterpret_cast<float*>(queue), (int64_t)1);
  if (clear)
    hipLaunchKernelGGL(k_zero64, dim3(stride_grid(per_record * m, 256)), dim3(256), 0, st, g2d.slot, per_record * m);
  const steepgs_opts o = raster_opts(*opts);
  const int grid = raster_grid(o, total_tiles);
  timer_begin(STEEPGS_TIMER_RENDER_BWD, st);
#define SG_LAUNCH_BWD(TW, TH)                                                                                        \
  (h6 ? launch_bwd<TW, TH, true>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_image,       \
                                 d_T_final, d_n_contrib, d_dL_dimage, d_target, g2d, m, queue)                      \
      : launch_bwd<TW, TH, false>(grid, st, d_splats, d_vals, d_tile_ranges, d_cams, V, o, total_tiles, d_image,     \
                                  d_T_final, d_n_contrib, d_dL_dimage, d_target, g2d, m, queue))
  if (o.tile_w == 16 && o.tile_h == 16)
    SG_LAUNCH_BWD(16, 16);
  else if (o.tile_w == 16 && o.tile_h == 8)
    SG_LAUNCH_BWD(16, 8);
  else
    SG_LAUNCH_BWD(8, 8);
#undef SG_LAUNCH_BWD
  timer_end(STEEPGS_TIMER_RENDER_BWD, st);
  timer_begin(STEEPGS_TIMER_PROJ_BWD, st);
  const dim3 pg((unsigned)ceil_div(n, 128));
  switch (sh_degree) {
    case 0: hipLaunchKernelGGL(k_proj_bwd<0>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, d_splats, g2d.slot, d_grads, d_S); break;
    case 1: hipLaunchKernelGGL(k_proj_bwd<1>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, d_splats, g2d.slot, d_grads, d_S); break;
    case 2: hipLaunchKernelGGL(k_proj_bwd<2>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, d_splats, g2d.slot, d_grads, d_S); break;
    default: hipLaunchKernelGGL(k_proj_bwd<3>, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, d_splats, g2d.slot, d_grads, d_S); break;
  }
  if (h6)
    hipLaunchKernelGGL(k_split6_lift, pg, dim3(128), 0, st, d_params, n, d_cams, V, o, d_tiles_touched, d_splats, g2d.slot,
                       g2d.h6, d_S6);
  timer_end(STEEPGS_TIMER_PROJ_BWD, st);
  if (d_grad2d && !h6)
    hipLaunchKernelGGL(k_export2d, dim3(stride_grid(m, 256)), dim3(256), 0, st, d_splats, d_tiles_touched, m, g2d.slot,
                       d_grad2d);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}



extern "C" steepgs_status steepgs_render_bwd_split(const float* d_params, int64_t n, int32_t sh_degree,
                                                   const steepgs_camera* d_cams, int32_t V, const steepgs_opts* opts,
                                                   const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                                                   const uint32_t* d_vals, const uint32_t* d_tile_ranges,
                                                   int32_t total_tiles, int64_t total_pixels, const float* d_image,
                                                   const float* d_T_final, const uint32_t* d_n_contrib,
                                                   const float* d_dL_dimage, const float* d_target, float* d_grads,
                                                   float* d_S, float* d_grad2d, void* d_ws, size_t ws_bytes,
                                                   void* stream) {
  return bwd_impl(d_params, n, sh_degree, d_cams, V, opts, d_splats, d_tiles_touched, d_vals, d_tile_ranges,
                  total_tiles, total_pixels, d_image, d_T_final, d_n_contrib, d_dL_dimage, d_target, d_grads, d_S,
                  nullptr, d_grad2d, d_ws, ws_bytes, stream);
}

extern "C" steepgs_status steepgs_render_bwd_clear(int64_t n, int32_t V, void* d_ws, size_t ws_bytes, void* stream) {
  if (n < 0 || V <= 0 || !d_ws) return STEEPGS_ERR_INVALID_ARG;
  if (n == 0) return STEEPGS_OK;
  const int64_t m = (int64_t)V * n;
  Slots g2d;
  uint32_t* queue;
  if (ws_bytes < bwd_layout(nullptr, m, false, &g2d, &queue)) return STEEPGS_ERR_WORKSPACE;
  bwd_layout(d_ws, m, false, &g2d, &queue);
  hipLaunchKernelGGL(k_zero64, dim3(stride_grid(kSlot * m, 256)), dim3(256), 0, as_stream(stream), g2d.slot,
                     kSlot * m);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}

extern "C" steepgs_status steepgs_render_bwd_split_cleared(
    const float* d_params, int64_t n, int32_t sh_degree, const steepgs_camera* d_cams, int32_t V,
    const steepgs_opts* opts, const steepgs_splat* d_splats, const uint32_t* d_tiles_touched, const uint32_t* d_vals,
    const uint32_t* d_tile_ranges, int32_t total_tiles, int64_t total_pixels, const float* d_image,
    const float* d_T_final, const uint32_t* d_n_contrib, const float* d_dL_dimage, const float* d_target,
    float* d_grads, float* d_S, float* d_grad2d, void* d_ws, size_t ws_bytes, void* stream) {
  return bwd_impl(d_params, n, sh_degree, d_cams, V, opts, d_splats, d_tiles_touched, d_vals, d_tile_ranges,
                  total_tiles, total_pixels, d_image, d_T_final, d_n_contrib, d_dL_dimage, d_target, d_grads, d_S,
                  nullptr, d_grad2d, d_ws, ws_bytes, stream, false);
}

extern "C" steepgs_status steepgs_render_bwd_split6(const float* d_params, int64_t n, int32_t sh_degree,
                                                    const steepgs_camera* d_cams, int32_t V, const steepgs_opts* opts,
                                                    const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                                                    const uint32_t* d_vals, const uint32_t* d_tile_ranges,
                                                    int32_t total_tiles, int64_t total_pixels, const float* d_image,
                                                    const float* d_T_final, const uint32_t* d_n_contrib,
                                                    const float* d_dL_dimage, const float* d_target, float* d_grads,
                                                    float* d_S, float* d_S6, void* d_ws, size_t ws_bytes,
                                                    void* stream) {
  if (!d_S6) return STEEPGS_ERR_INVALID_ARG;
  return bwd_impl(d_params, n, sh_degree, d_cams, V, opts, d_splats, d_tiles_touched, d_vals, d_tile_ranges,
                  total_tiles, total_pixels, d_image, d_T_final, d_n_contrib, d_dL_dimage, d_target, d_grads, d_S,
                  d_S6, nullptr, d_ws, ws_bytes, stream);
}
