// Shared device helpers of the SteepGS HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/steepgs.h"

#define SG_DEV __device__ __forceinline__

namespace sg {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// error plumbing for the host side

#define SG_TRY_LAUNCH()                                          \
  do {                                                           \
    hipError_t e_ = hipGetLastError();                           \
    if (e_ != hipSuccess) return STEEPGS_ERR_HIP;                \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline bool opts_ok(const steepgs_opts* o) {
  if (!o) return false;
  const bool tile_ok = (o->tile_w == 16 && o->tile_h == 16) || (o->tile_w == 16 && o->tile_h == 8) ||
                       (o->tile_w == 8 && o->tile_h == 8);
  const bool launch_ok = o->raster_wgs_per_cu >= 0 && o->raster_wgs_per_cu <= 64 &&
                         (o->raster_waves_per_wg == 0 || o->raster_waves_per_wg == 2 || o->raster_waves_per_wg == 4 ||
                          o->raster_waves_per_wg == 8);
  return tile_ok && launch_ok && o->radius_sigmas > 0.f && o->alpha_max > 0.f && o->alpha_max <= 1.f &&
         o->alpha_min >= 0.f && o->t_min >= 0.f && o->t_min < 1.f && o->near_z > 0.f && o->dilation >= 0.f &&
         o->alpha_max >= o->alpha_min;
}

// launch shape of the persistent raster kernels: waves per workgroup and the
// grid (never more workgroups than tiles need)
inline int raster_waves(const steepgs_opts& o) { return o.raster_waves_per_wg > 0 ? o.raster_waves_per_wg : 4; }
int device_cu_count();
inline int raster_grid(const steepgs_opts& o, int total_tiles) {
  const int waves = raster_waves(o);
  const int per_cu = o.raster_wgs_per_cu > 0 ? o.raster_wgs_per_cu : 8;
  const int64_t need = ((int64_t)total_tiles + waves - 1) / waves;
  const int64_t cap = (int64_t)device_cu_count() * per_cu;
  return (int)(need < cap ? need : cap);
}

// The options as the raster kernels take them: alpha capped at 1 - 2^-24, the
// largest float below one, even where alpha_max = 1 (smooth mode), so that
// 1 - alpha never vanishes for a saturated opacity (the blend's factor and the
// divisor of its derivative).
inline steepgs_opts raster_opts(const steepgs_opts& o) {
  steepgs_opts r = o;
  const float cap = 1.f - 5.9604645e-8f;  // 1 - 2^-24
  if (r.alpha_max > cap) r.alpha_max = cap;
  return r;
}

// compute units of the current device (cached per device id)
int device_cu_count();

// Grid for a grid-stride kernel over `items` work items of `per_block` each:
// enough workgroups to fill every CU several times over, never more than the
// items need.  Short-lived waves are limited by the rate at which the
// hardware launches them, so element-wise kernels loop instead.
inline unsigned stride_grid(int64_t items, int per_block) {
  const int64_t need = (items + per_block - 1) / per_block;
  const int64_t cap = (int64_t)device_cu_count() * 16;
  return (unsigned)(need < 1 ? 1 : (need < cap ? need : cap));
}

// optional launch timing (see steepgs_set_kernel_timer)
struct KernelTimer {
  hipEvent_t starts[1024];
  hipEvent_t stops[1024];
  int count = 0;
  int next = 0;
};
KernelTimer* kernel_timers();

inline void timer_begin(int which, hipStream_t st) {
  KernelTimer& t = kernel_timers()[which];
  if (t.count > 0) hipEventRecord(t.starts[t.next], st);
}
inline void timer_end(int which, hipStream_t st) {
  KernelTimer& t = kernel_timers()[which];
  if (t.count > 0) {
    hipEventRecord(t.stops[t.next], st);
    t.next = (t.next + 1) % t.count;
  }
}

// workspace carving: 256-byte aligned bump allocator over the caller's buffer
struct Carver {
  char* base;
  size_t used = 0;
  // the base is rounded up to 256 bytes (every workspace size has 256 bytes of
  // slack for it), so a caller's workspace needs no particular alignment
  explicit Carver(void* p)
      : base(p ? reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255)) : nullptr) {}
  template <class T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

// ---------------------------------------------------------------------------
// wave-level primitives

SG_DEV uint64_t ballot(bool p) { return __ballot(p); }
SG_DEV int lane_id() { return __lane_id(); }
SG_DEV uint64_t lanemask_lt() { return (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id())); }

// sum over the 64 lanes of a wave; every lane receives the total
SG_DEV float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// ---------------------------------------------------------------------------
// camera lookup for a global tile id (V is small; cameras are laid out with
// increasing tile_offset)

SG_DEV int view_of_tile(const steepgs_camera* __restrict__ cams, int V, int tile) {
  int v = 0;
  for (int k = 1; k < V; ++k)
    if (cams[k].tile_offset <= tile) v = k;
  return v;
}

// IEEE binary16 bits of x (nearest even) and the float value of the low 16
// bits of b: the record keeps the remainders of its float32 mean in this form
SG_DEV uint32_t half_bits(float x) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x); }
SG_DEV float half_value(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xFFFFu)); }

// The remainder rem = exact mean - float32 mean of a record
SG_DEV float2 mean_rem(const steepgs_splat& sp) {
  return make_float2(half_value(sp.mean_lo), half_value(sp.mean_lo >> 16));
}

// ---------------------------------------------------------------------------
// Per-pixel opacity of a projected Gaussian (Eq. sigma_2D):
//   alpha = min(alpha_max, o * exp(-1/2 d^T A d)),  d = x - mean,
// with the exponent in base 2 from the conic's eigen form (record fields
// axis, e_long, e_short): -1/2 d^T A d * log2(e) = e_long (axis . d)^2 +
// e_short (axis_perp . d)^2, axis_perp = (-axis_y, axis_x).  Two
// non-negative terms, so float32 loses no digits to cancellation when a thin
// footprint is seen along its long axis (the terms a dx^2, 2 b dx dy, c dy^2
// of the conic would).
// The offsets come from the float32 mean, d0 = x - mean_f = d + rem, which
// depends on the pixel only (not on the tile that holds it); the remainder
// enters through the entry's constants cl = axis . rem, cs = axis_perp . rem
// (rem_axes): axis . d = axis . d0 - cl, at no cost per pixel.  The forward
// and backward raster kernels evaluate it with this one routine, so that
// both see bit-identical values.
SG_DEV float splat_power2_axes(float dx0, float dy0, float ax, float ay, float cl, float cs, float el, float es,
                               float& pl, float& ps) {
  // explicit fused operations: one fixed rounding sequence in every kernel
  pl = __builtin_fmaf(ax, dx0, __builtin_fmaf(ay, dy0, -cl));
  ps = __builtin_fmaf(ax, dy0, __builtin_fmaf(-ay, dx0, -cs));
  return __builtin_fmaf(pl, el * pl, ps * (es * ps));
}

// the same, without the projections on the axes (pl = axis . d, ps = axis_perp . d)
SG_DEV float splat_power2(float dx0, float dy0, float ax, float ay, float cl, float cs, float el, float es) {
  float pl, ps;
  return splat_power2_axes(dx0, dy0, ax, ay, cl, cs, el, es, pl, ps);
}

// (cl, cs) of a record, see splat_power2
SG_DEV float2 rem_axes(const steepgs_splat& sp) {
  const float2 r = mean_rem(sp);
  return make_float2(__builtin_fmaf(sp.axis_x, r.x, sp.axis_y * r.y), __builtin_fmaf(sp.axis_x, r.y, -(sp.axis_y * r.x)));
}

// A pixel takes part in a Gaussian's blend only inside its footprint,
// d^T A d <= radius_sigmas^2, i.e. power2 = -1/2 d^T A d log2(e) >= this
// value.  The forward and backward raster kernels both test against it.
SG_DEV float footprint_power2_cut(const steepgs_opts& opt) {
  return -0.72134752044448170368f * opt.radius_sigmas * opt.radius_sigmas;
}

// The two per-pixel tests of an entry in one: inside the footprint and
// alpha = o 2^power >= alpha_min (alpha_max > alpha_min does not change the
// second), i.e. power >= max(cut, log2(alpha_min / o)).  The log2 form moves
// the alpha_min decision only within float32 rounding of alpha.  The forward
// and backward raster kernels take this one per-entry value.
SG_DEV float entry_power2_min(float o, float cut, const steepgs_opts& opt) {
  return opt.alpha_min > 0.f ? fmaxf(cut, __log2f(opt.alpha_min) - __log2f(o)) : cut;
}

// Half-extents of the region where a pixel can contribute: inside the
// footprint and alpha >= alpha_min, the ellipse d^T A d <= t with
// t = min(radius_sigmas^2, 2 ln(o / alpha_min)); its x half-width is
// sqrt(t (A^-1)_xx).  Widened by 1% and 1/16 pixel so a test against it is
// conservative for the fp32 evaluation; empty (negative) when
// o <= alpha_min.
SG_DEV void cutoff_extent(float a, float b, float c, float o, const steepgs_opts& opt, float& ex, float& ey) {
  float t = opt.radius_sigmas * opt.radius_sigmas;
  if (opt.alpha_min > 0.f) {
    if (!(o > opt.alpha_min)) {
      ex = ey = -INFINITY;
      return;
    }
    t = fminf(t, 2.f * __logf(o / opt.alpha_min));
  }
  const float det = a * c - b * b;
  ex = sqrtf(t * c / det) * 1.01f + 0.0625f;
  ey = sqrtf(t * a / det) * 1.01f + 0.0625f;
}

// Threshold of the same region for an ellipse test, d^T A d <= this value,
// widened like the extents (2% and 1e-3); negative when no pixel can
// contribute.
SG_DEV float cutoff_level(float o, const steepgs_opts& opt) {
  float t = opt.radius_sigmas * opt.radius_sigmas;
  if (opt.alpha_min > 0.f) {
    if (!(o > opt.alpha_min)) return -1.f;
    t = fminf(t, 2.f * __logf(o / opt.alpha_min));
  }
  return t * 1.0201f + 1e-3f;
}

// Conservative test of a pixel block [x0, x1] x [y0, y1] (pixel centres at
// integer coordinates) against the ellipse d^T A d <= t: false only when the
// minimum of the quadratic over the block exceeds t by more than 1e-4 of its
// terms' magnitude (far above the rounding of the blend's fp32 evaluation).
// With the mean outside the block the minimum lies on a face seen from the
// mean -- at most one face across x and one across y -- and on a face it is
// the stationary point along the face, clamped to the face's extent.
// ia, ic: reciprocals of a and c (their rounding moves the evaluated point
// along the face, which changes the value only at second order).
SG_DEV bool block_reach(float mx, float my, float a, float b, float c, float ia, float ic, float t, float x0, float y0,
                        float x1, float y1) {
  const bool fxl = mx < x0, fxh = mx > x1, fyl = my < y0, fyh = my > y1;
  if (!(fxl || fxh || fyl || fyh)) return true;
  float qmin = INFINITY;
  if (fxl || fxh) {
    const float f = (fxl ? x0 : x1) - mx;
    const float r = fminf(fmaxf(-(b * f) * ic, y0 - my), y1 - my);
    const float q = a * f * f + 2.f * b * f * r + c * r * r;
    const float M = a * f * f + 2.f * fabsf(b * f * r) + c * r * r;
    qmin = fminf(qmin, q - 1e-4f * M);
  }
  if (fyl || fyh) {
    const float f = (fyl ? y0 : y1) - my;
    const float r = fminf(fmaxf(-(b * f) * ia, x0 - mx), x1 - mx);
    const float q = c * f * f + 2.f * b * f * r + a * r * r;
    const float M = c * f * f + 2.f * fabsf(b * f * r) + a * r * r;
    qmin = fminf(qmin, q - 1e-4f * M);
  }
  return qmin <= t;
}

// wave-wide sum with DPP row operations; the total is returned to every lane
#define SG_DPP(v, ctrl, rmask) \
  __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (v)), (ctrl), (rmask), 0xf, false))
SG_DEV float wave_sum_dpp(float v) {
  v += SG_DPP(v, 0xb1, 0xf);   // quad_perm [1,0,3,2]
  v += SG_DPP(v, 0x4e, 0xf);   // quad_perm [2,3,0,1]
  v += SG_DPP(v, 0x141, 0xf);  // row_half_mirror: sums of 8
  v += SG_DPP(v, 0x140, 0xf);  // row_mirror: sums of 16
  v += SG_DPP(v, 0x142, 0xa);  // row_bcast:15 into rows 1 and 3: sums of 32
  v += SG_DPP(v, 0x143, 0xc);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// wave-uniform (scalar) copy of a 64-bit value that every lane holds alike;
// both halves are zero-extended (the builtin returns a signed int)
SG_DEV uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// Sums of nine per-lane values over the wavefront, delivered one per lane:
// a transposed butterfly (lane halves swapped with v_permlane32_swap and
// v_permlane16_swap, then DPP row rotations and quad permutations), about a
// quarter of the instructions of nine separate reductions.  On return the
// total of value k sits in lane reduce9_lane(k): 0, 32, 16, 48, 8, 40, 24,
// 56, 4 for k = 0..8; other lanes hold duplicates or zeros.
SG_DEV float sg_swap_add32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
SG_DEV float sg_swap_add16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
#define SG_DPP_ALL(v, ctrl) \
  __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (v)), (ctrl), 0xf, 0xf, false))
SG_DEV float reduce9(const float v[9]) {
  const int lane = __lane_id();
  // distance 32: pairs of values share a register, one per 32-lane half
  float s0 = v[0], s1 = v[2], s2 = v[4], s3 = v[6], s4 = v[8];
  s0 = sg_swap_add32(s0, v[1]);
  s1 = sg_swap_add32(s1, v[3]);
  s2 = sg_swap_add32(s2, v[5]);
  s3 = sg_swap_add32(s3, v[7]);
  s4 = sg_swap_add32(s4, 0.f);
  // distance 16: four values per register, one per 16-lane row
  const float t0 = sg_swap_add16(s0, s1);
  const float t1 = sg_swap_add16(s2, s3);
  const float t2 = sg_swap_add16(s4, 0.f);
  // every cross-lane read below runs with all lanes active, before any
  // per-lane selection (a DPP read from a switched-off lane yields 0)
  // distance 8: two values per row (row_ror:8 pairs lanes l and l^8)
  const float e0 = SG_DPP_ALL(t0, 0x128), e1 = SG_DPP_ALL(t1, 0x128), e2 = SG_DPP_ALL(t2, 0x128);
  const float u0 = (lane & 8) ? t1 + e1 : t0 + e0;
  const float u1 = t2 + e2;
  // distance 4 within each group of 8 (row_ror:12 reads lane l+4, row_ror:4 lane l-4)
  const float f0 = SG_DPP_ALL(u0, 0x12C), f1 = SG_DPP_ALL(u1, 0x124);
  float w = (lane & 4) ? u1 + f1 : u0 + f0;
  // distances 2 and 1 within quads
  w += SG_DPP_ALL(w, 0x4e);  // quad_perm [2,3,0,1]
  w += SG_DPP_ALL(w, 0xb1);  // quad_perm [1,0,3,2]
  return w;
}
// value index held by `lane` after reduce9, or -1
SG_DEV int reduce9_index(int lane) {
  if (lane == 4) return 8;
  if (lane & 7) return -1;
  return ((lane >> 5) & 1) | (((lane >> 4) & 1) << 1) | (((lane >> 3) & 1) << 2);
}

// largest value over the wave
SG_DEV uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t o = (uint32_t)__shfl_xor((int)v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

}  // namespace sg
