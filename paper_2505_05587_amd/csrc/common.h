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
  return tile_ok && o->radius_sigmas > 0.f && o->alpha_max > 0.f && o->alpha_max <= 1.f && o->alpha_min >= 0.f &&
         o->t_min >= 0.f && o->t_min < 1.f && o->near_z > 0.f && o->dilation >= 0.f;
}

// compute units of the current device (cached per device id)
int device_cu_count();

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
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
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

// ---------------------------------------------------------------------------
// Per-pixel opacity of a projected Gaussian (Eq. sigma_2D):
//   alpha = min(alpha_max, o * exp(-1/2 d^T A d)),  d = x - mean.
// The forward and backward raster kernels evaluate it with this one routine
// so that both see bit-identical values.
struct SplatLDS {
  float mx, my, ca, cb, cc, o;
};

SG_DEV float splat_power(float dx, float dy, float a, float b, float c) {
  return -0.5f * (a * dx * dx + c * dy * dy) - b * dx * dy;
}

}  // namespace sg
