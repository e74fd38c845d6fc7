// Stage 2: the instance list of the tile rasterizer (Sec. 3, "Rasterization":
// Gaussians are sorted by view-dependent depth).
//
// Result: one instance per (visible record, covered tile), ordered by
// (global tile, depth, record id) -- the order of a stable sort of the 64-bit
// keys tile << 32 | depth bits emitted record by record, tiles row-major.
//
// Instead of a 49-bit radix sort over all K instances, the records are first
// sorted by depth (N_v elements, 32-bit keys), instances are then emitted in
// that order, and a stable radix sort on the tile id alone (ceil(log2 tiles)
// bits) groups them per tile: equal tiles keep the depth order, equal depths
// keep the record order.  Same output, far less traffic.
//
// All kernels read the instance count K from device memory, so the whole
// stage can be captured in a HIP graph.
#include "projection.h"
#include "rectwalk.h"
#include "scan.h"

namespace sg {

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (u32 key, u32 value) pairs; the element count is
// read from device memory.  A fixed grid of workgroups cuts the input
// into contiguous ranges; each workgroup walks its range in tiles of kRsTile
// elements.  Per tile, every wavefront ranks its contiguous 64 x kRsItems elements
// with ballots (a wave-wide match on the digit) against wave-private digit
// counters, the workgroup combines the counters into tile-local digit
// offsets, scatters the tile into LDS in sorted order and writes it out so
// that consecutive lanes write consecutive addresses of one digit's run.

// 16 wavefronts of 6 elements per lane: one workgroup fills a CU (4 waves
// per SIMD at <= 128 VGPRs, the next tile's elements in flight) and a tile of
// 6144 elements gives digit runs long enough for mostly whole-line writes.
// Sort stage on 59 M instances and 16 M records: 256 x 16 2.34 ms, 1024 x 8
// 2.22 ms; in a later run 1024 x 8 2.250 ms against 2.233 ms for 1024 x 6
// with the next tile loaded ahead (at 1024 x 8 that load spills: 2.79 ms).
#ifndef SG_RS_THREADS
#define SG_RS_THREADS 1024
#endif
constexpr int kRsThreads = SG_RS_THREADS;
constexpr int kRsWaves = kRsThreads / 64;
#ifndef SG_RS_ITEMS
#define SG_RS_ITEMS 6
#endif
constexpr int kRsItems = SG_RS_ITEMS;            // elements per lane per tile
constexpr int kRsTile = kRsThreads * kRsItems;   // elements per workgroup tile
constexpr int kRsWaveSpan = 64 * kRsItems;       // contiguous elements per wavefront
constexpr int kRsGrid = 1024;  // largest grid (sizes the digit-count table)
constexpr int kRsMaxBits = 9;


SG_DEV void rs_range(uint64_t count, uint64_t& begin, uint64_t& end) {
  const uint64_t G = gridDim.x;
  uint64_t per = (count + G - 1) / G;
  per = (per + kRsTile - 1) / kRsTile * kRsTile;
  begin = (uint64_t)blockIdx.x * per;
  end = begin + per;
  if (begin > count) begin = count;
  if (end > count) end = count;
}

SG_DEV uint64_t rs_count(const uint64_t* d_count, const uint64_t* d_cap) {
  uint64_t count = *d_count;
  if (d_cap && count > *d_cap) count = 0;
  return count;
}

template <int BITS>
__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const uint32_t* __restrict__ keys,
                                                        const uint64_t* __restrict__ d_count,
                                                        const uint64_t* __restrict__ d_cap, int shift, int bits,
                                                        uint32_t* __restrict__ hist) {
  constexpr int DIG = 1 << BITS;
  // several counter copies per wavefront (by lane), so that lanes holding
  // equal digits -- common in clustered keys -- rarely update one address;
  // each copy's row is one word longer than the digit count, so that equal
  // digits of different copies fall in different LDS banks
  constexpr int SUB = BITS <= 8 ? 8 : 4;
  constexpr int COPIES = kRsWaves * SUB;
  constexpr int ROW = DIG + 1;
  __shared__ uint32_t h[COPIES][ROW];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int copy = wave * SUB + (tid & (SUB - 1));
  for (int d = tid; d < COPIES * ROW; d += kRsThreads) (&h[0][0])[d] = 0u;
  __syncthreads();
  uint64_t b, e;
  rs_range(rs_count(d_count, d_cap), b, e);
  const uint32_t mask = (1u << bits) - 1u;
  for (uint64_t base = b; base < e; base += kRsTile) {
    // all of the tile's loads first, then the counter updates
    uint32_t k[kRsItems];
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
      const uint64_t i = base + (uint64_t)(it * kRsThreads + tid);
      k[it] = i < e ? keys[i] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kRsItems; ++it)
      if (base + (uint64_t)(it * kRsThreads + tid) < e) atomicAdd(&h[copy][(k[it] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = tid; d < DIG; d += kRsThreads) {
    uint32_t t = 0;
    for (int w = 0; w < COPIES; ++w) t += h[w][d];
    hist[(size_t)d * gridDim.x + blockIdx.x] = t;
  }
}

template <int BITS>
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out,
                                                           const uint64_t* __restrict__ d_count,
                                                           const uint64_t* __restrict__ d_cap, int shift, int bits,
                                                           const uint32_t* __restrict__ hist_scanned,
                                                           uint32_t* __restrict__ ranges) {
  constexpr int DIG = 1 << BITS;
  constexpr int PER = DIG / kRsThreads > 0 ? DIG / kRsThreads : 1;  // digits per thread in the tile scan
  __shared__ uint32_t s_key[kRsTile], s_val[kRsTile];
  __shared__ uint32_t s_wc[kRsWaves][DIG];  // per-wave digit counts, then offsets
  __shared__ uint32_t s_cnt[DIG], s_start[DIG], s_run[DIG];
  __shared__ uint32_t s_scan[kRsThreads / 64 + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t lt = lanemask_lt();
  for (int d = tid; d < DIG; d += kRsThreads) s_run[d] = hist_scanned[(size_t)d * gridDim.x + blockIdx.x];
  uint64_t b, e;
  rs_range(rs_count(d_count, d_cap), b, e);
  // a tile's keys and values, loaded while the previous tile is ranked and
  // written (one workgroup fills the CU, so nothing else would overlap them)
  uint32_t nk[kRsItems], nv[kRsItems];
  auto load_tile = [&](uint64_t base) {
    const int n_tile = (int)((e - base) < (uint64_t)kRsTile ? (e - base) : (uint64_t)kRsTile);
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
      const int idx = wave * kRsWaveSpan + it * 64 + lane;
      const bool valid = idx < n_tile;
      nk[it] = valid ? keys_in[base + idx] : 0u;
      // no value array: the values are the element indices
      nv[it] = valid ? (vals_in ? vals_in[base + idx] : (uint32_t)(base + idx)) : 0u;
    }
  };
  if (b < e) load_tile(b);
  for (uint64_t base = b; base < e; base += kRsTile) {
    const int n_tile = (int)((e - base) < (uint64_t)kRsTile ? (e - base) : (uint64_t)kRsTile);
    for (int d = lane; d < DIG; d += 64) s_wc[wave][d] = 0u;
    uint32_t k[kRsItems], v[kRsItems], rank[kRsItems];
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
      k[it] = nk[it];
      v[it] = nv[it];
    }
    if (base + kRsTile < e) load_tile(base + kRsTile);
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
      const int idx = wave * kRsWaveSpan + it * 64 + lane;
      const bool valid = idx < n_tile;
      const uint32_t d = (k[it] >> shift) & mask;
      uint64_t peers = ballot(valid);
      // digit bits at and above `bits` are zero (masked): their ballots agree
#pragma unroll
      for (int q = 0; q < BITS; ++q) {
        const bool bit = (d >> q) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t r = (uint32_t)__popcll(peers & lt);
      const uint32_t c = s_wc[wave][d];
      rank[it] = c + r;
      // the lowest lane of each digit group advances the wave's counter; all
      // lanes have read it above (LDS operations of one wave complete in order)
      if (valid && r == 0) s_wc[wave][d] = c + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // tile totals per digit and the wave offsets within a digit
    for (int d = tid; d < DIG; d += kRsThreads) {
      uint32_t sum = 0;
      for (int w = 0; w < kRsWaves; ++w) {
        const uint32_t t = s_wc[w][d];
        s_wc[w][d] = sum;
        sum += t;
      }
      s_cnt[d] = sum;
    }
    __syncthreads();
    // tile-local start of each digit's run
    {
      uint32_t loc[PER], tot = 0;
      for (int q = 0; q < PER; ++q) {
        const int d = tid * PER + q;
        loc[q] = d < DIG ? s_cnt[d] : 0u;
        tot += loc[q];
      }
      uint32_t all;
      uint32_t run = block_exclusive_scan<uint32_t, kRsThreads>(tot, s_scan, all);
      for (int q = 0; q < PER; ++q) {
        const int d = tid * PER + q;
        if (d < DIG) s_start[d] = run;
        run += loc[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
      const int idx = wave * kRsWaveSpan + it * 64 + lane;
      if (idx < n_tile) {
        const uint32_t d = (k[it] >> shift) & mask;
        const uint32_t pos = s_start[d] + s_wc[wave][d] + rank[it];
        s_key[pos] = k[it];
        s_val[pos] = v[it];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
      const int i = it * kRsThreads + tid;
      if (i < n_tile) {
        const uint32_t key = s_key[i];
        const uint32_t d = (key >> shift) & mask;
        const uint32_t g = s_run[d] + ((uint32_t)i - s_start[d]);
        if (keys_out) keys_out[g] = key;
        vals_out[g] = s_val[i];
        if (ranges) {
          // last pass: the key's [begin, end) from the boundaries of its run
          // in this tile; at the ends of a digit run the neighbour lies in
          // another tile, so every boundary is an atomic maximum (begin
          // stored complemented: the largest ~g is the smallest g)
          const uint32_t rs = s_start[d], re = rs + s_cnt[d];
          if ((uint32_t)i == rs || s_key[i - 1] != key) atomicMax(&ranges[2 * (size_t)key], ~g);
          if ((uint32_t)i + 1 == re || s_key[i + 1] != key) atomicMax(&ranges[2 * (size_t)key + 1], g + 1u);
        }
      }
    }
    __syncthreads();
    for (int d = tid; d < DIG; d += kRsThreads) s_run[d] += s_cnt[d];
    __syncthreads();
  }
}

struct LoadU32 {
  const uint32_t* p;
  SG_DEV uint32_t operator()(int64_t i) const { return p[i]; }
};

template <int BITS>
static void radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, const uint64_t* d_count,
                       const uint64_t* d_cap, uint64_t max_count, int shift, int b, uint32_t* hist,
                       uint32_t* hist_partials, hipStream_t st, hipError_t& err, uint32_t* ranges) {
  // as many workgroups as are resident together (LDS and registers), capped
  // at kRsGrid, so that no second partial round follows the first
  static int per_cu = 0;  // same code object on every device
  if (per_cu == 0) {
    int r = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, k_rs_scatter<BITS>, kRsThreads, 0) != hipSuccess || r < 1) r = 1;
    per_cu = r;
  }
  int grid = device_cu_count() * per_cu;
  if (grid > kRsGrid) grid = kRsGrid;
  // no more workgroups than tiles of the largest possible input (small
  // inputs: fewer histogram rows to clear and scan)
  const uint64_t tiles = (max_count + kRsTile - 1) / kRsTile;
  if ((uint64_t)grid > tiles) grid = tiles > 0 ? (int)tiles : 1;
  hipLaunchKernelGGL(k_rs_hist<BITS>, dim3(grid), dim3(kRsThreads), 0, st, kin, d_count, d_cap, shift, b, hist);
  const int64_t hn = (int64_t)(1 << BITS) * grid;
  err = exclusive_scan<LoadU32, uint32_t, uint32_t>(LoadU32{hist}, hn, hist, hist_partials, st);
  if (err != hipSuccess) return;
  hipLaunchKernelGGL(k_rs_scatter<BITS>, dim3(grid), dim3(kRsThreads), 0, st, kin, vin, kout, vout, d_count, d_cap,
                     shift, b, hist, ranges);
}

// sorts (keys, vals) of `count` (device) elements on bits [0, total_bits),
// ping-ponging between buffer pair 0 = (k0, v0) and 1 = (k1, v1); the input is
// in pair `start`; returns the pair holding the result.  With
// first_keys, the first pass reads its keys there (not from pair `start`)
// and takes the element indices as values.
static int radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int start,
                            const uint64_t* d_count, const uint64_t* d_cap, uint64_t max_count, int total_bits,
                            uint32_t* hist, uint32_t* hist_partials, hipStream_t st, hipError_t& err,
                            const uint32_t* first_keys = nullptr, uint32_t* ranges = nullptr,
                            bool last_keys = true) {
  const int npass = (total_bits + kRsMaxBits - 1) / kRsMaxBits;
  const int bits = (total_bits + npass - 1) / npass;
  int cur = start;
  int shift = 0;
  err = hipSuccess;
  for (int p = 0; p < npass; ++p) {
    const int b = (shift + bits > total_bits) ? total_bits - shift : bits;
    const uint32_t* kin = cur ? k1 : k0;
    const uint32_t* vin = cur ? v1 : v0;
    if (p == 0 && first_keys) {
      kin = first_keys;
      vin = nullptr;
    }
    uint32_t* kout = cur ? k0 : k1;
    uint32_t* vout = cur ? v0 : v1;
    // the last pass may record the key ranges and skip writing the keys
    const bool last = p + 1 == npass;
    uint32_t* rng = last ? ranges : nullptr;
    if (last && !last_keys) kout = nullptr;
    if (b <= 8)
      radix_pass<8>(kin, vin, kout, vout, d_count, d_cap, max_count, shift, b, hist, hist_partials, st, err, rng);
    else
      radix_pass<9>(kin, vin, kout, vout, d_count, d_cap, max_count, shift, b, hist, hist_partials, st, err, rng);
    if (err != hipSuccess) return cur;
    cur ^= 1;
    shift += b;
  }
  err = hipGetLastError();
  return cur;
}

// ---------------------------------------------------------------------------
// instance pipeline

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void k_set_u64(uint64_t* __restrict__ p, uint64_t v) { *p = v; }

// ---------------------------------------------------------------------------
// Instance emission in depth order, walking every tile rectangle once.
//
// k_walk: each wavefront takes a chunk of 64 consecutive records of the depth
// order, walks their tile rectangles together (rect_walk_begin /
// rect_walk_locate), tests every tile against the footprint ellipse and
// keeps the hit ballots of the first kWalkKeep walk steps in global memory,
// with each record's walk rectangle (contiguous, in depth order) and the
// chunk's hit count.  An exclusive scan of the chunk counts gives each
// chunk's output offset.  k_emit replays the walk from the kept ballots and
// rectangles -- no gather of the projected records, no second ellipse test
// (steps beyond the kept ones are tested again) -- and writes the instances
// (global tile id, record id) from the chunk's offset.

constexpr int kWalkKeep = 16;  // ballots kept per chunk: 1024 rectangle positions

struct WalkRect {
  uint32_t xy0;  // x0 | y0 << 16
  uint32_t wh;   // width | height << 16 (0: nothing to walk)
};

SG_DEV void walk_record(const steepgs_splat* __restrict__ splats, const steepgs_camera* __restrict__ cams,
                        int64_t n, uint32_t r, const steepgs_opts& opt, RectRec& me, uint32_t& area) {
  area = walk_rect(splats[r], opt, me);
  const int v = (int)(r / (uint64_t)n);
  me.tag0 = r;
  me.tag1 = (uint32_t)cams[v].tile_offset;
  me.pad0 = (uint32_t)cams[v].tiles_x;
}

// One lane's input of the walk: the depth key and record id at its position
// of the depth order, and the record's first 32 bytes (mean, conic, opacity,
// tile rectangle).  Loaded two chunks (order) and one chunk (record) ahead.
struct WalkIn {
  uint32_t key, r;
  float4 lo, hi;  // (mean_x, mean_y, conic_a, conic_b), (conic_c, opacity, rect_lo, rect_hi)
};

SG_DEV void walk_in_order(const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ order, int64_t m,
                          int64_t c, int lane, WalkIn& w) {
  // both loads unconditional (no wait on the key before the order load)
  const int64_t s = c * 64 + lane;
  w.key = 0xFFFFFFFFu;
  w.r = 0xFFFFFFFFu;
  if (s < m) {
    w.key = skeys[s];
    w.r = order[s];
  }
}

SG_DEV void walk_in_record(const steepgs_splat* __restrict__ splats, WalkIn& w) {
  if (w.key != 0xFFFFFFFFu) {
    const float4* p = reinterpret_cast<const float4*>(splats + w.r);
    w.lo = p[0];
    w.hi = p[1];
  }
}

// occupancy hints (waves per SIMD) of the walk and the emission.  Measured
// on 59 M instances (sort stage): emission at 8 (a 24-byte spill) 2.169 ms
// against 2.195 at 6 and 2.193 at 7; the walk at 7 (spills) is slower.
#ifndef SG_WALK_WAVES_PER_EU
#define SG_WALK_WAVES_PER_EU 6
#endif
#ifndef SG_EMIT_WAVES_PER_EU
#define SG_EMIT_WAVES_PER_EU 8
#endif

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SG_WALK_WAVES_PER_EU))) k_walk(const steepgs_splat* __restrict__ splats,
                                              const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ order,
                                              int64_t m, int64_t n, const steepgs_camera* __restrict__ cams,
                                              steepgs_opts opt, WalkRect* __restrict__ rects,
                                              uint64_t* __restrict__ kept, uint32_t* __restrict__ chunk_hits,
                                              uint32_t* __restrict__ counts) {
  __shared__ RectWalkLds s_walk[4];
  __shared__ uint32_t s_cnt[256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  RectWalkLds& L = s_walk[wave];
  uint32_t* const cnt = s_cnt + wave * 64;
  const int64_t nchunks = (m + 63) / 64;
  const int64_t stride = (int64_t)gridDim.x * 4;
  // the chunk's records gathered while the previous chunk walks, its depth
  // order positions one chunk earlier still
  WalkIn cur = {}, nxt = {};
  int64_t c = (int64_t)blockIdx.x * 4 + wave;
  walk_in_order(skeys, order, m, c, lane, cur);
  walk_in_record(splats, cur);
  walk_in_order(skeys, order, m, c + stride, lane, nxt);
  for (; c < nchunks; c += stride) {
    const WalkIn w = cur;
    const int64_t s = c * 64 + lane;
    uint32_t area = 0;
    const uint32_t r = w.r;
    RectRec me = {};
    me.wdt = 1;
    me.a = me.c = 1.f;
    if (w.key != 0xFFFFFFFFu) {  // culled records sort last
      steepgs_splat sp;
      sp.mean_x = w.lo.x;
      sp.mean_y = w.lo.y;
      sp.conic_a = w.lo.z;
      sp.conic_b = w.lo.w;
      sp.conic_c = w.hi.x;
      sp.opacity = w.hi.y;
      sp.rect_lo = __float_as_uint(w.hi.z);
      sp.rect_hi = __float_as_uint(w.hi.w);
      area = walk_rect(sp, opt, me);
      const int v = (int)(r / (uint64_t)n);
      me.tag0 = r;
      me.tag1 = (uint32_t)cams[v].tile_offset;
      me.pad0 = (uint32_t)cams[v].tiles_x;
    }
    uint32_t aoff;
    const uint32_t atotal = rect_walk_begin(L, lane, area, me, aoff);
    // the next chunks' loads go out after this chunk's last one (the camera
    // fields above), so that no wait on this chunk's data waits on them
    cur = nxt;
    walk_in_record(splats, cur);
    walk_in_order(skeys, order, m, c + 2 * stride, lane, nxt);
    if (s < m) rects[s] = WalkRect{me.xy0, area ? (me.wdt | ((area / me.wdt) << 16)) : 0u};
    cnt[lane] = 0u;
    uint32_t hits = 0;
    uint64_t mine = 0;  // lane k keeps the ballot of step k
    int carry = 0;
    uint32_t k = 0;
    for (uint32_t j0 = 0; j0 < atotal; j0 += 64, ++k) {
      int tx, ty;
      const int owner = rect_walk_locate(L, lane, area, aoff, j0, carry, tx, ty);
      const RectRec R = L.get(owner);
      const bool hit = j0 + (uint32_t)lane < atotal && tile_hit_rcp(R.mx, R.my, R.a, R.b, R.c, R.ia, R.ic, opt, tx, ty);
      const uint64_t b = ballot(hit);
      if ((uint32_t)lane == k) mine = b;
      hits += (uint32_t)__popcll(b);
      if (counts && hit) atomicAdd(&cnt[owner], 1u);
      __builtin_amdgcn_wave_barrier();
    }
    if ((uint32_t)lane < k && lane < kWalkKeep) kept[c * kWalkKeep + lane] = mine;
    if (lane == 0) chunk_hits[c] = hits;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (counts && s < m) counts[r] = cnt[lane];
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SG_EMIT_WAVES_PER_EU))) k_emit(const steepgs_splat* __restrict__ splats,
                                              const uint32_t* __restrict__ order, const WalkRect* __restrict__ rects,
                                              const uint64_t* __restrict__ kept,
                                              const uint64_t* __restrict__ chunk_off, int64_t m, int64_t n,
                                              const steepgs_camera* __restrict__ cams, steepgs_opts opt,
                                              const uint64_t* __restrict__ d_num, uint64_t capacity,
                                              uint32_t* __restrict__ tkeys, uint32_t* __restrict__ ivals) {
  __shared__ RectWalkLds s_walk[4];
  if (*d_num > capacity) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  RectWalkLds& L = s_walk[wave];
  const uint64_t lt = lanemask_lt();
  const int64_t nchunks = (m + 63) / 64;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wave; c < nchunks; c += (int64_t)gridDim.x * 4) {
    const int64_t s = c * 64 + lane;
    const WalkRect wr = s < m ? rects[s] : WalkRect{0u, 0u};
    uint32_t area = (wr.wh & 0xFFFFu) * (wr.wh >> 16);
    const uint32_t r = area ? order[s] : 0u;
    RectRec me = {};
    me.a = me.c = 1.f;
    me.xy0 = wr.xy0;
    me.wdt = area ? (wr.wh & 0xFFFFu) : 1u;
    if (area) {
      const int v = (int)(r / (uint64_t)n);
      me.tag0 = r;
      me.tag1 = (uint32_t)cams[v].tile_offset;
      me.pad0 = (uint32_t)cams[v].tiles_x;
    }
    // total area beyond the kept ballots: those steps test their tiles again,
    // which needs the records' conics
    uint32_t incl = area;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t t = __shfl_up(incl, d, 64);
      if (lane >= d) incl += t;
    }
    const bool retest = __shfl(incl, 63, 64) > 64u * kWalkKeep;
    if (retest && area) {
      uint32_t a2;
      walk_record(splats, cams, n, r, opt, me, a2);
    }
    uint32_t aoff;
    const uint32_t atotal = rect_walk_begin(L, lane, area, me, aoff);
    const uint64_t mine = lane < kWalkKeep ? kept[c * kWalkKeep + lane] : 0ull;
    uint64_t cursor = chunk_off[c];
    int carry = 0;
    uint32_t k = 0;
    for (uint32_t j0 = 0; j0 < atotal; j0 += 64, ++k) {
      int tx, ty;
      const int owner = rect_walk_locate(L, lane, area, aoff, j0, carry, tx, ty);
      const RectRec R = L.get(owner);
      uint64_t b;
      if (k < (uint32_t)kWalkKeep) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine, (int)k);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mine >> 32), (int)k);
        b = ((uint64_t)hi << 32) | lo;
      } else {
        b = ballot(j0 + (uint32_t)lane < atotal && tile_hit_rcp(R.mx, R.my, R.a, R.b, R.c, R.ia, R.ic, opt, tx, ty));
      }
      if ((b >> lane) & 1ull) {
        const uint64_t o = cursor + (uint64_t)__popcll(b & lt);
        tkeys[o] = R.tag1 + (uint32_t)ty * R.pad0 + (uint32_t)tx;
        ivals[o] = R.tag0;
      }
      cursor += (uint64_t)__popcll(b);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

__global__ void k_instance_total(const uint64_t* __restrict__ total, uint64_t capacity,
                                 uint64_t* __restrict__ d_num, int32_t* __restrict__ d_status) {
  const uint64_t K = *total;
  *d_num = K;
  *d_status = (K > capacity) ? (int32_t)STEEPGS_ERR_CAPACITY : (int32_t)STEEPGS_OK;
}

// per-tile [begin, end) of the sorted list: the last tile pass leaves
// (~begin, end) for every tile it saw (~begin >= 1, as begin < 2^32 - 1) and
// the zero fill (0, 0) for the others
__global__ void k_ranges_fix(uint32_t* __restrict__ ranges, int64_t tiles) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tiles) {
    const uint32_t b = ranges[2 * t];
    ranges[2 * t] = b ? ~b : 0u;
  }
}

__global__ void k_keys64(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ vals,
                         const uint32_t* __restrict__ dkeys, const uint64_t* __restrict__ d_num,
                         uint64_t capacity, uint64_t* __restrict__ keys) {
  const uint64_t K = *d_num;
  if (K > capacity) return;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < K; s += (uint64_t)gridDim.x * blockDim.x)
    keys[s] = ((uint64_t)tkeys[s] << 32) | (uint64_t)dkeys[vals[s]];
}

struct SortWs {
  uint32_t *dkA, *dvA, *dkB, *dvB;
  WalkRect* rects;        // walk rectangle per record, depth order
  uint64_t* kept;         // kept hit ballots per chunk
  uint32_t* chunk_hits;   // instances per chunk of 64 records
  uint64_t* chunk_off;    // their exclusive scan
  uint64_t* partials64;
  uint32_t *tkA, *tkB, *ivB;
  uint32_t* hist;
  uint32_t* hist_partials;
  uint64_t* counters;  // [0] record count, [1] capacity
};

static size_t sort_layout(void* base, int64_t m, uint64_t cap, SortWs& w) {
  Carver c(base);
  w.dkA = c.take<uint32_t>(m);
  w.dvA = c.take<uint32_t>(m);
  w.dkB = c.take<uint32_t>(m);
  w.dvB = c.take<uint32_t>(m);
  const int64_t nchunks = ceil_div(m, 64);
  w.rects = c.take<WalkRect>(m);
  w.kept = c.take<uint64_t>((size_t)nchunks * kWalkKeep);
  w.chunk_hits = c.take<uint32_t>(nchunks);
  w.chunk_off = c.take<uint64_t>(nchunks);
  w.partials64 = c.take<uint64_t>(scan_partials_count(nchunks) + 1);
  w.tkA = c.take<uint32_t>(cap);
  w.tkB = c.take<uint32_t>(cap);
  w.ivB = c.take<uint32_t>(cap);
  w.hist = c.take<uint32_t>((size_t)(1 << kRsMaxBits) * kRsGrid);
  w.hist_partials = c.take<uint32_t>(scan_partials_count((int64_t)(1 << kRsMaxBits) * kRsGrid) + 1);
  w.counters = c.take<uint64_t>(4);
  return c.used + 256;
}

size_t sort_workspace(int64_t m, uint64_t cap) {
  SortWs w;
  return sort_layout(nullptr, m, cap, w);
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_sort(const steepgs_splat* d_splats, const uint32_t* d_tiles_touched,
                                       const uint32_t* d_depth_keys, int64_t n,
                                       int32_t V, const steepgs_camera* d_cams, const steepgs_opts* opts,
                                       int32_t total_tiles, uint64_t* d_keys, uint32_t* d_vals, uint64_t capacity,
                                       uint32_t* d_tile_ranges, uint32_t* d_counts, uint64_t* d_num_instances,
                                       int32_t* d_status, void* d_ws, size_t ws_bytes, void* stream) {
  if (n < 0 || V <= 0 || total_tiles <= 0 || !opts) return STEEPGS_ERR_INVALID_ARG;
  if (!d_tile_ranges || !d_num_instances || !d_status || !d_cams) return STEEPGS_ERR_INVALID_ARG;
  if (capacity > 0xFFFFFFFFull) return STEEPGS_ERR_INVALID_ARG;
  const int64_t m = (int64_t)V * n;
  hipStream_t st = as_stream(stream);
  SortWs w;
  const size_t need = sort_layout(nullptr, m, capacity, w);
  if (!d_ws || ws_bytes < need) return STEEPGS_ERR_WORKSPACE;
  sort_layout(d_ws, m, capacity, w);
  timer_begin(STEEPGS_TIMER_SORT, st);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)ceil_div(2 * (int64_t)total_tiles, 256)), dim3(256), 0, st,
                     d_tile_ranges, 0u, 2 * (int64_t)total_tiles);
  if (m == 0) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, d_num_instances, (uint64_t)0);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, reinterpret_cast<uint32_t*>(d_status), 0u, (int64_t)1);
    timer_end(STEEPGS_TIMER_SORT, st);
    SG_TRY_LAUNCH();
    return STEEPGS_OK;
  }
  if (!d_splats || !d_tiles_touched || !d_depth_keys || (capacity > 0 && !d_vals)) return STEEPGS_ERR_INVALID_ARG;
  hipError_t err = hipSuccess;
  // 1. depth order of the records (culled last), on the projection's keys
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, w.counters, (uint64_t)m);
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, w.counters + 1, (uint64_t)capacity);
  const int where = radix_sort_pairs(w.dkA, w.dvA, w.dkB, w.dvB, 0, w.counters, nullptr, (uint64_t)m, 32, w.hist,
                                     w.hist_partials, st, err, d_depth_keys);
  if (err != hipSuccess) return STEEPGS_ERR_HIP;
  const uint32_t* order = where ? w.dvB : w.dvA;
  const uint32_t* skeys = where ? w.dkB : w.dkA;
  // 2. walk the tile rectangles in depth order (hits per chunk of 64
  // records, optional exact counts), offsets of the chunks, K and the
  // capacity check, then the instances (tile id, record) in depth order
  int tile_bits = 1;
  while (tile_bits < 32 && ((uint64_t)1 << tile_bits) < (uint64_t)total_tiles) ++tile_bits;
  const int npass = (tile_bits + kRsMaxBits - 1) / kRsMaxBits;
  const int start = npass & 1;
  uint32_t* ek = start ? w.tkB : w.tkA;
  uint32_t* ev = start ? w.ivB : d_vals;
  const int64_t nchunks = ceil_div(m, 64);
  const int egrid = (int)std::min<int64_t>(ceil_div(nchunks, 4), (int64_t)device_cu_count() * 16);
  hipLaunchKernelGGL(k_walk, dim3(egrid), dim3(256), 0, st, d_splats, skeys, order, m, n, d_cams, *opts, w.rects,
                     w.kept, w.chunk_hits, d_counts);
  err = exclusive_scan<LoadU32, uint64_t, uint64_t>(LoadU32{w.chunk_hits}, nchunks, w.chunk_off, w.partials64, st);
  if (err != hipSuccess) return STEEPGS_ERR_HIP;
  hipLaunchKernelGGL(k_instance_total, dim3(1), dim3(1), 0, st, w.partials64 + scan_partials_count(nchunks), capacity,
                     d_num_instances, d_status);
  if (capacity > 0)
    hipLaunchKernelGGL(k_emit, dim3(egrid), dim3(256), 0, st, d_splats, order, w.rects, w.kept, w.chunk_off, m, n,
                       d_cams, *opts, d_num_instances, capacity, ek, ev);
  if (capacity > 0) {
    // 3. stable sort by tile (equal tiles keep the depth order)
    // (the last pass records each tile's range; the sorted tile ids are
    // written only for the optional 64-bit keys)
    int fin = radix_sort_pairs(w.tkA, d_vals, w.tkB, w.ivB, start, d_num_instances, w.counters + 1, capacity,
                               tile_bits, w.hist, w.hist_partials, st, err, nullptr, d_tile_ranges, d_keys != nullptr);
    if (err != hipSuccess) return STEEPGS_ERR_HIP;
    if (fin != 0) return STEEPGS_ERR_HIP;  // cannot happen: start chosen so the result lands in d_vals
    // 4. per-tile ranges from the last pass's (~begin, end), and the optional 64-bit keys
    hipLaunchKernelGGL(k_ranges_fix, dim3((unsigned)ceil_div((int64_t)total_tiles, 256)), dim3(256), 0, st,
                       d_tile_ranges, (int64_t)total_tiles);
    if (d_keys)
      hipLaunchKernelGGL(k_keys64, dim3(2048), dim3(256), 0, st, w.tkA, d_vals, d_depth_keys, d_num_instances, capacity,
                         d_keys);
  }
  timer_end(STEEPGS_TIMER_SORT, st);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
