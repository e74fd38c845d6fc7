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
#include "common.h"
#include "scan.h"

namespace sg {

// ---------------------------------------------------------------------------
// stable LSD radix sort of (u32 key, u32 value) pairs, count in device memory.
// The input is cut into kRsChunks contiguous chunks, one per wavefront; each
// wave ranks its elements with ballots (a wave-wide match on the digit) and
// keeps private per-digit cursors in LDS, so no block barrier is needed inside
// the scatter loop.

constexpr int kRsBlocks = 1024;
constexpr int kRsWaves = 4;
constexpr int kRsChunks = kRsBlocks * kRsWaves;
constexpr int kRsMaxBits = 10;

SG_DEV void rs_chunk(uint64_t count, int chunk_id, uint64_t& begin, uint64_t& end) {
  uint64_t per = (count + kRsChunks - 1) / kRsChunks;
  per = (per + 63) & ~uint64_t(63);
  begin = (uint64_t)chunk_id * per;
  end = begin + per;
  if (begin > count) begin = count;
  if (end > count) end = count;
}

__global__ void __launch_bounds__(256) k_rs_hist(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ d_count,
                                                 const uint64_t* __restrict__ d_cap, int shift, int bits,
                                                 uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kRsWaves][1 << kRsMaxBits];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int digits = 1 << bits;
  for (int d = lane; d < digits; d += 64) h[wave][d] = 0;
  uint64_t count = *d_count;
  if (d_cap && count > *d_cap) count = 0;
  const int chunk = blockIdx.x * kRsWaves + wave;
  uint64_t b, e;
  rs_chunk(count, chunk, b, e);
  const uint32_t mask = (uint32_t)digits - 1;
  for (uint64_t base = b; base < e; base += 64) {
    const uint64_t idx = base + lane;
    if (idx < e) atomicAdd(&h[wave][(keys[idx] >> shift) & mask], 1u);
  }
  for (int d = lane; d < digits; d += 64) hist[(size_t)d * kRsChunks + chunk] = h[wave][d];
}

__global__ void __launch_bounds__(256) k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                    const uint32_t* __restrict__ vals_in,
                                                    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                    const uint64_t* __restrict__ d_count,
                                                    const uint64_t* __restrict__ d_cap, int shift, int bits,
                                                    const uint32_t* __restrict__ hist_scanned) {
  __shared__ uint32_t cur[kRsWaves][1 << kRsMaxBits];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int digits = 1 << bits;
  const int chunk = blockIdx.x * kRsWaves + wave;
  for (int d = lane; d < digits; d += 64) cur[wave][d] = hist_scanned[(size_t)d * kRsChunks + chunk];
  uint64_t count = *d_count;
  if (d_cap && count > *d_cap) count = 0;
  uint64_t b, e;
  rs_chunk(count, chunk, b, e);
  const uint32_t mask = (uint32_t)digits - 1;
  const uint64_t lt = lanemask_lt();
  for (uint64_t base = b; base < e; base += 64) {
    const uint64_t idx = base + lane;
    const bool valid = idx < e;
    const uint32_t key = valid ? keys_in[idx] : 0u;
    const uint32_t val = valid ? vals_in[idx] : 0u;
    const uint32_t d = (key >> shift) & mask;
    uint64_t peers = ballot(valid);
    for (int k = 0; k < bits; ++k) {
      const bool bit = (d >> k) & 1u;
      const uint64_t m = ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t pos = cur[wave][d] + rank;
    if (valid) {
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    // the lowest lane of each digit group advances that digit's cursor; all
    // lanes have read their cursor above (LDS operations of one wave complete
    // in program order)
    if (valid && rank == 0) cur[wave][d] += (uint32_t)__popcll(peers);
  }
}

struct LoadU32 {
  const uint32_t* p;
  SG_DEV uint32_t operator()(int64_t i) const { return p[i]; }
};

// sorts (keys, vals) of `count` (device) elements on bits [0, total_bits),
// ping-ponging between buffer pair 0 = (k0, v0) and 1 = (k1, v1); the input is
// in pair `start`; returns the pair holding the result
static int radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int start,
                            const uint64_t* d_count, const uint64_t* d_cap, int total_bits, uint32_t* hist,
                            uint32_t* hist_partials, hipStream_t st, hipError_t& err) {
  const int npass = (total_bits + kRsMaxBits - 1) / kRsMaxBits;
  const int bits = (total_bits + npass - 1) / npass;
  int cur = start;
  int shift = 0;
  for (int p = 0; p < npass; ++p) {
    const int b = (shift + bits > total_bits) ? total_bits - shift : bits;
    uint32_t* kin = cur ? k1 : k0;
    uint32_t* vin = cur ? v1 : v0;
    uint32_t* kout = cur ? k0 : k1;
    uint32_t* vout = cur ? v0 : v1;
    hipLaunchKernelGGL(k_rs_hist, dim3(kRsBlocks), dim3(256), 0, st, kin, d_count, d_cap, shift, b, hist);
    const int64_t hn = (int64_t)(1 << b) * kRsChunks;
    err = exclusive_scan<LoadU32, uint32_t, uint32_t>(LoadU32{hist}, hn, hist, hist_partials, st);
    if (err != hipSuccess) return cur;
    hipLaunchKernelGGL(k_rs_scatter, dim3(kRsBlocks), dim3(256), 0, st, kin, vin, kout, vout, d_count, d_cap, shift,
                       b, hist);
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

__global__ void k_depth_keys(const steepgs_splat* __restrict__ splats, const uint32_t* __restrict__ tiles,
                             int64_t m, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  keys[r] = tiles[r] ? __float_as_uint(splats[r].depth) : 0xFFFFFFFFu;  // culled records sort last
  vals[r] = (uint32_t)r;
}

struct LoadTilesSorted {
  const uint32_t* tiles;
  const uint32_t* order;
  SG_DEV uint32_t operator()(int64_t s) const { return tiles[order[s]]; }
};

__global__ void k_instance_total(const uint64_t* __restrict__ total, uint64_t capacity,
                                 uint64_t* __restrict__ d_num, int32_t* __restrict__ d_status, uint64_t* cap_out) {
  const uint64_t K = *total;
  *d_num = K;
  *d_status = (K > capacity) ? (int32_t)STEEPGS_ERR_CAPACITY : (int32_t)STEEPGS_OK;
  *cap_out = capacity;
}

__global__ void __launch_bounds__(256) k_emit(const steepgs_splat* __restrict__ splats,
                                              const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ order,
                                              const uint64_t* __restrict__ offs, int64_t m, int64_t n,
                                              const steepgs_camera* __restrict__ cams,
                                              const uint64_t* __restrict__ d_num, uint64_t capacity,
                                              uint32_t* __restrict__ tkeys, uint32_t* __restrict__ ivals) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m || *d_num > capacity) return;
  const uint32_t r = order[s];
  const uint32_t cnt = tiles[r];
  if (cnt == 0) return;
  uint64_t o = offs[s];
  const steepgs_splat& sp = splats[r];
  const int x0 = sp.rect_lo & 0xFFFF, y0 = sp.rect_lo >> 16, x1 = sp.rect_hi & 0xFFFF, y1 = sp.rect_hi >> 16;
  const int v = (int)(r / (uint64_t)n);
  const uint32_t base = (uint32_t)cams[v].tile_offset;
  const uint32_t tx = (uint32_t)cams[v].tiles_x;
  for (int y = y0; y <= y1; ++y)
    for (int x = x0; x <= x1; ++x) {
      tkeys[o] = base + (uint32_t)y * tx + (uint32_t)x;
      ivals[o] = r;
      ++o;
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ tkeys, const uint64_t* __restrict__ d_num, uint64_t capacity,
                         uint32_t* __restrict__ ranges) {
  const uint64_t K = *d_num;
  if (K > capacity) return;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < K; s += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t t = tkeys[s];
    if (s == 0 || tkeys[s - 1] != t) ranges[2 * (size_t)t] = (uint32_t)s;
    if (s + 1 == K || tkeys[s + 1] != t) ranges[2 * (size_t)t + 1] = (uint32_t)(s + 1);
  }
}

__global__ void k_keys64(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ vals,
                         const steepgs_splat* __restrict__ splats, const uint64_t* __restrict__ d_num,
                         uint64_t capacity, uint64_t* __restrict__ keys) {
  const uint64_t K = *d_num;
  if (K > capacity) return;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < K; s += (uint64_t)gridDim.x * blockDim.x)
    keys[s] = ((uint64_t)tkeys[s] << 32) | (uint64_t)__float_as_uint(splats[vals[s]].depth);
}

struct SortWs {
  uint32_t *dkA, *dvA, *dkB, *dvB;
  uint64_t* offs;
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
  w.offs = c.take<uint64_t>(m);
  w.partials64 = c.take<uint64_t>(scan_partials_count(m) + 1);
  w.tkA = c.take<uint32_t>(cap);
  w.tkB = c.take<uint32_t>(cap);
  w.ivB = c.take<uint32_t>(cap);
  w.hist = c.take<uint32_t>((size_t)(1 << kRsMaxBits) * kRsChunks);
  w.hist_partials = c.take<uint32_t>(scan_partials_count((int64_t)(1 << kRsMaxBits) * kRsChunks) + 1);
  w.counters = c.take<uint64_t>(4);
  return c.used + 256;
}

size_t sort_workspace(int64_t m, uint64_t cap) {
  SortWs w;
  return sort_layout(nullptr, m, cap, w);
}

}  // namespace sg

using namespace sg;

extern "C" steepgs_status steepgs_sort(const steepgs_splat* d_splats, const uint32_t* d_tiles_touched, int64_t n,
                                       int32_t V, const steepgs_camera* d_cams, const steepgs_opts* opts,
                                       int32_t total_tiles, uint64_t* d_keys, uint32_t* d_vals, uint64_t capacity,
                                       uint32_t* d_tile_ranges, uint64_t* d_num_instances, int32_t* d_status,
                                       void* d_ws, size_t ws_bytes, void* stream) {
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
  if (!d_splats || !d_tiles_touched || (capacity > 0 && !d_vals)) return STEEPGS_ERR_INVALID_ARG;
  hipError_t err = hipSuccess;
  // 1. depth order of the records (culled last)
  hipLaunchKernelGGL(k_depth_keys, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, d_splats, d_tiles_touched, m,
                     w.dkA, w.dvA);
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, w.counters, (uint64_t)m);
  int where = radix_sort_pairs(w.dkA, w.dvA, w.dkB, w.dvB, 0, w.counters, nullptr, 32, w.hist, w.hist_partials, st,
                               err);
  if (err != hipSuccess) return STEEPGS_ERR_HIP;
  const uint32_t* order = where ? w.dvB : w.dvA;
  // 2. instance offsets in depth order; K and the capacity check
  err = exclusive_scan<LoadTilesSorted, uint64_t, uint64_t>(LoadTilesSorted{d_tiles_touched, order}, m, w.offs,
                                                           w.partials64, st);
  if (err != hipSuccess) return STEEPGS_ERR_HIP;
  uint64_t* total = w.partials64 + scan_partials_count(m);
  hipLaunchKernelGGL(k_instance_total, dim3(1), dim3(1), 0, st, total, capacity, d_num_instances, d_status,
                     w.counters + 1);
  // 3. emit instances (tile id, record) in depth order, then stable sort by tile
  int tile_bits = 1;
  while (tile_bits < 32 && ((uint64_t)1 << tile_bits) < (uint64_t)total_tiles) ++tile_bits;
  const int npass = (tile_bits + kRsMaxBits - 1) / kRsMaxBits;
  const int start = npass & 1;
  uint32_t* ek = start ? w.tkB : w.tkA;
  uint32_t* ev = start ? w.ivB : d_vals;
  if (capacity > 0) {
    hipLaunchKernelGGL(k_emit, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, d_splats, d_tiles_touched, order,
                       w.offs, m, n, d_cams, d_num_instances, capacity, ek, ev);
    int fin = radix_sort_pairs(w.tkA, d_vals, w.tkB, w.ivB, start, d_num_instances, w.counters + 1, tile_bits, w.hist,
                               w.hist_partials, st, err);
    if (err != hipSuccess) return STEEPGS_ERR_HIP;
    if (fin != 0) return STEEPGS_ERR_HIP;  // cannot happen: start chosen so the result lands in d_vals
    // 4. per-tile ranges and the optional 64-bit keys
    hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(256), 0, st, w.tkA, d_num_instances, capacity, d_tile_ranges);
    if (d_keys)
      hipLaunchKernelGGL(k_keys64, dim3(2048), dim3(256), 0, st, w.tkA, d_vals, d_splats, d_num_instances, capacity,
                         d_keys);
  }
  timer_end(STEEPGS_TIMER_SORT, st);
  SG_TRY_LAUNCH();
  return STEEPGS_OK;
}
