// Device-wide exclusive prefix sum (reduce, scan partials, scan) used by the
// instance sort and by densification.  Sizes are host-known; nothing here
// reads a device count.
#pragma once

#include "common.h"

namespace sg {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // elements per block

// exclusive scan over the 256 threads of a block; returns the block total
template <class T, int kThreads = kScanThreads>
SG_DEV T block_exclusive_scan(T x, T* lds /*[kThreads/64 + 1]*/, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T inc = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  T wave_off = 0, tot = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) wave_off += lds[w];
    tot += lds[w];
  }
  __syncthreads();
  total = tot;
  return wave_off + inc - x;
}

template <class Load, class Acc>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(Load in, int64_t N, Acc* __restrict__ partials) {
  __shared__ Acc lds[kScanThreads / 64 + 1];
  // only the block's total is needed: strided (coalesced) reads, any order
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  Acc s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads;
    if (i < N) s += (Acc)in(i);
  }
  Acc total;
  block_exclusive_scan<Acc>(s, lds, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// single block: in-place exclusive scan of `count` partials; grand total to *total_out
template <class Acc>
__global__ void __launch_bounds__(kScanThreads) k_scan_partials(Acc* __restrict__ partials, int64_t count,
                                                                  Acc* __restrict__ total_out) {
  __shared__ Acc lds[kScanThreads / 64 + 1];
  const int64_t per = (count + kScanThreads - 1) / kScanThreads;
  const int64_t b = (int64_t)threadIdx.x * per;
  Acc s = 0;
  for (int64_t k = 0; k < per; ++k)
    if (b + k < count) s += partials[b + k];
  Acc total;
  Acc run = block_exclusive_scan<Acc>(s, lds, total);
  for (int64_t k = 0; k < per; ++k)
    if (b + k < count) {
      Acc x = partials[b + k];
      partials[b + k] = run;
      run += x;
    }
  if (threadIdx.x == 0 && total_out) *total_out = total;
}

// Each wavefront scans a contiguous quarter of the block's elements in rounds
// of 64 consecutive elements (coalesced loads and stores), carrying the
// running sum from round to round; the block's partial and the totals of the
// wavefronts before it give the starting offset.
template <class Load, class Acc, class Out>
__global__ void __launch_bounds__(kScanThreads) k_scan_final(Load in, int64_t N, const Acc* __restrict__ partials,
                                                               Out* __restrict__ out) {
  constexpr int kWaves = kScanThreads / 64;
  __shared__ Acc lds[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)wave * (kScanTile / kWaves) + lane;
  Acc v[kScanItems];
  Acc s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * 64;
    v[k] = i < N ? (Acc)in(i) : Acc(0);
    s += v[k];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) lds[wave] = s;
  __syncthreads();
  Acc carry = partials[blockIdx.x];
  for (int w = 0; w < wave; ++w) carry += lds[w];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    Acc inc = v[k];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const Acc y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    const int64_t i = base + (int64_t)k * 64;
    if (i < N) out[i] = (Out)(carry + inc - v[k]);
    carry += __shfl(inc, 63, 64);
  }
}

inline size_t scan_partials_count(int64_t N) { return (size_t)ceil_div(N > 0 ? N : 1, kScanTile); }

// Enqueue an exclusive scan of N elements read through `in` into `out`;
// `partials` holds scan_partials_count(N) + 1 accumulators; the grand total
// is left in partials[scan_partials_count(N)].
template <class Load, class Acc, class Out>
hipError_t exclusive_scan(Load in, int64_t N, Out* out, Acc* partials, hipStream_t st) {
  const int64_t nb = (int64_t)scan_partials_count(N);
  hipLaunchKernelGGL((k_scan_reduce<Load, Acc>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, N, partials);
  hipLaunchKernelGGL((k_scan_partials<Acc>), dim3(1), dim3(kScanThreads), 0, st, partials, nb, partials + nb);
  hipLaunchKernelGGL((k_scan_final<Load, Acc, Out>), dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, N, partials,
                     out);
  return hipGetLastError();
}

}  // namespace sg
