// sort.hip - group the hits of a batch by material so that every wave runs a
// single program (tile histograms -> scan in longest-program-first order ->
// tile scatter).  Hits whose material id is out of range go to the last bucket.
#include "device_common.h"
#include "shade.h"

namespace pmc {

constexpr uint32_t kSortBatch = 8;    // material ids loaded per thread before they are used
constexpr uint32_t kSortThreads = 1024;  // threads per tile (block)

// Counting sort over tiles: tile k (a block) histograms its hits in LDS and
// adds its non-zero bucket counts to the global counts of the buckets (a few
// dozen atomics per tile: a tile covers a few screen regions, so few
// materials); one block scans the counts (buckets ranked by decreasing
// program length, invalid ids last, so longer programs come first in the
// permutation); each tile then histograms again, reserves its ranges in the
// buckets with one atomic per non-zero bucket, and scatters its hits, ranking
// them in LDS.  The order of hits within a bucket carries no meaning.
__device__ __forceinline__ void tile_histogram(const uint32_t* material, uint32_t beg,
                                               uint32_t end, uint32_t n_mats, uint32_t* hist) {
  for (uint32_t g0 = beg; g0 < end; g0 += kSortBatch * kSortThreads) {
    uint32_t bb[kSortBatch];
#pragma unroll
    for (uint32_t k = 0; k < kSortBatch; ++k) {     // all loads of the batch in flight at once
      const uint32_t i = g0 + k * kSortThreads + threadIdx.x;
      const uint32_t m = i < end ? material[i] : 0xFFFFFFFFu;
      bb[k] = i < end ? (m < n_mats ? m : n_mats) : 0xFFFFFFFFu;
    }
#pragma unroll
    for (uint32_t k = 0; k < kSortBatch; ++k) {
      const uint32_t b = bb[k];
      const bool valid = b != 0xFFFFFFFFu;
      uint64_t act = __ballot(valid);
      while (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t bl = __builtin_amdgcn_readlane(b, leader);
        const uint64_t match = __ballot(valid && b == bl);
        if (lane_id() == leader) atomicAdd(&hist[bl], (uint32_t)__popcll(match));
        act &= ~match;
      }
    }
  }
}

__global__ __launch_bounds__(kSortThreads) void k_tile_hist(const uint32_t* material, uint32_t n,
                                                   uint32_t n_mats, uint32_t tile,
                                                   const uint32_t* rank, uint32_t* counts) {
  extern __shared__ uint32_t hist[];
  const uint32_t nb = n_mats + 1;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0u;
  __syncthreads();
  const uint32_t beg = blockIdx.x * tile;
  tile_histogram(material, beg, min(beg + tile, n), n_mats, hist);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    const uint32_t c = hist[b];
    if (c) atomicAdd(&counts[b < n_mats ? rank[b] : n_mats], c);
  }
}

__global__ __launch_bounds__(kSortThreads) void k_tile_scatter(const uint32_t* material, uint32_t n,
                                                      uint32_t n_mats, uint32_t tile,
                                                      const uint32_t* rank, uint32_t* cursor,
                                                      uint32_t* perm) {
  extern __shared__ uint32_t base[];
  const uint32_t nb = n_mats + 1;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) base[b] = 0u;
  __syncthreads();
  const uint32_t beg = blockIdx.x * tile;
  const uint32_t end = min(beg + tile, n);
  tile_histogram(material, beg, end, n_mats, base);
  __syncthreads();
  // this tile's range in each of its buckets (the bucket cursors start at the
  // buckets' first positions)
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    const uint32_t c = base[b];
    if (c) base[b] = atomicAdd(&cursor[b < n_mats ? rank[b] : n_mats], c);
  }
  __syncthreads();
  for (uint32_t g0 = beg; g0 < end; g0 += kSortBatch * kSortThreads) {
    uint32_t bb[kSortBatch];
#pragma unroll
    for (uint32_t k = 0; k < kSortBatch; ++k) {
      const uint32_t i = g0 + k * kSortThreads + threadIdx.x;
      const uint32_t m = i < end ? material[i] : 0xFFFFFFFFu;
      bb[k] = i < end ? (m < n_mats ? m : n_mats) : 0xFFFFFFFFu;
    }
#pragma unroll
    for (uint32_t k = 0; k < kSortBatch; ++k) {
      const uint32_t i = g0 + k * kSortThreads + threadIdx.x;
      const uint32_t b = bb[k];
      const bool valid = b != 0xFFFFFFFFu;
      uint64_t act = __ballot(valid);
      while (act) {
        const int leader = __ffsll((unsigned long long)act) - 1;
        const uint32_t bl = __builtin_amdgcn_readlane(b, leader);
        const uint64_t match = __ballot(valid && b == bl);
        uint32_t old = 0;
        if (lane_id() == leader) old = atomicAdd(&base[bl], (uint32_t)__popcll(match));
        old = __shfl(old, leader, 64);
        if (valid && b == bl) perm[old + (uint32_t)__popcll(match & lanemask_lt())] = i;
        act &= ~match;
      }
    }
  }
}

// Exclusive scan of a small count matrix by one block: the matrix is loaded
// into LDS with coalesced reads, each thread scans a contiguous segment, a
// block-wide scan of the segment totals gives their offsets, and the result
// goes back with coalesced writes.  Also clears reset[0 .. n_reset).
constexpr uint32_t kSmallScanMax = 36864;            // 144 KiB of LDS
constexpr uint32_t kSmallScanThreads = 1024;

__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t* in, uint32_t n,
                                                     uint32_t* out, uint32_t* reset,
                                                     uint32_t n_reset) {
  extern __shared__ uint32_t buf[];
  __shared__ uint32_t wsum[kSmallScanThreads / 64];
  const uint32_t t = threadIdx.x;
#pragma unroll 8
  for (uint32_t i = t; i < n; i += kSmallScanThreads) buf[i] = in[i];
  if (t < n_reset) reset[t] = 0u;
  __syncthreads();
  const uint32_t per = (n + kSmallScanThreads - 1) / kSmallScanThreads;
  const uint32_t beg = min(t * per, n), end = min(beg + per, n);
  uint32_t s = 0;
  for (uint32_t i = beg; i < end; ++i) s += buf[i];
  // block exclusive scan of s: inclusive scan within the wave, then over wave totals
  uint32_t x = s;
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[t >> 6] = x;
  __syncthreads();
  if (t < 64) {
    uint32_t w = t < kSmallScanThreads / 64 ? wsum[t] : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (t < kSmallScanThreads / 64) wsum[t] = w;
  }
  __syncthreads();
  uint32_t run = x - s + ((t >> 6) ? wsum[(t >> 6) - 1] : 0u);
  for (uint32_t i = beg; i < end; ++i) {
    const uint32_t v = buf[i];
    buf[i] = run;
    run += v;
  }
  __syncthreads();
#pragma unroll 8
  for (uint32_t i = t; i < n; i += kSmallScanThreads) out[i] = buf[i];
}

hipError_t prepare_sort_kernels() {
  return hipFuncSetAttribute((const void*)k_scan_small,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kSmallScanMax * 4);
}

// Tiles of 8192 hits: the per-tile work (clearing and reading the LDS
// histogram, a few atomics) is small against its 8192 ids, and 8.3 M hits give
// about a thousand blocks.
constexpr uint32_t kSortTile = 8192;

hipError_t launch_material_sort_tiled(const uint32_t* material, uint32_t n, uint32_t n_mats,
                                      const uint32_t* rank, uint32_t* mat_counts,
                                      uint32_t* offsets, uint32_t* scan_sums, uint32_t* perm,
                                      uint32_t* reset, uint32_t n_reset, hipStream_t s) {
  (void)scan_sums;
  const uint32_t nb = n_mats + 1;
  if (nb > kSmallScanMax || n_reset > kSmallScanThreads) return hipErrorInvalidValue;
  const uint32_t n_tiles = (n + kSortTile - 1) / kSortTile;
  const size_t lds = (size_t)nb * sizeof(uint32_t);
  hipError_t e = launch_fill_u32(mat_counts, 0u, nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_hist, dim3(n_tiles), dim3(kSortThreads), lds, s, material, n, n_mats,
                     kSortTile, rank, mat_counts);
  // bucket starts -> offsets (the cursors the scatter advances); also clears reset[]
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kSmallScanThreads), (size_t)nb * 4, s,
                     mat_counts, nb, offsets, reset, n_reset);
  hipLaunchKernelGGL(k_tile_scatter, dim3(n_tiles), dim3(kSortThreads), lds, s, material, n,
                     n_mats, kSortTile, rank, offsets, perm);
  return hipGetLastError();
}

}  // namespace pmc
