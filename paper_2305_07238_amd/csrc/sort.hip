// sort.hip - group the hits of a batch by material so that every wave runs a
// single program (tile histograms -> scan in longest-program-first order ->
// tile scatter).  Hits whose material id is out of range go to the last bucket.
#include "device_common.h"
#include "shade.h"

namespace pmc {

// Tiled counting sort without global atomics: tile k (a block) histograms
// its hits in LDS and writes hist[rank(b)][k]; an exclusive scan over that
// matrix (bucket rank major, tile minor) gives every (bucket, tile) its output
// offset; each tile then scatters its hits, ranking them in LDS.  Buckets are
// ranked by decreasing program length (invalid ids last), so longer programs
// come first in the permutation.
__global__ __launch_bounds__(256) void k_tile_hist(const uint32_t* material, uint32_t n,
                                                   uint32_t n_mats, uint32_t tile,
                                                   uint32_t n_tiles, const uint32_t* rank,
                                                   uint32_t* mat_counts) {
  extern __shared__ uint32_t hist[];
  const uint32_t nb = n_mats + 1;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0u;
  __syncthreads();
  const uint32_t beg = blockIdx.x * tile;
  const uint32_t end = min(beg + tile, n);
  for (uint32_t i0 = beg; i0 < end; i0 += blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const bool valid = i < end;
    uint32_t b = 0;
    if (valid) {
      uint32_t m = material[i];
      b = m < n_mats ? m : n_mats;
    }
    uint64_t act = __ballot(valid);
    while (act) {
      const int leader = __ffsll((unsigned long long)act) - 1;
      const uint32_t bl = __builtin_amdgcn_readlane(b, leader);
      const uint64_t match = __ballot(valid && b == bl);
      if (lane_id() == leader) atomicAdd(&hist[bl], (uint32_t)__popcll(match));
      act &= ~match;
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    const uint32_t r = b < n_mats ? rank[b] : n_mats;
    mat_counts[(uint64_t)r * n_tiles + blockIdx.x] = hist[b];
  }
}

__global__ __launch_bounds__(256) void k_tile_scatter(const uint32_t* material, uint32_t n,
                                                      uint32_t n_mats, uint32_t tile,
                                                      uint32_t n_tiles, const uint32_t* rank,
                                                      const uint32_t* offsets, uint32_t* perm) {
  extern __shared__ uint32_t base[];
  const uint32_t nb = n_mats + 1;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    const uint32_t r = b < n_mats ? rank[b] : n_mats;
    base[b] = offsets[(uint64_t)r * n_tiles + blockIdx.x];
  }
  __syncthreads();
  const uint32_t beg = blockIdx.x * tile;
  const uint32_t end = min(beg + tile, n);
  for (uint32_t i0 = beg; i0 < end; i0 += blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const bool valid = i < end;
    uint32_t b = 0;
    if (valid) {
      uint32_t m = material[i];
      b = m < n_mats ? m : n_mats;
    }
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

uint32_t sort_tiles(uint32_t n) {
  uint32_t t = (n + 4095) / 4096;
  return t < 1 ? 1 : (t > 512 ? 512 : t);
}

hipError_t launch_material_sort_tiled(const uint32_t* material, uint32_t n, uint32_t n_mats,
                                      const uint32_t* rank, uint32_t* mat_counts,
                                      uint32_t* offsets, uint32_t* scan_sums, uint32_t* perm,
                                      uint32_t* reset, uint32_t n_reset, hipStream_t s) {
  const uint32_t nb = n_mats + 1;
  const uint32_t n_tiles = sort_tiles(n);
  const uint32_t tile = (n + n_tiles - 1) / n_tiles;
  const size_t lds = (size_t)nb * sizeof(uint32_t);
  hipLaunchKernelGGL(k_tile_hist, dim3(n_tiles), dim3(256), lds, s, material, n, n_mats, tile,
                     n_tiles, rank, mat_counts);
  hipError_t e = launch_exclusive_scan(mat_counts, nb * n_tiles, offsets, nullptr, scan_sums,
                                       nullptr, s);
  if (e != hipSuccess) return e;
  if (n_reset) {
    e = launch_fill_u32(reset, 0u, n_reset, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tile_scatter, dim3(n_tiles), dim3(256), lds, s, material, n, n_mats, tile,
                     n_tiles, rank, offsets, perm);
  return hipGetLastError();
}

}  // namespace pmc
