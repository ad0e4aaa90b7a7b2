// sort.hip - group the hits of a batch by material so that every wave runs a
// single program (histogram -> scan in longest-program-first order -> scatter).
// Within a material the original order is kept inside each 64-hit wave; the
// order of waves is the order their atomics land.  Hits whose material id is
// out of range go to the last bucket.
#include "device_common.h"
#include "shade.h"

namespace pmc {

constexpr uint32_t kLdsHistMax = 16384;   // buckets histogrammed in LDS (64 KiB)

__global__ __launch_bounds__(256) void k_hist(const uint32_t* material, uint32_t n,
                                              uint32_t n_mats, uint32_t* counts) {
  extern __shared__ uint32_t hist[];
  const uint32_t nb = n_mats + 1;
  const bool use_lds = nb <= kLdsHistMax;
  if (use_lds)
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t end = ((n + stride - 1) / stride) * stride;   // uniform trip count
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < end; i += stride) {
    const bool valid = i < n;
    uint32_t b = 0;
    if (valid) {
      uint32_t m = material[i];
      b = m < n_mats ? m : n_mats;
    }
    // one atomic per (wave, bucket): hits arrive in screen order, so a wave
    // usually holds one or two materials
    uint64_t act = __ballot(valid);
    while (act) {
      const int leader = __ffsll((unsigned long long)act) - 1;
      const uint32_t bl = __builtin_amdgcn_readlane(b, leader);
      const uint64_t match = __ballot(valid && b == bl);
      if (lane_id() == leader) {
        if (use_lds) atomicAdd(&hist[bl], (uint32_t)__popcll(match));
        else atomicAdd(&counts[bl], (uint32_t)__popcll(match));
      }
      act &= ~match;
    }
  }
  __syncthreads();
  if (use_lds)
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
      if (hist[b]) atomicAdd(&counts[b], hist[b]);
}

// One block: exclusive scan of the bucket counts in rank order (materials by
// decreasing program length, invalid bucket last) -> cursor[bucket].  The
// counts are cleared for the next batch, and `reset[0 .. n_reset)` is zeroed.
__global__ __launch_bounds__(1024) void k_bucket_scan(uint32_t* counts, uint32_t n_mats,
                                                      const uint32_t* lpt, uint32_t* cursor,
                                                      uint32_t* reset, uint32_t n_reset) {
  __shared__ uint32_t part[1024];
  const uint32_t nb = n_mats + 1;
  const uint32_t per = (nb + blockDim.x - 1) / blockDim.x;
  const uint32_t r0 = threadIdx.x * per;
  uint32_t local = 0;
  for (uint32_t r = r0; r < r0 + per && r < nb; ++r) local += counts[r < n_mats ? lpt[r] : n_mats];
  part[threadIdx.x] = local;
  __syncthreads();
  for (uint32_t off = 1; off < blockDim.x; off <<= 1) {     // Hillis-Steele inclusive scan
    uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - local;
  for (uint32_t r = r0; r < r0 + per && r < nb; ++r) {
    uint32_t b = r < n_mats ? lpt[r] : n_mats;
    cursor[b] = run;
    run += counts[b];
    counts[b] = 0u;
  }
  if (threadIdx.x < n_reset) reset[threadIdx.x] = 0u;
}

// Block-aggregated scatter: a block takes kScatterTile consecutive hits, ranks
// them per bucket in LDS (one LDS atomic per wave and bucket), reserves one
// global range per bucket present in the tile, then writes the permutation.
constexpr uint32_t kScatterThreads = 512;
constexpr uint32_t kScatterPer = 32;
constexpr uint32_t kScatterTile = kScatterThreads * kScatterPer;

__global__ __launch_bounds__(512) void k_scatter_block(const uint32_t* material, uint32_t n,
                                                       uint32_t n_mats, uint32_t* cursor,
                                                       uint32_t* perm) {
  extern __shared__ uint32_t sh[];
  const uint32_t nb = n_mats + 1;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) sh[b] = 0u;
  __syncthreads();
  const uint32_t base = blockIdx.x * kScatterTile;
  uint32_t pos[kScatterPer], bk[kScatterPer];
#pragma unroll
  for (uint32_t r = 0; r < kScatterPer; ++r) {
    const uint32_t i = base + r * kScatterThreads + threadIdx.x;
    const bool valid = i < n;
    uint32_t b = 0;
    if (valid) {
      uint32_t m = material[i];
      b = m < n_mats ? m : n_mats;
    }
    uint32_t p = 0;
    uint64_t act = __ballot(valid);
    while (act) {
      const int leader = __ffsll((unsigned long long)act) - 1;
      const uint32_t bl = __builtin_amdgcn_readlane(b, leader);
      const uint64_t match = __ballot(valid && b == bl);
      uint32_t old = 0;
      if (lane_id() == leader) old = atomicAdd(&sh[bl], (uint32_t)__popcll(match));
      old = __shfl(old, leader, 64);
      if (valid && b == bl) p = old + (uint32_t)__popcll(match & lanemask_lt());
      act &= ~match;
    }
    pos[r] = p;
    bk[r] = b;
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    const uint32_t c = sh[b];
    if (c) sh[b] = atomicAdd(&cursor[b], c);
  }
  __syncthreads();
#pragma unroll
  for (uint32_t r = 0; r < kScatterPer; ++r) {
    const uint32_t i = base + r * kScatterThreads + threadIdx.x;
    if (i < n) perm[sh[bk[r]] + pos[r]] = i;
  }
}

__global__ __launch_bounds__(256) void k_scatter(const uint32_t* material, uint32_t n,
                                                 uint32_t n_mats, uint32_t* cursor,
                                                 uint32_t* perm) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
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
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&cursor[bl], (uint32_t)__popcll(match));
    base = __shfl(base, leader, 64);
    if (valid && b == bl) perm[base + (uint32_t)__popcll(match & lanemask_lt())] = i;
    act &= ~match;
  }
}

hipError_t launch_material_sort(const uint32_t* material, uint32_t n, uint32_t n_mats,
                                const uint32_t* lpt_order, uint32_t* counts, uint32_t* cursor,
                                uint32_t* perm, uint32_t* reset, uint32_t n_reset,
                                hipStream_t s) {
  // counts[] is all-zero on entry (cleared at allocation and by each scan)
  const uint32_t nb = n_mats + 1;
  // few, large blocks: every block adds its bucket counts with one global atomic
  // per bucket, and same-address atomics serialise across the XCDs
  uint32_t blocks = (n + 16383) / 16384;
  blocks = blocks < 128 ? (blocks ? blocks : 1) : 128;
  const bool lds_ok = nb <= kLdsHistMax;
  hipLaunchKernelGGL(k_hist, dim3(blocks), dim3(256), lds_ok ? nb * sizeof(uint32_t) : 0, s,
                     material, n, n_mats, counts);
  hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, counts, n_mats, lpt_order, cursor,
                     reset, n_reset);
  if (lds_ok)
    hipLaunchKernelGGL(k_scatter_block, dim3((n + kScatterTile - 1) / kScatterTile),
                       dim3(kScatterThreads), nb * sizeof(uint32_t), s, material, n, n_mats,
                       cursor, perm);
  else
    hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, material, n, n_mats,
                       cursor, perm);
  return hipGetLastError();
}

}  // namespace pmc
