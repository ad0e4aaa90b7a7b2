// util.hip - fill kernels (used instead of memset nodes so every step of a
// frame can be captured in a HIP graph) and the statistics reduction.
#include "device_common.h"
#include "shade.h"

namespace pmc {

__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t value, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

static unsigned fill_grid(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  return (unsigned)(g < 8192 ? (g ? g : 1) : 8192);
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t value, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

// slots[kStatSlots][kStatStride] -> out (+=), then clear the slots.
// One workgroup of 1024 threads: thread t adds counter t % kStatStride over the
// slots t / kStatStride, t / kStatStride + 32, ...; then 32 threads add the
// 32 partial sums of each counter.
constexpr int kReduceThreads = 1024;
constexpr int kReduceRows = kReduceThreads / kStatStride;     // 32
static_assert(kReduceThreads % kStatStride == 0 && kStatSlots % kReduceRows == 0, "reduce layout");

__global__ __launch_bounds__(kReduceThreads) void k_stats_reduce(unsigned long long* slots,
                                                                unsigned long long* out) {
  __shared__ unsigned long long part[kReduceThreads];
  const int t = threadIdx.x, q = t % kStatStride, row = t / kStatStride;
  constexpr int kPer = kStatSlots / kReduceRows;
  unsigned long long v[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) v[j] = slots[(row + j * kReduceRows) * kStatStride + q];
  unsigned long long s = 0ull;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {            // all loads above are in flight before the clears
    s += v[j];
    slots[(row + j * kReduceRows) * kStatStride + q] = 0ull;
  }
  part[t] = s;
  __syncthreads();
  if (t < kStatStride) {
    unsigned long long tot = 0ull;
    for (int r = 0; r < kReduceRows; ++r) tot += part[r * kStatStride + t];
    if (out) out[t] += tot;
  }
}

hipError_t launch_stats_reduce(unsigned long long* slots, pmc_stats* out, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(kReduceThreads), 0, s, slots,
                     reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

// ------------------------------------------------------------ scan ---

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanItems = 16;
constexpr uint32_t kScanTile = kScanThreads * kScanItems;   // cells per scan block

uint32_t scan_blocks(uint32_t n) { return (n + kScanTile - 1) / kScanTile; }

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // 256 threads = 4 waves
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  uint32_t wbase = 0, all = 0;
  for (int k = 0; k < 4; ++k) {
    if (k < w) wbase += sh[k];
    all += sh[k];
  }
  __syncthreads();
  *total = all;
  return wbase + x - v;
}

__global__ __launch_bounds__(256) void k_scan_up(const uint32_t* cnt, uint32_t n,
                                                 uint32_t* block_sums) {
  __shared__ uint32_t sh[4];
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t s = 0;
  for (uint32_t k = 0; k < kScanItems; ++k)
    if (base + k < n) s += cnt[base + k];
  uint32_t total;
  block_excl_scan(s, sh, &total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_top(uint32_t* block_sums, uint32_t nb,
                                                  uint32_t* total) {
  __shared__ uint32_t sh[4];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < nb; b0 += 256) {
    uint32_t i = b0 + threadIdx.x;
    uint32_t v = i < nb ? block_sums[i] : 0u;
    uint32_t tsum;
    uint32_t ex = block_excl_scan(v, sh, &tsum);
    if (i < nb) block_sums[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += tsum;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(256) void k_scan_down(const uint32_t* cnt, uint32_t n,
                                                   const uint32_t* block_sums, uint32_t* start,
                                                   uint32_t* cursor) {
  __shared__ uint32_t sh[4];
  const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? cnt[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = block_sums[blockIdx.x] + block_excl_scan(s, sh, &total);
#pragma unroll
  for (uint32_t k = 0; k < kScanItems; ++k) {
    if (base + k < n) {
      start[base + k] = run;
      if (cursor) cursor[base + k] = run;
    }
    run += v[k];
  }
}


hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t n, uint32_t* out, uint32_t* out_copy,
                                 uint32_t* block_sums, uint32_t* total, hipStream_t s) {
  const uint32_t nb = scan_blocks(n ? n : 1);
  hipLaunchKernelGGL(k_scan_up, dim3(nb), dim3(kScanThreads), 0, s, in, n, block_sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, block_sums, nb, total);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, in, n, block_sums, out,
                     out_copy);
  return hipGetLastError();
}

}  // namespace pmc
