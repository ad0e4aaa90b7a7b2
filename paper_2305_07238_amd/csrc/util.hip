// util.hip - fill kernels (used instead of memset nodes so every step of a
// frame can be captured in a HIP graph) and the statistics reduction.
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
__global__ void k_stats_reduce(unsigned long long* slots, unsigned long long* out) {
  const int q = threadIdx.x;
  if (q >= kStatStride) return;
  unsigned long long s = 0;
  for (int k = 0; k < kStatSlots; ++k) {
    s += slots[k * kStatStride + q];
    slots[k * kStatStride + q] = 0ull;
  }
  if (out) out[q] += s;
}

hipError_t launch_stats_reduce(unsigned long long* slots, pmc_stats* out, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(64), 0, s, slots,
                     reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

}  // namespace pmc
