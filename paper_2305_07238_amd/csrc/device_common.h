// device_common.h - device-side helpers shared by the HIP kernels of libpmc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "program.h"

namespace pmc {

// Uniform (wave-invariant) program data is read through the constant address
// space so the compiler emits scalar loads (SMEM, scalar cache) for it.
#define PMC_CONST __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ const PMC_CONST T* as_const(const T* p) {
  return (const PMC_CONST T*)(p);
}

// ---- 64-bit finalizer (SplitMix64 output mix, Steele/Lea/Flood 2014) ------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSeedCell = 0x9E3779B97F4A7C15ull;    // Hash: cell index
constexpr uint64_t kSeedVerify = 0xC2B2AE3D27D4EB4Full;  // Hash2: verification key

// ---- x mod N_c without a division ------------------------------------------
// N_c a power of two: a mask.  Otherwise the direct remainder of Lemire, Kaser
// and Kurz ("Faster remainder by direct computation", 2019): with
// M = ceil(2^64 / n), x mod n = hi64((M * x mod 2^64) * n), exact for 32-bit x, n.
struct CellMap {
  uint32_t n, mask;          // mask = n - 1 when n is a power of two above 1, else 0
  uint64_t magic;            // ceil(2^64 / n); 0 for n = 1
};

__host__ __device__ inline CellMap make_cell_map(uint32_t n) {
  CellMap c;
  c.n = n;
  c.mask = (n > 1u && (n & (n - 1u)) == 0u) ? n - 1u : 0u;
  c.magic = n > 1u ? ~0ull / n + 1ull : 0ull;
  return c;
}

__device__ __forceinline__ uint32_t cell_of(const CellMap& c, uint32_t x) {
  if (c.mask) return x & c.mask;
  return (uint32_t)__umul64hi(c.magic * (uint64_t)x, (uint64_t)c.n);
}

// ---- descriptor of a cacheable output (Sec. 3.1 Eq. 1, Sec. 3.2) -----------
struct Key {
  uint32_t cell, hash2;
  int32_t level, tx, ty;
  bool bypass;
};

// Descriptor of a cacheable output (Sec. 3.1, Eq. 1), one routine for both
// kinds so that a kernel carries a single copy of the arithmetic:
//   texel (kind 0): coordinates (u, v), m2 = min(|g1|^2, |g2|^2) in binary64
//     (the products are exact there);
//   world cell (kind 1, the paper's other shading-point information): the
//     world position (x, y, z), m2 = w^2 of the footprint width w.
// Level: floor(lambda) with lambda = -log2(sqrt(m2)) (Eq. 1); frexp gives
// m2 = f 2^e, f in [1/2, 1), and floor(lambda) = floor((-e + [f == 1/2]) / 2);
// m2 = 0 takes the finest level.  Indices floor(c 2^L) must lie in the int32
// range, else the hit bypasses.  Words: texel k0 = mat << 32 | node << 16 |
// socket << 8 | L, k1 = (u32)tx << 32 | (u32)ty; cell k0 additionally has bit
// 7 (never set by a texel level, L <= 20), k1 = qx << 42 | qy << 21 | qz with
// each index mod 2^21.
// h2mask keeps bits of the verification hash (all 32 in the method; fewer only
// to force verification collisions in tests).
__device__ __forceinline__ Key make_key(uint32_t mat, uint32_t node_sock, bool cell_kind,
                                        float c0, float c1, float c2, double m2, bool finite,
                                        int bias, int lmax, const CellMap& cells,
                                        uint32_t h2mask) {
  Key k;
  k.cell = 0; k.hash2 = 1; k.level = 0; k.tx = 0; k.ty = 0; k.bypass = true;
  if (!finite) return k;
  int L;
  if (m2 == 0.0) {
    L = lmax;
  } else {
    int e;
    const double f = frexp(m2, &e);
    const int t = -e + (f == 0.5 ? 1 : 0);
    L = (t >> 1) + bias;                   // arithmetic shift = floor division by 2
    L = L < 0 ? 0 : (L > lmax ? lmax : L);
  }
  const double x = ldexp((double)c0, L), y = ldexp((double)c1, L), z = ldexp((double)c2, L);
  const double lim = 2147483648.0;
  if (!(x >= -lim && x < lim && y >= -lim && y < lim && z >= -lim && z < lim)) return k;
  const int qx = (int)floor(x), qy = (int)floor(y), qz = (int)floor(z);
  uint64_t k0 = ((uint64_t)mat << 32) | (uint64_t)node_sock | (uint64_t)(uint32_t)L;
  uint64_t k1;
  if (cell_kind) {
    const uint64_t M = (1ull << 21) - 1ull;
    k0 |= 0x80ull;
    k1 = (((uint64_t)(uint32_t)qx & M) << 42) | (((uint64_t)(uint32_t)qy & M) << 21) |
         ((uint64_t)(uint32_t)qz & M);
  } else {
    k1 = ((uint64_t)(uint32_t)qx << 32) | (uint64_t)(uint32_t)qy;
  }
  const uint64_t hc = mix64(k1 ^ mix64(k0 ^ kSeedCell));
  const uint64_t hv = mix64(k1 ^ mix64(k0 ^ kSeedVerify));
  k.cell = cell_of(cells, (uint32_t)(hc >> 32));
  k.hash2 = (uint32_t)hv & h2mask;
  if (k.hash2 == 0) k.hash2 = 1;
  k.level = L; k.tx = qx; k.ty = qy; k.bypass = false;
  return k;
}

// Descriptor hashes of raw descriptor words (Algorithm 1 surface).
__device__ __forceinline__ void raw_hash(uint64_t k0, uint64_t k1, const CellMap& cells,
                                         uint32_t h2mask, uint32_t* cell, uint32_t* hash2) {
  uint64_t hc = mix64(k1 ^ mix64(k0 ^ kSeedCell));
  uint64_t hv = mix64(k1 ^ mix64(k0 ^ kSeedVerify));
  *cell = cell_of(cells, (uint32_t)(hc >> 32));
  uint32_t h = (uint32_t)hv & h2mask;
  *hash2 = h ? h : 1u;
}

// ---- 32-bit value codes (Sec. 3.3) -----------------------------------------
// FLOAT: binary32 bits.  COLOR: RGB9E5 (Khronos EXT_texture_shared_exponent,
// N = 9, B = 15), computed exactly: only power-of-two scalings and an exact
// round-half-up.
__device__ __forceinline__ uint32_t round_half_up(float x) {
  float t = floorf(x);
  return (uint32_t)t + ((x - t) >= 0.5f ? 1u : 0u);
}

__device__ __forceinline__ uint32_t rgb9e5_encode(float r, float g, float b) {
  const float kMax = 65408.0f;
  r = fminf(fmaxf(r, 0.0f), kMax);
  g = fminf(fmaxf(g, 0.0f), kMax);
  b = fminf(fmaxf(b, 0.0f), kMax);
  float mx = fmaxf(r, fmaxf(g, b));
  int exp_p = 0;
  if (mx > 0.0f) {
    int e;
    frexpf(mx, &e);                      // mx = f 2^e, floor(log2 mx) = e - 1
    int fl = e - 1;
    exp_p = (fl < -16 ? -16 : fl) + 16;
  }
  float scale = ldexpf(1.0f, 24 - exp_p);
  if (round_half_up(mx * scale) == 512u) {
    exp_p += 1;
    scale *= 0.5f;
  }
  uint32_t rm = round_half_up(r * scale), gm = round_half_up(g * scale),
           bm = round_half_up(b * scale);
  return rm | (gm << 9) | (bm << 18) | ((uint32_t)exp_p << 27);
}

__device__ __forceinline__ float3 rgb9e5_decode(uint32_t c) {
  int e = (int)(c >> 27) - 24;
  return make_float3(ldexpf((float)(c & 0x1FF), e), ldexpf((float)((c >> 9) & 0x1FF), e),
                     ldexpf((float)((c >> 18) & 0x1FF), e));
}

// ---- wave helpers -----------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace pmc
