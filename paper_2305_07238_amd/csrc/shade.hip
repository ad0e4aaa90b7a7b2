// shade.hip - the shading kernel: descriptor keys, cache probes, the node
// interpreter and cache inserts for one batch of hits.
//
// Paper passages: Sec. 2 (networks executed as data in storage order),
// Sec. 3 (at a cacheable node look up first; on a hit use the value and skip
// the sub-graph, otherwise evaluate it and store the result), Sec. 3.1 and
// Eq. 1 (descriptor: material, node, level, texel), Sec. 3.2 (two hashes,
// N_c cells x N_e entries, keep the first value), Sec. 3.3 and Algorithm 1
// (lock-free insert with one 64-bit compare-and-swap of hash2 << 32 | code).
//
// Execution model (gfx950, wave64): a wave takes 64 hits (a chunk).  Hits are
// normally sorted by material first, so a chunk holds one material and the
// program is read with scalar loads; a chunk that straddles materials runs
// the program once per material with the other lanes masked off.  Per lane:
//   1. compute the key of every cacheable output and probe its cell
//      (all K probes are issued before any result is used);
//   2. miss_mask = outputs not found; run each instruction whose need mask
//      intersects the wave's needs (EXEC = lanes that need it), so a wave whose
//      lanes all hit skips the sub-graphs entirely;
//   3. after a cacheable output is computed on a miss, encode and insert it
//      (CACHED: Algorithm 1 CAS; SNAPSHOT: append an insert candidate);
//   4. write the BSDF inputs.
#include "shade.h"

#include "device_common.h"

namespace pmc {

// ---------------------------------------------------------------- helpers ---

struct LaneRegs {                      // per-wave register file in LDS, [reg][lane]
  float* base;
  int lane;
  __device__ __forceinline__ float get(int r) const { return base[r * 64 + lane]; }
  __device__ __forceinline__ void set(int r, float v) const { base[r * 64 + lane] = v; }
};

struct HitData {
  float u, v;
  float4 g;
  float3 n;
};

// Descriptor of cacheable output cd at hit h: a UV texel (Sec. 3.1, Eq. 1) or,
// for outputs that depend on the world position, a world-space cell (the
// position and width are read here only, so the UV-only path holds no
// registers for them).
__device__ __forceinline__ Key key_of(const ShadeArgs& a, uint32_t m, uint32_t h,
                                      uint32_t node_sock, uint8_t kind, const HitData& hd) {
  const bool cell = kind == KEY_CELL;
  float c0 = hd.u, c1 = hd.v, c2 = 0.0f;
  double m2;
  bool finite;
  if (cell) {
    const float* p = a.position + (uint64_t)h * 3;
    const float w = a.width[h];
    c0 = p[0]; c1 = p[1]; c2 = p[2];
    finite = isfinite(c0) && isfinite(c1) && isfinite(c2) && isfinite(w);
    m2 = (double)w * (double)w;
  } else {
    const float4 g = hd.g;
    finite = isfinite(c0) && isfinite(c1) && isfinite(g.x) && isfinite(g.y) && isfinite(g.z) &&
             isfinite(g.w);
    const double s1 = (double)g.x * (double)g.x + (double)g.y * (double)g.y;
    const double s2 = (double)g.z * (double)g.z + (double)g.w * (double)g.w;
    m2 = s1 < s2 ? s1 : s2;
  }
  return make_key(m, node_sock, cell, c0, c1, c2, m2, finite, a.level_bias, a.level_max,
                  a.cells, a.hash2_mask);
}

__device__ __forceinline__ float read_f(uint32_t op, const PMC_CONST float* k, const LaneRegs& R,
                                        const HitData& hd) {
  uint32_t kind = op & 0xFF, kofs = (op >> 8) & 0xFF, r = op >> 16;
  switch (kind) {
    case OPK_CONST_F: case OPK_CONST_C: return k[kofs];
    case OPK_REG_F: case OPK_REG_F2C: return R.get(r);
    case OPK_REG_C2F: case OPK_REG_C:
      return (R.get(r) + R.get(r + 1) + R.get(r + 2)) / 3.0f;
    default: return 0.0f;
  }
}

__device__ __forceinline__ float3 read_c(uint32_t op, const PMC_CONST float* k, const LaneRegs& R,
                                         const HitData& hd) {
  uint32_t kind = op & 0xFF, kofs = (op >> 8) & 0xFF, r = op >> 16;
  switch (kind) {
    case OPK_CONST_C: return make_float3(k[kofs], k[kofs + 1], k[kofs + 2]);
    case OPK_CONST_F: { float x = k[kofs]; return make_float3(x, x, x); }
    case OPK_REG_C: case OPK_REG_C2F: return make_float3(R.get(r), R.get(r + 1), R.get(r + 2));
    case OPK_REG_F: case OPK_REG_F2C: { float x = R.get(r); return make_float3(x, x, x); }
    case OPK_NORMAL: return hd.n;
    default: return make_float3(0.f, 0.f, 0.f);
  }
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return a + t * (b - a); }
__device__ __forceinline__ float clamp01f(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Noise corner hash: low 32 bits of mix64(((u32)i << 32 | (u32)j) ^ seed * golden).
__device__ __forceinline__ uint32_t lattice_hash(int i, int j, uint64_t sgold) {
  uint64_t z = ((uint64_t)(uint32_t)i << 32) | (uint64_t)(uint32_t)j;
  return (uint32_t)mix64(z ^ sgold);
}

__device__ float value_noise(float u, float v, float f0, int octaves, uint32_t seed) {
  float total = 0.0f, norm = 0.0f, amp = 1.0f, freq = f0;
  for (int o = 0; o < octaves; ++o) {
    uint64_t sg = (uint64_t)(seed + (uint32_t)o) * kGolden;
    float px = u * freq, py = v * freq;
    float fi = floorf(px), fj = floorf(py);
    float fx = px - fi, fy = py - fj;
    int i = (int)fi, j = (int)fj;
    const float s = 2.3283064365386963e-10f;  // 2^-32
    float h00 = (float)lattice_hash(i, j, sg) * s;
    float h10 = (float)lattice_hash(i + 1, j, sg) * s;
    float h01 = (float)lattice_hash(i, j + 1, sg) * s;
    float h11 = (float)lattice_hash(i + 1, j + 1, sg) * s;
    float sx = fx * fx * (3.0f - 2.0f * fx);
    float sy = fy * fy * (3.0f - 2.0f * fy);
    float n = lerpf(lerpf(h00, h10, sx), lerpf(h01, h11, sx), sy);
    total += amp * n;
    norm += amp;
    amp *= 0.5f;
    freq *= 2.0f;
  }
  return total / norm;
}

// gradient g(h & 7) of {(1,0),(-1,0),(0,1),(0,-1),(1,1),(-1,1),(1,-1),(-1,-1)} dotted with (dx, dy)
__device__ __forceinline__ float grad_dot(uint32_t h, float dx, float dy) {
  uint32_t id = h & 7u;
  float gx = (id == 2u || id == 3u) ? 0.0f : ((id & 1u) ? -1.0f : 1.0f);
  float gy = id < 2u ? 0.0f : (id < 4u ? ((id & 1u) ? -1.0f : 1.0f) : ((id & 2u) ? -1.0f : 1.0f));
  return gx * dx + gy * dy;
}

__device__ __forceinline__ float fade5(float t) {
  return t * t * t * (t * (t * 6.0f - 15.0f) + 10.0f);
}

__device__ float perlin_noise(float u, float v, float f0, int octaves, uint32_t seed) {
  float total = 0.0f, norm = 0.0f, amp = 1.0f, freq = f0;
  for (int o = 0; o < octaves; ++o) {
    uint64_t sg = (uint64_t)(seed + (uint32_t)o) * kGolden;
    float px = u * freq, py = v * freq;
    float fi = floorf(px), fj = floorf(py);
    float fx = px - fi, fy = py - fj;
    int i = (int)fi, j = (int)fj;
    float d00 = grad_dot(lattice_hash(i, j, sg), fx, fy);
    float d10 = grad_dot(lattice_hash(i + 1, j, sg), fx - 1.0f, fy);
    float d01 = grad_dot(lattice_hash(i, j + 1, sg), fx, fy - 1.0f);
    float d11 = grad_dot(lattice_hash(i + 1, j + 1, sg), fx - 1.0f, fy - 1.0f);
    float qx = fade5(fx), qy = fade5(fy);
    float n = lerpf(lerpf(d00, d10, qx), lerpf(d01, d11, qx), qy);
    total += amp * n;
    norm += amp;
    amp *= 0.5f;
    freq *= 2.0f;
  }
  return 0.5f + 0.5f * (total / norm);
}

// Value noise of the world position: octave o at frequency f0 2^o, lattice
// corner (i, j, k) valued lo32(mix64(((u32)i << 32 | (u32)j) ^
// mix64((u32)k ^ (seed + o) G))) 2^-32, trilinear with smoothstep weights.
__device__ float position_noise(const ShadeArgs& a, uint32_t h, float f0, int octaves,
                               uint32_t seed) {
  const float* pp = a.position + (uint64_t)h * 3;
  const float p0 = pp[0], p1 = pp[1], p2 = pp[2];
  float total = 0.0f, norm = 0.0f, amp = 1.0f, freq = f0;
#pragma unroll 1
  for (int o = 0; o < octaves; ++o) {
    const uint64_t sg = (uint64_t)(seed + (uint32_t)o) * kGolden;
    const float px = p0 * freq, py = p1 * freq, pz = p2 * freq;
    const float fi = floorf(px), fj = floorf(py), fk = floorf(pz);
    const float fx = px - fi, fy = py - fj, fz = pz - fk;
    const int i = (int)fi, j = (int)fj, kk = (int)fk;
    const float wx = fx * fx * (3.0f - 2.0f * fx), wy = fy * fy * (3.0f - 2.0f * fy),
                wz = fz * fz * (3.0f - 2.0f * fz);
    float val = 0.0f;
    // corners in the order dz, dy, dx (dx fastest)
#pragma unroll 1
    for (int c = 0; c < 8; ++c) {
      const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
      const uint64_t kz = mix64((uint64_t)(uint32_t)(kk + dz) ^ sg);
      const uint64_t ij = ((uint64_t)(uint32_t)(i + dx) << 32) | (uint64_t)(uint32_t)(j + dy);
      const float hv = (float)(uint32_t)mix64(ij ^ kz) * 2.3283064365386963e-10f;  // 2^-32
      val += (dx ? wx : 1.0f - wx) * (dy ? wy : 1.0f - wy) * (dz ? wz : 1.0f - wz) * hv;
    }
    total += amp * val;
    norm += amp;
    amp *= 0.5f;
    freq *= 2.0f;
  }
  return total / norm;
}

__device__ __forceinline__ int wrap_index(int i, uint32_t w) {
  if ((w & (w - 1u)) == 0u) return i & (int)(w - 1u);
  int r = i % (int)w;
  return r < 0 ? r + (int)w : r;
}

__device__ __forceinline__ float4 texel(const uint32_t* pool, uint64_t off, uint32_t w, int i,
                                        int j) {
  uint32_t t = pool[off + (uint64_t)j * w + (uint32_t)i];
  const float s = 1.0f / 255.0f;
  return make_float4((float)(t & 0xFF) * s, (float)((t >> 8) & 0xFF) * s,
                     (float)((t >> 16) & 0xFF) * s, (float)(t >> 24) * s);
}

__device__ __forceinline__ float4 image_texture(const ShadeArgs& a, uint32_t tex, float u,
                                                float v) {
  const PMC_CONST TexDesc* td = as_const(a.tex) + tex;
  uint64_t off = td->offset;
  uint32_t w = td->w, h = td->h;
  float x = u * (float)w - 0.5f, y = v * (float)h - 0.5f;
  float x0 = floorf(x), y0 = floorf(y);
  float fx = x - x0, fy = y - y0;
  int i0 = (int)x0, j0 = (int)y0;
  int ia = wrap_index(i0, w), ib = wrap_index(i0 + 1, w);
  int ja = wrap_index(j0, h), jb = wrap_index(j0 + 1, h);
  float4 t00 = texel(a.texels, off, w, ia, ja), t10 = texel(a.texels, off, w, ib, ja);
  float4 t01 = texel(a.texels, off, w, ia, jb), t11 = texel(a.texels, off, w, ib, jb);
  float4 r;
  r.x = lerpf(lerpf(t00.x, t10.x, fx), lerpf(t01.x, t11.x, fx), fy);
  r.y = lerpf(lerpf(t00.y, t10.y, fx), lerpf(t01.y, t11.y, fx), fy);
  r.z = lerpf(lerpf(t00.z, t10.z, fx), lerpf(t01.z, t11.z, fx), fy);
  r.w = lerpf(lerpf(t00.w, t10.w, fx), lerpf(t01.w, t11.w, fx), fy);
  return r;
}

__device__ __forceinline__ float4 color_ramp(const PMC_CONST float* p, float fac) {
  // p: 8 positions then 8 RGBA stops
  const PMC_CONST float* c = p + 8;
  if (!(fac > p[0])) return make_float4(c[0], c[1], c[2], c[3]);
  if (fac >= p[7]) return make_float4(c[28], c[29], c[30], c[31]);
  int k = 0;
#pragma unroll
  for (int q = 1; q < 7; ++q) k += (fac >= p[q]) ? 1 : 0;   // positions ascending
  float pk = p[k], pk1 = p[k + 1];
  float t = (fac - pk) / (pk1 - pk);
  const PMC_CONST float* a = c + 4 * k;
  const PMC_CONST float* b = c + 4 * (k + 1);
  return make_float4(lerpf(a[0], b[0], t), lerpf(a[1], b[1], t), lerpf(a[2], b[2], t),
                     lerpf(a[3], b[3], t));
}

__device__ __forceinline__ float3 normalize_or(float3 v, float3 fb) {
  float l = sqrtf(v.x * v.x + v.y * v.y + v.z * v.z);
  if (!(l >= 1e-12f)) return fb;
  return make_float3(v.x / l, v.y / l, v.z / l);
}

// Orthonormal basis after Duff et al. 2017 (JCGT 6(1)); sign = +1 when n.z >= 0.
__device__ __forceinline__ float3 normal_map(float3 c, float strength, float3 n) {
  float3 t = make_float3(2.0f * c.x - 1.0f, 2.0f * c.y - 1.0f, 2.0f * c.z - 1.0f);
  float sign = n.z >= 0.0f ? 1.0f : -1.0f;
  float a = -1.0f / (sign + n.z);
  float b = n.x * n.y * a;
  float3 T = make_float3(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  float3 B = make_float3(b, sign + n.y * n.y * a, -n.y);
  float3 v = make_float3(t.x * T.x + t.y * B.x + t.z * n.x, t.x * T.y + t.y * B.y + t.z * n.y,
                         t.x * T.z + t.y * B.z + t.z * n.z);
  v = normalize_or(v, n);
  float3 m = make_float3(n.x + strength * (v.x - n.x), n.y + strength * (v.y - n.y),
                         n.z + strength * (v.z - n.z));
  return normalize_or(m, n);
}

// ----------------------------------------------------------- cache access ---

struct Counters {
  uint32_t v[kNumCounters];
};

__device__ __forceinline__ uint64_t* entry_word(const ShadeArgs& a, uint32_t cell, uint32_t i) {
  return a.table + ((uint64_t)cell * a.n_entries + i) * a.entry_words;
}

// Lookup: first entry whose hash equals hash2 is a hit; an empty entry or the
// end of the cell is a miss.  All entries of a chunk of 8 are loaded at once.
__device__ __forceinline__ bool cache_lookup(const ShadeArgs& a, uint32_t cell, uint32_t hash2,
                                             uint32_t* code, uint32_t* slot) {
  *slot = 0xFFu;
  for (uint32_t base = 0; base < a.n_entries; base += 8) {
    uint64_t w[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      w[j] = (base + j < a.n_entries) ? *entry_word(a, cell, base + j) : 0ull;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (base + j >= a.n_entries) return false;
      if ((uint32_t)(w[j] >> 32) == hash2) {
        *code = (uint32_t)w[j];
        return true;
      }
      if (w[j] == 0ull) {
        *slot = base + j;
        return false;
      }
    }
  }
  return false;
}

// Cooperative lookup for 128-byte cells (8 entries of 16 bytes): every lane
// owns one cell (hash2 == 0: no lookup).  In round t the 8 lanes of group
// g = lane / 8 read the 8 words of the cell owned by lane 8t + g, so each load
// instruction fetches 8 whole cells and every cell line is fetched once.  The
// loads are unconditional (a lane without a lookup reads cell 0) so all eight
// rounds can be in flight together.  The first entry holding hash2 or empty
// decides, as in the per-lane scan; *slot gets the first empty entry (8 = none)
// for the insert that may follow a miss.  All 64 lanes must be active.
__device__ __forceinline__ bool coop_lookup128(const ShadeArgs& a, uint32_t cell, uint32_t hash2,
                                               uint32_t* code, uint32_t* slot) {
  const int lane = lane_id();
  const int g = lane >> 3, j = lane & 7;
  const char* base = reinterpret_cast<const char*>(a.table);
  uint64_t w[8];
  uint32_t hs[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int src = 8 * t + g;
    const uint32_t c_src = __shfl(cell, src, 64);
    hs[t] = __shfl(hash2, src, 64);
    const uint32_t c_use = hs[t] != 0u ? c_src : 0u;
    w[t] = *reinterpret_cast<const uint64_t*>(base + (uint64_t)c_use * 128u + j * 16);
  }
  bool found = false;
  uint32_t cd = 0u, empty = 8u;
  const int gg = lane & 7;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const uint64_t hb = __ballot(hs[t] != 0u && (uint32_t)(w[t] >> 32) == hs[t]);
    const uint64_t eb = __ballot(hs[t] != 0u && w[t] == 0ull);
    // owners of round t are lanes 8t .. 8t+7; owner 8t + gg reads group gg's bits
    const uint32_t hm = (uint32_t)(hb >> (8 * gg)) & 0xFFu;
    const uint32_t em = (uint32_t)(eb >> (8 * gg)) & 0xFFu;
    const uint32_t any = hm | em;
    const int first = any ? __ffs(any) - 1 : 0;
    const uint32_t v = __shfl((uint32_t)w[t], 8 * gg + first, 64);
    if ((lane >> 3) == t) {
      const bool hit = any && ((hm >> first) & 1u);
      found = hit;
      cd = v;
      empty = (any && !hit) ? (uint32_t)first : 8u;
    }
  }
  *code = cd;
  *slot = empty;
  return found;
}

__device__ __forceinline__ uint64_t load_relaxed(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Algorithm 1: find the first entry holding hash2 or empty, then CAS(0 -> new).
// OVERWRITE: a full cell evicts the entry with the smallest stamp, if older
// than this frame.  PRIORITY (after Sec. 5: prefer directly visible samples
// when storage is short): a full cell gives up its entry of the largest path
// depth (aux field), then the smallest stamp; it is replaced when its depth is
// larger than the sample's, or equal and older than this frame, and the new
// entry keeps the sample's depth.  Returns the outcome (counted by the caller
// without branches, which keeps the counters in registers).
enum { INS_DONE = 0, INS_PRESENT = 1, INS_CAS_FAIL = 2, INS_FULL = 3, INS_OVERWRITE = 4 };

__device__ __forceinline__ uint32_t lane_bounce(const ShadeArgs& a, uint32_t h) {
  return (a.policy == PMC_POLICY_PRIORITY && a.bounce) ? a.bounce[h] : 0u;
}

__device__ __forceinline__ void store_stamp(const ShadeArgs& a, uint64_t* p, uint32_t bounce) {
  if (a.entry_words != 2) return;
  ((uint32_t*)p)[2] = a.frame + 1u;
  if (a.policy == PMC_POLICY_PRIORITY) ((uint32_t*)p)[3] = bounce;
}

// The entry of the cell a key may take: the first one that holds the key or
// is empty (entries fill front to back and are never emptied singly, so a
// key never sits behind an empty entry); n_entries when the cell is full of
// other keys.
__device__ __forceinline__ uint32_t claimable_entry(const ShadeArgs& a, uint32_t cell,
                                                    uint32_t hash2) {
  uint32_t e = 0u;
  for (; e < a.n_entries; ++e) {
    const uint32_t h = (uint32_t)(load_relaxed(entry_word(a, cell, e)) >> 32);
    if (h == hash2 || h == 0u) break;
  }
  return e;
}

__device__ __forceinline__ int cache_insert(const ShadeArgs& a, uint32_t cell, uint32_t hash2,
                                            uint32_t code, uint32_t bounce = 0u) {
  const uint64_t neu = ((uint64_t)hash2 << 32) | code;
  const uint32_t e = claimable_entry(a, cell, hash2);
  if (e < a.n_entries) {
    // one compare-and-swap from the empty word; it fails if the entry holds
    // the key already or another key took it meanwhile
    uint64_t* p = entry_word(a, cell, e);
    uint64_t expected = 0ull;
    bool ok = __hip_atomic_compare_exchange_strong(p, &expected, neu, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ok) store_stamp(a, p, bounce);
    return ok ? INS_DONE : ((uint32_t)(expected >> 32) == hash2 ? INS_PRESENT : INS_CAS_FAIL);
  }
  const bool prio = a.policy == PMC_POLICY_PRIORITY;
  if ((a.policy == PMC_POLICY_OVERWRITE || prio) && a.entry_words == 2) {
    // victim: smallest (-depth, stamp) (depth 0 for OVERWRITE), lowest index on ties
    uint32_t best_st = 0xFFFFFFFFu, best_b = 0u;
    int victim = -1;
    for (uint32_t i = 0; i < a.n_entries; ++i) {
      uint32_t* sp = (uint32_t*)entry_word(a, cell, i) + 2;
      uint32_t st = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t b = prio ? __hip_atomic_load(sp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : 0u;
      if (victim < 0 || b > best_b || (b == best_b && st < best_st)) {
        best_st = st;
        best_b = b;
        victim = (int)i;
      }
    }
    const bool older = best_st < a.frame + 1u;
    const bool replace = prio ? (best_b > bounce || (best_b == bounce && older)) : older;
    if (victim >= 0 && replace) {
      uint64_t* p = entry_word(a, cell, (uint32_t)victim);
      uint64_t observed = load_relaxed(p);
      bool ok = (uint32_t)(observed >> 32) != hash2 &&
                __hip_atomic_compare_exchange_strong(p, &observed, neu, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ok) store_stamp(a, p, bounce);
      return ok ? INS_OVERWRITE : INS_CAS_FAIL;
    }
  }
  return INS_FULL;
}

// FIRST policy with the probe's scan reused: the lookup found entries
// 0 .. slot-1 holding other keys and entry `slot` empty (slot >= n_entries: the
// cell was full).  Entries never change once written under FIRST, so a CAS at
// `slot` is Algorithm 1 with its scan taken at lookup time.
__device__ __forceinline__ int cache_insert_at(const ShadeArgs& a, uint32_t cell, uint32_t hash2,
                                               uint32_t code, uint32_t slot) {
  if (slot >= a.n_entries) return INS_FULL;
  uint64_t* p = entry_word(a, cell, slot);
  uint64_t expected = 0ull;
  const uint64_t neu = ((uint64_t)hash2 << 32) | code;
  bool ok = __hip_atomic_compare_exchange_strong(p, &expected, neu, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (ok) store_stamp(a, p, 0u);
  return ok ? INS_DONE : ((uint32_t)(expected >> 32) == hash2 ? INS_PRESENT : INS_CAS_FAIL);
}

__device__ __forceinline__ void count_insert(Counters& cnt, bool did, int o) {
  cnt.v[CNT_INSERTS] += (uint32_t)(did && o == INS_DONE);
  cnt.v[CNT_PRESENT] += (uint32_t)(did && o == INS_PRESENT);
  cnt.v[CNT_CAS_FAIL] += (uint32_t)(did && o == INS_CAS_FAIL);
  cnt.v[CNT_FULL] += (uint32_t)(did && o == INS_FULL);
  cnt.v[CNT_OVERWRITES] += (uint32_t)(did && o == INS_OVERWRITE);
}

// Snapshot mode: the insert becomes a candidate {cell, seq, code, hash2}
// applied after the batch in seq order.  One atomic per wave reserves slots.
__device__ __forceinline__ void append_candidate(const ShadeArgs& a, bool want, uint32_t cell,
                                                 uint32_t hash2, uint32_t code, uint32_t seq,
                                                 Counters& cnt) {
  uint64_t m = __ballot(want);
  if (m == 0ull) return;
  int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(a.cand_count, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  cnt.v[CNT_CANDIDATES] += (uint32_t)want;
  if (want) {
    uint32_t pos = base + (uint32_t)__popcll(m & lanemask_lt());
    if (pos < a.cand_cap) a.cand[pos] = make_uint4(cell, seq, code, hash2);
  }
}

// Insert log (training data of the surrogate networks): one 32-byte record
// {material, ordinal, u, v, value} per logged insert.  The log has 64 regions,
// each with its own counter (a wave appends to region wave_id % 64 with one
// atomic); a full region drops further records.
__device__ __forceinline__ void log_append(const ShadeArgs& a, bool want, uint32_t m, uint32_t ord,
                                           float u, float v, float3 val, bool is_c,
                                           Counters& cnt) {
  const uint64_t mk = __ballot(want);
  if (mk == 0ull) return;
  const uint32_t region = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & 63u;
  const int leader = __ffsll((unsigned long long)mk) - 1;
  uint32_t base = a.log_region_cap;
  if (lane_id() == leader) {
    uint32_t* ctr = a.log_count + region;
    if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < a.log_region_cap)
      base = atomicAdd(ctr, (uint32_t)__popcll(mk));
  }
  base = __shfl(base, leader, 64);
  if (want) {
    const uint32_t pos = base + (uint32_t)__popcll(mk & lanemask_lt());
    if (pos < a.log_region_cap) {
      uint4* d = reinterpret_cast<uint4*>(a.log + (uint64_t)region * a.log_region_cap + pos);
      d[0] = make_uint4(m, ord, __float_as_uint(u), __float_as_uint(v));
      d[1] = make_uint4(__float_as_uint(val.x), is_c ? __float_as_uint(val.y) : 0u,
                        is_c ? __float_as_uint(val.z) : 0u, 0u);
      cnt.v[CNT_LOGGED]++;
    }
  }
}

// Surrogate output kept on an audited lane, to be compared with the graph's.
struct Audit {
  uint32_t mask;     // surrogated ordinals that the graph evaluates instead (0: none)
  uint32_t slot;
  float y[4];
};

__device__ __forceinline__ Audit no_audit() {
  Audit au;
  au.mask = 0u;
  au.slot = 0u;
  au.y[0] = au.y[1] = au.y[2] = au.y[3] = 0.0f;
  return au;
}

// Surrogate networks, first pass (whole wave active; m wave-uniform; `mine`
// marks the lanes of material m).  A lane of a trusted material whose
// surrogated outputs missed is parked: its hit index and those outputs go to
// the queue (one in 64 marked audited) and it is not evaluated now.  After the
// pass the networks run over the queue in dense waves, and the finish pass
// completes the parked hits with the networks' values.  Returns true for the
// lanes parked.
template <int MODE>
__device__ __forceinline__ bool surrogate_park(const ShadeArgs& a, uint32_t m, bool mine,
                                               uint32_t h, uint32_t ins, uint32_t region,
                                               Counters& cnt) {
  if (m >= a.n_mats) return false;
  const PMC_CONST MatHeader* H = as_const(a.hdr) + m;
  const uint32_t smask = H->surr_mask;
  if (smask == 0u) return false;
  if (as_const(a.surr_state)[H->surr_slot].trusted == 0u) return false;
  const uint32_t sm = mine ? (ins & smask) : 0u;
  if (__ballot(sm != 0u) == 0ull) return false;
  // plain entries fill the run's region from the front, audited ones from the
  // back, so the finish pass gives the audited hits (full evaluation) waves of
  // their own
  const bool audit = sm != 0u && surrogate_audited(a.frame, h);
  const uint64_t mk = __ballot(sm != 0u && !audit);
  const uint64_t ma = __ballot(audit);
  uint32_t base = 0u, abase = 0u;
  if (lane_id() == 0) {
    if (mk) base = atomicAdd(a.surr_queue_count + region, (uint32_t)__popcll(mk));
    if (ma) abase = atomicAdd(a.surr_queue_count + kQueueRegions + region, (uint32_t)__popcll(ma));
  }
  base = __shfl(base, 0, 64);
  abase = __shfl(abase, 0, 64);
  if (sm == 0u) return false;
  const uint32_t pos = audit ? a.surr_queue_cap - 1u - (abase + (uint32_t)__popcll(ma & lanemask_lt()))
                             : base + (uint32_t)__popcll(mk & lanemask_lt());
  a.surr_queue[(uint64_t)region * a.surr_queue_cap + pos] =
      make_uint2(h, sm | (audit ? 0x100u : 0u));
  return true;
}

// The second passes walk the queue in 64-entry chunks: the plain entries of
// regions 0, 1, ... first, then the audited ones.  Lane r of a wave holds
// region r's counts and chunk prefix sums (kQueueRegions = 64 = wave size).
struct QueueMap {
  uint32_t n0, n1;          // lane r: plain and audited entries of region r
  uint32_t incl0, incl1;    // lane r: chunks of regions 0..r (inclusive prefix)
  uint32_t c0, c1;          // total plain and audited chunks
};

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(x, (unsigned)o, 64);
    if (lane >= o) x += t;
  }
  return x;
}

__device__ __forceinline__ QueueMap queue_map(const ShadeArgs& a) {
  static_assert(kQueueRegions == 64, "one region per lane");
  QueueMap Q;
  const int r = lane_id();
  Q.n0 = a.surr_queue_count[r];
  Q.n1 = a.surr_queue_count[kQueueRegions + r];
  Q.incl0 = wave_incl_scan((Q.n0 + 63u) / 64u);
  Q.incl1 = wave_incl_scan((Q.n1 + 63u) / 64u);
  Q.c0 = __shfl(Q.incl0, 63, 64);
  Q.c1 = __shfl(Q.incl1, 63, 64);
  return Q;
}

// Entry index of this lane in chunk c < c0 + c1 (valid when *act).
__device__ __forceinline__ uint64_t queue_entry(const ShadeArgs& a, const QueueMap& Q, uint32_t c,
                                                bool* act) {
  const bool audited = c >= Q.c0;
  const uint32_t cc = audited ? c - Q.c0 : c;
  const uint32_t incl = audited ? Q.incl1 : Q.incl0;
  const uint32_t cnt = audited ? Q.n1 : Q.n0;
  // the region holding chunk cc: the first whose inclusive prefix exceeds cc
  const int r = (int)__popcll(__ballot(incl <= cc));
  const uint32_t r_incl = __shfl(incl, r, 64), r_n = __shfl(cnt, r, 64);
  const uint32_t r_first = r_incl - (r_n + 63u) / 64u;
  const uint32_t off = (cc - r_first) * 64u + (uint32_t)lane_id();
  *act = off < r_n;
  const uint64_t base = (uint64_t)r * a.surr_queue_cap;
  return audited ? base + a.surr_queue_cap - r_n + off : base + off;
}

// Finish pass: the network's outputs y stand in for the parked outputs `sm`
// that still miss (they go to the outputs' registers and leave the misses: no
// sub-graph evaluation, no insert).  An audited lane instead keeps them in *au
// and is evaluated by the graph.
template <int MODE>
__device__ __forceinline__ void surrogate_substitute(const ShadeArgs& a, uint32_t m, uint32_t h,
                                                     const HitData& hd, uint32_t sm, bool audit,
                                                     float4 yv, const LaneRegs& R, Counters& cnt,
                                                     uint32_t& miss, uint32_t& ins, Audit& au) {
  sm &= ins;
  if (sm == 0u) return;
  const PMC_CONST MatHeader* H = as_const(a.hdr) + m;
  const float y[4] = {yv.x, yv.y, yv.z, yv.w};
  if (audit) {
    au.mask = sm;
    au.slot = H->surr_slot;
    au.y[0] = y[0]; au.y[1] = y[1]; au.y[2] = y[2]; au.y[3] = y[3];
    cnt.v[CNT_AUDITED] += (uint32_t)__popc(sm);
    return;
  }
  const uint32_t cbeg = H->cach_begin;
  for (uint32_t c = 0; c < 8u; ++c) {
    if (!((sm >> c) & 1u)) continue;
    const CachDesc cd = a.cach[cbeg + c];
    const uint32_t ch = (H->surr_chan >> (4u * c)) & 0xFu;
    const int r = cd.reg;
    const float v0 = pick4(y, ch);
    R.set(r, v0);
    float v1 = v0, v2 = v0;
    if (cd.otype == OT_COLOR) {
      v1 = pick4(y, ch + 1u);
      v2 = pick4(y, ch + 2u);
      R.set(r + 1, v1);
      R.set(r + 2, v2);
    }
    if (a.dbg_state) a.dbg_state[(uint64_t)h * 8 + c] = 4;
    if (a.dbg_value) {
      float* dv = a.dbg_value + ((uint64_t)h * 8 + c) * 3;
      dv[0] = v0; dv[1] = v1; dv[2] = v2;
    }
    if (a.surr_insert) {
      // the network's value goes into the table like a graph value
      const bool is_c = cd.otype == OT_COLOR;
      bool want = isfinite(v0) && (!is_c || (isfinite(v1) && isfinite(v2)));
      const uint32_t code = is_c ? rgb9e5_encode(v0, v1, v2) : __float_as_uint(v0);
      const Key k = key_of(a, m, h, cd.node_sock, cd.key, hd);
      want = want && !k.bypass;
      cnt.v[CNT_INS_TRIED] += (uint32_t)want;
      if (MODE == PMC_MODE_SNAPSHOT) {
        append_candidate(a, want, k.cell, k.hash2, code, h * 32u + c, cnt);
      } else {
        const int o = want ? cache_insert(a, k.cell, k.hash2, code, lane_bounce(a, h)) : INS_FULL;
        count_insert(cnt, want, o);
      }
    }
  }
  cnt.v[CNT_SURR_USED] += (uint32_t)__popc(sm);
  miss &= ~sm;
  ins &= ~sm;
}

// ------------------------------------------------------------- the kernel ---

// Probe every cacheable output of the lane's material (Sec. 3: look up at the
// cacheable node first).  Runs with the whole wave active, before the
// per-material split.  Found values go to their registers.  Returns the miss
// mask (bypassed outputs count as misses); *ins gets the misses that may be
// inserted.  COUNT = false when the lookups were already counted (deferred hits).
// Ordinals in `skip` are known misses (parked surrogate outputs): not looked up,
// returned as insertable misses.
template <int MODE, bool COUNT>
__device__ __forceinline__ uint32_t probe_chunk(const ShadeArgs& a, bool active, uint32_t m,
                                                uint32_t h, const HitData& hd, const LaneRegs& R,
                                                Counters& cnt, uint32_t* ins, uint32_t* slots,
                                                uint32_t skip = 0u) {
  // sorted batches: the chunk's lanes usually share one material, whose header
  // and descriptors then come through the scalar cache (per-lane vector loads
  // of them put two more dependent memory round trips before the first key)
  const uint64_t act = __ballot(active);
  const uint32_t m0 = __builtin_amdgcn_readlane(m, act ? __ffsll((unsigned long long)act) - 1 : 0);
  const bool uni = act != 0ull && __ballot(active && m != m0) == 0ull && m0 < a.n_mats;
  uint32_t n_cach = 0u, cbeg = 0u;
  if (uni) {
    const PMC_CONST MatHeader* H = as_const(a.hdr) + m0;
    n_cach = active ? H->n_cach : 0u;
    cbeg = H->cach_begin;
  } else if (active && m < a.n_mats) {
    const MatHeader* H = a.hdr + m;
    n_cach = H->n_cach;
    cbeg = H->cach_begin;
  }
  uint32_t miss = 0u, insm = 0u, slot_bits = 0xFFFFFFFFu;
  const bool coop = a.n_entries == 8u && a.entry_words == 2u;
  for (uint32_t c = 0; __ballot(c < n_cach) != 0ull; ++c) {
    const bool has = c < n_cach;
    if (MODE == PMC_MODE_UNCACHED) {
      if (has) {
        miss |= 1u << c;
        if (a.dbg_state) a.dbg_state[(uint64_t)h * 8 + c] = 0;
      }
      continue;
    }
    CachDesc cd;
    cd.node_sock = 0u; cd.reg = 0; cd.otype = 0; cd.key = KEY_TEXEL;
    Key k;
    k.bypass = true; k.cell = 0u; k.hash2 = 0u;
    if (has) {
      if (uni) {
        const PMC_CONST CachDesc* cp =
            as_const(a.cach) + (__builtin_amdgcn_readfirstlane(cbeg) + c);
        cd.node_sock = cp->node_sock;
        cd.reg = cp->reg;
        cd.otype = cp->otype;
        cd.key = cp->key;
      } else {
        cd = a.cach[cbeg + c];
      }
      k = key_of(a, m, h, cd.node_sock, cd.key, hd);
    }
    const bool skipped = (skip >> c) & 1u;
    const uint32_t h2 = (has && !k.bypass && !skipped) ? k.hash2 : 0u;
    uint32_t code = 0u, slot = 0xFFu;
    bool found;
    if (__ballot(h2 != 0u) == 0ull) {
      found = false;                              // nothing to look up in this round
    } else if (coop) {
      found = coop_lookup128(a, k.cell, h2, &code, &slot);
    } else {
      found = false;
      if (h2) found = cache_lookup(a, k.cell, h2, &code, &slot);
    }
    if (!has) continue;
    // 4 bits per ordinal: first empty entry (15 = none or beyond 15)
    slot_bits = (slot_bits & ~(0xFu << (4 * c))) | ((slot < 15u ? slot : 15u) << (4 * c));
    if (COUNT) cnt.v[CNT_BYPASSES] += (uint32_t)k.bypass;
    cnt.v[COUNT ? CNT_PROBES : CNT_PROBES_DEFERRED] += (uint32_t)(!k.bypass && !skipped);
    if (COUNT) cnt.v[CNT_CACHE_HITS] += (uint32_t)(!k.bypass && found);
    uint8_t st = 0;
    if (k.bypass) {
      miss |= 1u << c;
      st = 2;
    } else {
      if (found) {
        st = 1;
        const int r = cd.reg;
        if (cd.otype == OT_COLOR) {
          float3 v = rgb9e5_decode(code);
          R.set(r, v.x); R.set(r + 1, v.y); R.set(r + 2, v.z);
          if (a.dbg_value) {
            float* dv = a.dbg_value + ((uint64_t)h * 8 + c) * 3;
            dv[0] = v.x; dv[1] = v.y; dv[2] = v.z;
          }
        } else {
          float v = __uint_as_float(code);
          R.set(r, v);
          if (a.dbg_value) a.dbg_value[((uint64_t)h * 8 + c) * 3] = v;
        }
      } else {
        miss |= 1u << c;
        insm |= 1u << c;
      }
    }
    if (a.dbg_state) a.dbg_state[(uint64_t)h * 8 + c] = st;
  }
  if (a.dbg_state && active && m < a.n_mats)
    for (uint32_t c = n_cach; c < 8; ++c) a.dbg_state[(uint64_t)h * 8 + c] = 3;
  *ins = insm;
  *slots = slot_bits;
  return miss;
}

// Interpret instructions [first, first + count) of material m (Sec. 2).  An
// instruction runs for a lane iff its need mask has kAlways or meets the
// lane's misses (Sec. 3: a found value makes its sub-graph unnecessary).  A
// cacheable output computed on a miss is encoded and stored (Algorithm 1), or
// becomes a snapshot candidate.
template <int MODE, bool DEF, bool SURR>
__device__ __forceinline__ void run_program(const ShadeArgs& a, uint32_t m, uint32_t h,
                                            const HitData& hd, const LaneRegs& R, Counters& cnt,
                                            uint32_t first, uint32_t count, uint32_t miss,
                                            uint32_t ins, uint32_t slots, const Audit& au) {
  const PMC_CONST Instr* I = as_const(a.instr) + first;
  const PMC_CONST MatHeader* MH = as_const(a.hdr) + m;
  const uint32_t cbeg = MH->cach_begin;
  for (uint32_t i = 0; i < count; ++i, ++I) {
    const uint32_t exec = I->exec;
    const bool need = (exec & kAlways) != 0u || (exec & miss) != 0u;
    if (!need) continue;
    cnt.v[CNT_NODES_EXEC]++;
    const PMC_CONST float* K = I->k;
    float3 o0 = make_float3(0.f, 0.f, 0.f);
    float o1 = 0.0f;
    switch (I->op) {
      case PMC_OP_IMAGE_TEXTURE: {
        cnt.v[CNT_TEX_EVALS]++;
        if (DEF) cnt.v[CNT_TEX_DEFERRED]++;
        float4 t = image_texture(a, I->param, hd.u, hd.v);
        o0 = make_float3(t.x, t.y, t.z);
        o1 = t.w;
        break;
      }
      case PMC_OP_VALUE_NOISE:
        o0.x = value_noise(hd.u, hd.v, K[7], I->variant, I->param);
        break;
      case PMC_OP_PERLIN_NOISE:
        o0.x = perlin_noise(hd.u, hd.v, K[7], I->variant, I->param);
        break;
      case PMC_OP_POSITION_NOISE:
        o0.x = position_noise(a, h, K[7], I->variant, I->param);
        break;
      case PMC_OP_MIX: {
        float t = clamp01f(read_f(I->src[0], K, R, hd));
        float3 x = read_c(I->src[1], K, R, hd), y = read_c(I->src[2], K, R, hd);
        o0 = make_float3(x.x + t * (y.x - x.x), x.y + t * (y.y - x.y), x.z + t * (y.z - x.z));
        break;
      }
      case PMC_OP_MATH: {
        float x = read_f(I->src[0], K, R, hd), y = read_f(I->src[1], K, R, hd), r;
        const uint32_t v = I->variant;
        if (v == PMC_MATH_ADD) r = x + y;
        else if (v == PMC_MATH_MUL) r = x * y;
        else r = x > 0.0f ? powf(x, y) : 0.0f;
        if (I->flags & PMC_NODE_CLAMP) r = clamp01f(r);
        o0.x = r;
        break;
      }
      case PMC_OP_COLOR_RAMP: {
        float4 t = color_ramp(as_const(a.pool) + I->param, read_f(I->src[0], K, R, hd));
        o0 = make_float3(t.x, t.y, t.z);
        o1 = t.w;
        break;
      }
      case PMC_OP_NORMAL_MAP:
        o0 = normal_map(read_c(I->src[0], K, R, hd), read_f(I->src[1], K, R, hd), hd.n);
        break;
      default:
        break;
    }
    // write the outputs; a socket that was found in the cache keeps the cached value
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const uint32_t dst = I->dst[s];
      if (dst == kNoReg) continue;
      const uint32_t ord = I->cord[s];
      const bool is_c = I->otype[s] != OT_FLOAT;
      const float3 val = s == 0 ? o0 : make_float3(o1, o1, o1);
      if (ord == kNoOrd || ((miss >> ord) & 1u)) {
        R.set(dst, val.x);
        if (is_c) { R.set(dst + 1, val.y); R.set(dst + 2, val.z); }
      }
      if (MODE != PMC_MODE_UNCACHED && ord != kNoOrd) {
        bool want = (ins >> ord) & 1u;
        uint32_t code = 0u, cell = 0u, hash2 = 0u;
        const bool finite = isfinite(val.x) && (!is_c || (isfinite(val.y) && isfinite(val.z)));
        cnt.v[CNT_NONFINITE] += (uint32_t)(want && !finite);
        want = want && finite;
        cnt.v[CNT_INS_TRIED] += (uint32_t)want;
        if (DEF) cnt.v[CNT_INS_TRIED_DEFERRED] += (uint32_t)want;
        if (want) {
          {
            code = is_c ? rgb9e5_encode(val.x, val.y, val.z) : __float_as_uint(val.x);
            const PMC_CONST CachDesc* cd = as_const(a.cach) + cbeg + ord;
            Key k = key_of(a, m, h, cd->node_sock, cd->key, hd);
            cell = k.cell;
            hash2 = k.hash2;
          }
        }
        bool logged = want;
        if (MODE == PMC_MODE_SNAPSHOT) {
          append_candidate(a, want, cell, hash2, code, h * 32u + ord, cnt);
        } else {
          int o = INS_FULL;
          if (want) {
            const uint32_t slot = (slots >> (4 * ord)) & 0xFu;
            if (a.policy == PMC_POLICY_FIRST && slot != 0xFu) {
              o = cache_insert_at(a, cell, hash2, code, slot);
              // another key took that entry since the lookup: run Algorithm 1 afresh
              if (o == INS_CAS_FAIL) o = cache_insert(a, cell, hash2, code);
            } else {
              o = cache_insert(a, cell, hash2, code, lane_bounce(a, h));
            }
          }
          count_insert(cnt, want, o);
          logged = want && (o == INS_DONE || o == INS_OVERWRITE);
        }
        if (a.log && ((MH->surr_mask >> ord) & 1u))
          log_append(a, logged, m, ord, hd.u, hd.v, val, is_c, cnt);
        if (SURR) {
          // audited lanes: the graph's value against the network's
          const bool aud = (au.mask >> ord) & 1u;
          uint32_t ebits = 0u;
          if (aud) {
            const uint32_t ch = (MH->surr_chan >> (4u * ord)) & 0xFu;
            float e = fabsf(val.x - pick4(au.y, ch));
            if (is_c) {
              const float e1 = fabsf(val.y - pick4(au.y, ch + 1u));
              const float e2 = fabsf(val.z - pick4(au.y, ch + 2u));
              e = (e1 > e || e1 != e1) ? e1 : e;
              e = (e2 > e || e2 != e2) ? e2 : e;
            }
            ebits = e != e ? 0x7FC00000u : __float_as_uint(e);   // NaN above every error
          }
          // one update per wave (the lanes share the material's slot): the per-lane
          // atomics on a few addresses serialised the audited waves
          const uint64_t am = __ballot(aud);
          if (am) {
            uint32_t mx = 0u;
            for (uint64_t t = am; t; t &= t - 1ull)
              mx = max(mx, (uint32_t)__builtin_amdgcn_readlane(
                                (int)ebits, __ffsll((unsigned long long)t) - 1));
            if (lane_id() == __ffsll((unsigned long long)am) - 1) {
              SurrState* ss = a.surr_state + au.slot;
              atomicMax(&ss->live_err_bits, mx);
              atomicAdd(&ss->live_n, (uint32_t)__popcll(am));
            }
          }
        }
      }
    }
  }
}

__device__ __forceinline__ void write_outputs(const ShadeArgs& a, uint32_t m, uint32_t h,
                                              const HitData& hd, const LaneRegs& R) {
  const PMC_CONST MatHeader* H = as_const(a.hdr) + m;
  const PMC_CONST float* OK = H->out_k;
  float3 base = read_c(H->out_src[0], OK, R, hd);
  float rough = read_f(H->out_src[1], OK, R, hd);
  float3 nrm = read_c(H->out_src[2], OK, R, hd);
  a.out_base[(uint64_t)h * 3 + 0] = base.x;
  a.out_base[(uint64_t)h * 3 + 1] = base.y;
  a.out_base[(uint64_t)h * 3 + 2] = base.z;
  a.out_rough[h] = rough;
  a.out_normal[(uint64_t)h * 3 + 0] = nrm.x;
  a.out_normal[(uint64_t)h * 3 + 1] = nrm.y;
  a.out_normal[(uint64_t)h * 3 + 2] = nrm.z;
}

__device__ __forceinline__ void shade_default(const ShadeArgs& a, uint32_t h, const HitData& hd) {
  a.out_base[(uint64_t)h * 3 + 0] = 0.8f;
  a.out_base[(uint64_t)h * 3 + 1] = 0.8f;
  a.out_base[(uint64_t)h * 3 + 2] = 0.8f;
  a.out_rough[h] = 0.5f;
  a.out_normal[(uint64_t)h * 3 + 0] = hd.n.x;
  a.out_normal[(uint64_t)h * 3 + 1] = hd.n.y;
  a.out_normal[(uint64_t)h * 3 + 2] = hd.n.z;
  if (a.dbg_state)
    for (int c = 0; c < 8; ++c) a.dbg_state[(uint64_t)h * 8 + c] = 3;
}

// Full evaluation of this lane after its probes: the whole program, outputs.
// DEF: the lane is a deferred hit (counted apart).
template <int MODE, bool DEF, bool SURR>
__device__ __forceinline__ void shade_full(const ShadeArgs& a, uint32_t m, uint32_t h,
                                           const HitData& hd, const LaneRegs& R, Counters& cnt,
                                           uint32_t miss, uint32_t ins, uint32_t slots,
                                           const Audit& au) {
  const PMC_CONST MatHeader* H = as_const(a.hdr) + m;
  cnt.v[CNT_NODES_TOTAL] += H->n_instr;
  run_program<MODE, DEF, SURR>(a, m, h, hd, R, cnt, H->instr_begin, H->n_instr, miss, ins, slots,
                               au);
  write_outputs(a, m, h, hd, R);
}

struct LaneHit {
  bool active;
  uint32_t h, mat;
  HitData hd;
};

// A lane's hit: its index (through the processing order) and then its data.
// The two halves are separate so a wave can fetch the next chunk's hits while
// it works on the current one.
struct LaneIdx {
  bool active;
  uint32_t h;
};

__device__ __forceinline__ LaneIdx lane_index(const uint32_t* list, uint32_t list_n,
                                              uint32_t chunk) {
  LaneIdx I;
  const uint32_t idx = chunk * 64u + (uint32_t)lane_id();
  I.active = idx < list_n;
  I.h = I.active ? (list ? list[idx] : idx) : 0u;
  return I;
}

__device__ __forceinline__ LaneHit fetch_lane(const ShadeArgs& a, LaneIdx I) {
  LaneHit L;
  L.active = I.active;
  L.h = I.h;
  L.mat = 0xFFFFFFFFu;
  L.hd.u = L.hd.v = 0.0f;
  L.hd.g = make_float4(0.f, 0.f, 0.f, 0.f);
  L.hd.n = make_float3(0.f, 0.f, 1.f);
  if (L.active) {
    const uint32_t h = I.h;
    L.mat = a.material[h];
    float2 uv = reinterpret_cast<const float2*>(a.uv)[h];
    L.hd.u = uv.x;
    L.hd.v = uv.y;
    L.hd.g = reinterpret_cast<const float4*>(a.duv)[h];
    L.hd.n = make_float3(a.normal[(uint64_t)h * 3], a.normal[(uint64_t)h * 3 + 1],
                         a.normal[(uint64_t)h * 3 + 2]);
  }
  return L;
}

__device__ __forceinline__ LaneHit load_lane(const ShadeArgs& a, const uint32_t* list,
                                             uint32_t list_n, uint32_t chunk) {
  return fetch_lane(a, lane_index(list, list_n, chunk));
}

// KIND_FULL: every lane of the chunk is evaluated completely.
// The chunk's hits arrive in L; `next` (when valid) is the index of the wave's
// next chunk, whose hits are fetched into *Ln once the probes of this chunk
// are consumed, so the loads overlap the evaluation below.
template <int MODE, bool SURR>
__device__ __forceinline__ void chunk_full(const ShadeArgs& a, const LaneHit& L, LaneIdx next,
                                           LaneHit* Ln, const LaneRegs& R, Counters& cnt,
                                           uint32_t region) {
  cnt.v[CNT_HITS] += (uint32_t)L.active;
  uint32_t ins = 0u, slots = 0u;
  uint32_t miss = probe_chunk<MODE, true>(a, L.active, L.mat, L.h, L.hd, R, cnt, &ins, &slots);
  *Ln = fetch_lane(a, next);
  uint64_t pending = __ballot(L.active);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t m = __builtin_amdgcn_readlane(L.mat, leader);
    const bool mine = L.active && L.mat == m;
    pending &= ~__ballot(mine);
    const bool parked = SURR && surrogate_park<MODE>(a, m, mine, L.h, ins, region, cnt);
    // every lookup of the material's lanes hit: only the always-needed nodes run,
    // so the short hit program replaces the walk over the whole program (which
    // fetches every instruction to test its need mask)
    const bool all_hit = __ballot(mine && !parked && miss != 0u) == 0ull;
    if (mine && !parked) {
      if (m < a.n_mats && all_hit) {
        const PMC_CONST MatHeader* H = as_const(a.hdr) + m;
        cnt.v[CNT_NODES_TOTAL] += H->n_instr;
        run_program<MODE, false, false>(a, m, L.h, L.hd, R, cnt, H->hit_begin, H->n_hit, 0u, 0u,
                                        0u, no_audit());
        write_outputs(a, m, L.h, L.hd, R);
      } else if (m < a.n_mats) {
        shade_full<MODE, false, false>(a, m, L.h, L.hd, R, cnt, miss, ins, slots, no_audit());
      } else {
        cnt.v[CNT_INVALID]++;
        shade_default(a, L.h, L.hd);
      }
    }
  }
}

// Per-wave staging buffer of deferred hits (LDS): ids of hits of one material
// whose lookups missed.  A wave walks a run of consecutive, material-sorted
// chunks; sparse misses are collected here and evaluated together in one
// dense pass (Sec. 3: evaluate the sub-graph on a miss) when the buffer is
// full, when the material changes, or at the end of the run.
struct DeferBuf {
  uint32_t* ids;      // 64 entries
  uint32_t count;     // wave-uniform
  uint32_t mat;       // wave-uniform
  uint32_t region;    // surrogate queue region of the current run
};

// Evaluate the staged hits (all 64 lanes active on entry).  The lookups are
// repeated: in CACHED mode they may now find values inserted since.
template <int MODE, bool SURR>
__device__ __forceinline__ void flush_deferred(const ShadeArgs& a, DeferBuf& B, const LaneRegs& R,
                                            Counters& cnt) {
  const uint32_t m = B.mat;
  const bool act = (uint32_t)lane_id() < B.count;
  LaneHit L = load_lane(a, B.ids, B.count, 0u);
  uint32_t ins = 0u, slots = 0u;
  uint32_t miss = probe_chunk<MODE, false>(a, act, m, L.h, L.hd, R, cnt, &ins, &slots);
  const bool parked = SURR && surrogate_park<MODE>(a, m, act, L.h, ins, B.region, cnt);
  if (act && !parked)
    shade_full<MODE, true, false>(a, m, L.h, L.hd, R, cnt, miss, ins, slots, no_audit());
  B.count = 0u;
}

// KIND_PROBE: probe first.  Lanes whose lookups all hit run only the hit
// program.  If more than defer_max lanes of the chunk missed, the chunk is
// dense enough to be evaluated in place; otherwise its missing lanes go to the
// wave's staging buffer.
template <int MODE, bool SURR>
__device__ __forceinline__ void chunk_probe(const ShadeArgs& a, const LaneHit& L, LaneIdx next,
                                            LaneHit* Ln, const LaneRegs& R, Counters& cnt,
                                            DeferBuf& B) {
  cnt.v[CNT_HITS] += (uint32_t)L.active;
  uint32_t ins = 0u, slots = 0u;
  uint32_t miss = probe_chunk<MODE, true>(a, L.active, L.mat, L.h, L.hd, R, cnt, &ins, &slots);
  *Ln = fetch_lane(a, next);
  bool deferred = false;
  uint64_t pending = __ballot(L.active);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t m = __builtin_amdgcn_readlane(L.mat, leader);
    const bool mine = L.active && L.mat == m;
    pending &= ~__ballot(mine);
    const uint32_t d = (uint32_t)__popcll(__ballot(mine && miss != 0u));
    const bool dense = d > a.defer_max;
    const bool parked = SURR && dense && surrogate_park<MODE>(a, m, mine, L.h, ins, B.region, cnt);
    if (mine && !parked) {
      if (m < a.n_mats) {
        const PMC_CONST MatHeader* H = as_const(a.hdr) + m;
        if (dense) {
          shade_full<MODE, false, false>(a, m, L.h, L.hd, R, cnt, miss, ins, slots, no_audit());
        } else if (miss != 0u) {
          deferred = true;
        } else {
          cnt.v[CNT_NODES_TOTAL] += H->n_instr;
          run_program<MODE, false, false>(a, m, L.h, L.hd, R, cnt, H->hit_begin, H->n_hit, 0u,
                                          0u, 0u, no_audit());
          write_outputs(a, m, L.h, L.hd, R);
        }
      } else {
        cnt.v[CNT_INVALID]++;
        shade_default(a, L.h, L.hd);
      }
    }
  }
  // stage the deferred lanes, one material at a time (the chunk's own work is done,
  // so a flush may reuse the register file)
  cnt.v[CNT_DEFERRED] += (uint32_t)deferred;
  uint64_t dm = __ballot(deferred);
  while (dm) {
    const int leader = __ffsll((unsigned long long)dm) - 1;
    const uint32_t m = __builtin_amdgcn_readlane(L.mat, leader);
    const bool member = deferred && L.mat == m;
    const uint64_t mm = __ballot(member);
    dm &= ~mm;
    if (B.count != 0u && B.mat != m) flush_deferred<MODE, SURR>(a, B, R, cnt);
    B.mat = m;
    const uint32_t n_new = (uint32_t)__popcll(mm);
    const uint32_t room = 64u - B.count;
    const uint32_t r = (uint32_t)__popcll(mm & lanemask_lt());
    if (member && r < room) B.ids[B.count + r] = L.h;
    if (n_new >= room) {
      B.count = 64u;
      flush_deferred<MODE, SURR>(a, B, R, cnt);
      if (member && r >= room) B.ids[r - room] = L.h;
      B.count = n_new - room;
    } else {
      B.count += n_new;
    }
  }
}

__device__ __forceinline__ void flush_counters(const ShadeArgs& a, Counters& cnt) {
  if (!a.stat_slots) return;
  unsigned long long* slot = a.stat_slots + (uint64_t)(blockIdx.x % kStatSlots) * kStatStride;
#pragma unroll
  for (int q = 0; q < kNumCounters; ++q) {
    uint32_t s = wave_sum(cnt.v[q]);
    if (lane_id() == 0 && s) atomicAdd(slot + q, (unsigned long long)s);
  }
}

// The shading kernels (every thread of the workgroup calls it once, at the
// end): each wave leaves its counter sums in its LDS staging words, free by
// now, and wave 0 adds the workgroup's and takes one atomic per counter, so
// the counters' atomics do not pile up on a few addresses.
__device__ __forceinline__ void flush_counters_block(const ShadeArgs& a, Counters& cnt,
                                                     float* lds) {
  if (!a.stat_slots) return;
  const uint32_t stride = a.n_regs * 64u + 64u;          // floats per wave
  const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t* mine = reinterpret_cast<uint32_t*>(lds + w * stride + a.n_regs * 64u);
#pragma unroll
  for (int q = 0; q < kNumCounters; ++q) {
    const uint32_t s = wave_sum(cnt.v[q]);
    if (lane_id() == 0) mine[q] = s;
  }
  __syncthreads();
  if (w == 0 && lane_id() < kNumCounters) {
    const int q = lane_id();
    unsigned long long t = 0ull;
    for (uint32_t k = 0; k < nw; ++k)
      t += reinterpret_cast<const uint32_t*>(lds + k * stride + a.n_regs * 64u)[q];
    if (t) atomicAdd(a.stat_slots + (uint64_t)(blockIdx.x % kStatSlots) * kStatStride + q, t);
  }
}

// One run = `chunk_waves` consecutive chunks handled by one wave.
template <int MODE, int KIND, bool SURR>
__device__ __forceinline__ void do_run(const ShadeArgs& a, uint32_t first, uint32_t n_chunks,
                                       const LaneRegs& R, Counters& cnt, DeferBuf& B) {
  const uint32_t last = min(first + a.chunk_waves, n_chunks);
  B.region = (first / a.chunk_waves) % kQueueRegions;
  LaneHit L = load_lane(a, a.perm, a.n, first);
  for (uint32_t c = first; c < last; ++c) {
    // index of the next chunk now (its load is in flight during the probes),
    // its hit data once this chunk's probes are consumed
    LaneIdx next;
    next.active = false;
    next.h = 0u;
    if (c + 1u < last) next = lane_index(a.perm, a.n, c + 1u);
    LaneHit Ln;
    if (KIND == KIND_PROBE) chunk_probe<MODE, SURR>(a, L, next, &Ln, R, cnt, B);
    else chunk_full<MODE, SURR>(a, L, next, &Ln, R, cnt, B.region);
    L = Ln;
  }
  if (KIND == KIND_PROBE && B.count != 0u) flush_deferred<MODE, SURR>(a, B, R, cnt);
}

// LDS per wave: the register file [n_regs][64] floats, then 64 staging ids.
__device__ __forceinline__ float* wave_lds(float* lds, const ShadeArgs& a) {
  return lds + (threadIdx.x >> 6) * (a.n_regs * 64 + 64);
}

// STATS = false: the counters are dead code and take no registers.
template <int MODE, int KIND, bool STATS, bool SURR>
__device__ __forceinline__ void shade_flat_body(const ShadeArgs& a) {
  extern __shared__ float lds[];
  float* wl = wave_lds(lds, a);
  LaneRegs R{wl, lane_id()};
  DeferBuf B{reinterpret_cast<uint32_t*>(wl + a.n_regs * 64), 0u, 0u, 0u};
  Counters cnt;
#pragma unroll
  for (int q = 0; q < kNumCounters; ++q) cnt.v[q] = 0u;
  const uint32_t n_chunks = (a.n + 63u) / 64u;
  const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint32_t first = w * a.chunk_waves;
  if (first < n_chunks) do_run<MODE, KIND, SURR>(a, first, n_chunks, R, cnt, B);
  if (STATS) flush_counters_block(a, cnt, lds);
}

// Persistent variant: a fixed grid of waves walks the runs with a static stride
// (no shared work counter: same-address atomics serialise across the XCDs).
// The material sort orders hits by decreasing program length, so the stride
// deals the long programs out first.
template <int MODE, int KIND, bool STATS, bool SURR>
__device__ __forceinline__ void shade_persistent_body(const ShadeArgs& a) {
  extern __shared__ float lds[];
  float* wl = wave_lds(lds, a);
  LaneRegs R{wl, lane_id()};
  DeferBuf B{reinterpret_cast<uint32_t*>(wl + a.n_regs * 64), 0u, 0u, 0u};
  Counters cnt;
#pragma unroll
  for (int q = 0; q < kNumCounters; ++q) cnt.v[q] = 0u;
  const uint32_t n_chunks = (a.n + 63u) / 64u;
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  for (uint32_t first = w * a.chunk_waves; first < n_chunks; first += waves * a.chunk_waves)
    do_run<MODE, KIND, SURR>(a, first, n_chunks, R, cnt, B);
  if (STATS) flush_counters_block(a, cnt, lds);
}

// Kernels.  The cached variants without counters are compiled for 4 waves per
// SIMD (at most 128 VGPRs): the probe-heavy path is latency bound and gains
// more from the extra wave than it loses to a few spilled registers.  The
// uncached and the counting variants keep the compiler's own register budget.
template <int MODE, int KIND, bool STATS, bool SURR>
__global__ __launch_bounds__(256) void k_shade_flat(ShadeArgs a) {
  shade_flat_body<MODE, KIND, STATS, SURR>(a);
}

template <int MODE, int KIND, bool STATS, bool SURR>
__global__ __launch_bounds__(256) void k_shade_persistent(ShadeArgs a) {
  shade_persistent_body<MODE, KIND, STATS, SURR>(a);
}

template <int MODE, int KIND, bool STATS, bool SURR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_shade_flat_w4(ShadeArgs a) {
  shade_flat_body<MODE, KIND, STATS, SURR>(a);
}

template <int MODE, int KIND, bool STATS, bool SURR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_shade_persistent_w4(ShadeArgs a) {
  shade_persistent_body<MODE, KIND, STATS, SURR>(a);
}

// ------------------------------------------------- surrogate second passes ---

// The networks over the queue of parked hits, 64 entries per step of a wave; a
// step whose entries span materials runs each material's network with all
// lanes active and keeps the lanes of that material.
__global__ __launch_bounds__(256) void k_surr_queue(ShadeArgs a) {
  const QueueMap Q = queue_map(a);
  const uint32_t n_chunks = Q.c0 + Q.c1;
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  // contiguous runs of chunks per wave: the queue follows the material order,
  // so a wave reloads its network only where the material changes
  const uint32_t per = (n_chunks + waves - 1u) / waves;
  const uint32_t wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint32_t c_end = min(n_chunks, (wv + 1u) * per);
  NetRegs N;
  uint32_t loaded = 0xFFFFFFFFu;
  for (uint32_t c = wv * per; c < c_end; ++c) {
    bool act;
    const uint64_t idx = queue_entry(a, Q, c, &act);
    const uint32_t h = act ? a.surr_queue[idx].x : 0u;
    const uint32_t mat = act ? a.material[h] : 0xFFFFFFFFu;
    const float2 uv = act ? reinterpret_cast<const float2*>(a.uv)[h] : make_float2(0.f, 0.f);
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    uint64_t pending = __ballot(act);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint32_t m = __builtin_amdgcn_readlane(mat, leader);
      const bool mine = act && mat == m;
      pending &= ~__ballot(mine);
      const uint32_t slot = (as_const(a.hdr) + m)->surr_slot;
      if (slot != loaded) {
        load_net(a.surr_w + slot, N);
        loaded = slot;
      }
      float y[4];
      net_wave(N, uv.x, uv.y, y);
      if (mine) out = make_float4(y[0], y[1], y[2], y[3]);
    }
    if (act) a.surr_val[idx] = out;
  }
}

// Finish pass over the parked hits: probe again, take the networks' values for
// the parked outputs that still miss (or audit them), evaluate the rest.
template <int MODE, bool STATS>
__device__ __forceinline__ void shade_finish_body(const ShadeArgs& a) {
  extern __shared__ float lds[];
  float* wl = wave_lds(lds, a);
  LaneRegs R{wl, lane_id()};
  Counters cnt;
#pragma unroll
  for (int q = 0; q < kNumCounters; ++q) cnt.v[q] = 0u;
  const QueueMap Q = queue_map(a);
  const uint32_t n_chunks = Q.c0 + Q.c1;
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  for (uint32_t c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < n_chunks;
       c += waves) {
    bool act;
    const uint64_t idx = queue_entry(a, Q, c, &act);
    const uint2 e = act ? a.surr_queue[idx] : make_uint2(0u, 0u);
    LaneIdx I;
    I.active = act;
    I.h = e.x;
    const LaneHit L = fetch_lane(a, I);
    const float4 yv = act ? a.surr_val[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t ins = 0u, slots = 0u;
    // the parked outputs missed in the first pass: look up only the others
    uint32_t miss = probe_chunk<MODE, false>(a, act, L.mat, L.h, L.hd, R, cnt, &ins, &slots,
                                             e.y & 0xFFu);
    uint64_t pending = __ballot(act);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint32_t m = __builtin_amdgcn_readlane(L.mat, leader);
      const bool mine = act && L.mat == m;
      pending &= ~__ballot(mine);
      if (mine) {
        Audit au = no_audit();
        surrogate_substitute<MODE>(a, m, L.h, L.hd, e.y & 0xFFu, (e.y & 0x100u) != 0u, yv, R,
                                   cnt, miss, ins, au);
        shade_full<MODE, true, true>(a, m, L.h, L.hd, R, cnt, miss, ins, slots, au);
      }
    }
  }
  if (STATS) flush_counters_block(a, cnt, lds);
}

template <int MODE, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_shade_finish(ShadeArgs a) {
  shade_finish_body<MODE, STATS>(a);
}

hipError_t launch_surr_queue(const ShadeArgs& a, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_queue, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_surr_finish(const ShadeArgs& a, uint32_t grid, hipStream_t s) {
  const size_t lds = shade_lds_bytes(a.n_regs);
  const bool stats = a.stat_slots != nullptr;
  if (a.mode == PMC_MODE_SNAPSHOT) {
    if (stats) hipLaunchKernelGGL((k_shade_finish<PMC_MODE_SNAPSHOT, true>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_shade_finish<PMC_MODE_SNAPSHOT, false>), dim3(grid), dim3(256), lds, s, a);
  } else {
    if (stats) hipLaunchKernelGGL((k_shade_finish<PMC_MODE_CACHED, true>), dim3(grid), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_shade_finish<PMC_MODE_CACHED, false>), dim3(grid), dim3(256), lds, s, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------- host launchers ---

size_t shade_lds_bytes(uint32_t n_regs, uint32_t waves) {
  return (size_t)waves * (n_regs * 64 + 64) * sizeof(float);
}

template <int MODE, int KIND, bool STATS, bool SURR>
static void launch_one(const ShadeArgs& a, bool persistent, dim3 grid, dim3 block, size_t lds,
                       hipStream_t s) {
  // the counting variants keep the compiler's register budget: their 23
  // per-lane counters would spill under the 4-wave cap
  constexpr bool w4 = MODE != PMC_MODE_UNCACHED && !STATS;
  if constexpr (w4) {
    if (persistent)
      hipLaunchKernelGGL((k_shade_persistent_w4<MODE, KIND, STATS, SURR>), grid, block, lds, s, a);
    else
      hipLaunchKernelGGL((k_shade_flat_w4<MODE, KIND, STATS, SURR>), grid, block, lds, s, a);
  } else {
    if (persistent)
      hipLaunchKernelGGL((k_shade_persistent<MODE, KIND, STATS, SURR>), grid, block, lds, s, a);
    else
      hipLaunchKernelGGL((k_shade_flat<MODE, KIND, STATS, SURR>), grid, block, lds, s, a);
  }
}

template <int KIND, bool STATS>
static void launch_kind(const ShadeArgs& a, bool persistent, bool surr, dim3 grid, dim3 block,
                        size_t lds, hipStream_t s) {
  if (a.mode == PMC_MODE_UNCACHED)
    launch_one<PMC_MODE_UNCACHED, KIND, STATS, false>(a, persistent, grid, block, lds, s);
  else if (a.mode == PMC_MODE_CACHED && surr)
    launch_one<PMC_MODE_CACHED, KIND, STATS, true>(a, persistent, grid, block, lds, s);
  else if (a.mode == PMC_MODE_CACHED)
    launch_one<PMC_MODE_CACHED, KIND, STATS, false>(a, persistent, grid, block, lds, s);
  else if (surr)
    launch_one<PMC_MODE_SNAPSHOT, KIND, STATS, true>(a, persistent, grid, block, lds, s);
  else
    launch_one<PMC_MODE_SNAPSHOT, KIND, STATS, false>(a, persistent, grid, block, lds, s);
}

hipError_t launch_shade(const ShadeArgs& a, int kind, bool persistent, bool surr, uint32_t grid,
                        uint32_t block_waves, hipStream_t s) {
  const uint32_t waves = persistent ? 4u : block_waves;
  const size_t lds = shade_lds_bytes(a.n_regs, waves);
  const dim3 g(grid), b(64u * waves);
  const bool stats = a.stat_slots != nullptr;
  if (kind == KIND_PROBE) {
    if (stats) launch_kind<KIND_PROBE, true>(a, persistent, surr, g, b, lds, s);
    else launch_kind<KIND_PROBE, false>(a, persistent, surr, g, b, lds, s);
  } else {
    if (stats) launch_kind<KIND_FULL, true>(a, persistent, surr, g, b, lds, s);
    else launch_kind<KIND_FULL, false>(a, persistent, surr, g, b, lds, s);
  }
  return hipGetLastError();
}

// ------------------------------------------------------- debug key export ---

__global__ void k_debug_keys(ShadeArgs a, pmc_key_record* out) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.n) return;
  const uint32_t m = a.material[h];
  HitData hd;
  const float2 uv = reinterpret_cast<const float2*>(a.uv)[h];
  hd.u = uv.x;
  hd.v = uv.y;
  hd.g = reinterpret_cast<const float4*>(a.duv)[h];
  hd.n = make_float3(0.f, 0.f, 1.f);
  uint32_t n_cach = m < a.n_mats ? a.hdr[m].n_cach : 0u;
  for (uint32_t c = 0; c < 8; ++c) {
    pmc_key_record r;
    r.cell = 0; r.hash2 = 0; r.level = 0; r.tx = 0; r.ty = 0; r.bypass = 2;
    if (c < n_cach) {
      const CachDesc cd = a.cach[a.hdr[m].cach_begin + c];
      Key k = key_of(a, m, h, cd.node_sock, cd.key, hd);
      r.bypass = k.bypass ? 1u : 0u;
      if (!k.bypass) {
        r.cell = k.cell; r.hash2 = k.hash2; r.level = k.level; r.tx = k.tx; r.ty = k.ty;
      }
    }
    out[(uint64_t)h * 8 + c] = r;
  }
}

hipError_t launch_debug_keys(const ShadeArgs& a, pmc_key_record* out, hipStream_t s) {
  hipLaunchKernelGGL(k_debug_keys, dim3((a.n + 255) / 256), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

// ------------------------------------------------- Algorithm 1, raw surface ---

__global__ void k_insert_raw(ShadeArgs a, const uint64_t* k0, const uint64_t* k1,
                             const uint32_t* enc, uint64_t n) {
  Counters cnt;
#pragma unroll
  for (int q = 0; q < kNumCounters; ++q) cnt.v[q] = 0u;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int o = INS_FULL;
  if (i < n) {
    uint32_t cell, hash2;
    raw_hash(k0[i], k1[i], a.cells, a.hash2_mask, &cell, &hash2);
    o = cache_insert(a, cell, hash2, enc[i]);
  }
  count_insert(cnt, i < n, o);
  flush_counters(a, cnt);
}

__global__ void k_lookup_raw(ShadeArgs a, const uint64_t* k0, const uint64_t* k1, uint64_t n,
                             uint32_t* enc_out, uint8_t* hit) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t cell, hash2, code = 0;
  raw_hash(k0[i], k1[i], a.cells, a.hash2_mask, &cell, &hash2);
  uint32_t slot;
  bool f = cache_lookup(a, cell, hash2, &code, &slot);
  hit[i] = f ? 1 : 0;
  enc_out[i] = f ? code : 0u;
}

hipError_t launch_insert_raw(const ShadeArgs& a, const uint64_t* k0, const uint64_t* k1,
                             const uint32_t* enc, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_insert_raw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, k0, k1,
                     enc, n);
  return hipGetLastError();
}

hipError_t launch_lookup_raw(const ShadeArgs& a, const uint64_t* k0, const uint64_t* k1,
                             uint64_t n, uint32_t* enc_out, uint8_t* hit, hipStream_t s) {
  hipLaunchKernelGGL(k_lookup_raw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, k0, k1,
                     n, enc_out, hit);
  return hipGetLastError();
}

}  // namespace pmc
