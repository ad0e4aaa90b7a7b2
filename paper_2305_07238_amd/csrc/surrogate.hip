// surrogate.hip - training, error probe and inference of the per-material
// surrogate networks on the matrix cores (16x16x16 FP16 products, FP32 sums).
//
// Training: a slot's Adam steps all run in one launch, on one workgroup (4
// waves) or, data parallel, on `replicas` workgroups that split every step's
// batch (see below).  A wave takes 32 samples at a time (two 16-sample
// tiles).  The forward and backward passes chain register to register (the
// layout argument is in surrogate.h); the weight gradients contract over the
// samples, which needs the activations with the sample index in the K
// position, so each wave also writes its activations and output gradients
// unit-major into LDS and reads them back as matrix operands.  The four
// waves' gradients are summed into LDS in wave order (deterministic), then
// 256 threads apply Adam to the FP32 master weights and refresh the binary16
// copies in LDS.
#include "device_common.h"
#include "shade.h"
#include "surrogate.h"

namespace pmc {

namespace {

constexpr int kTW = 4;                     // waves per training block
constexpr int kMaxReplicas = 64;           // workgroups per slot (data parallel)
constexpr int kRS = 40;                    // unit-major row stride (halves): 32 samples + pad
constexpr int kS1 = 40, kS2 = 72, kS3T = 4;
constexpr int OFF_W1 = 0;                              // [64][kS1]
constexpr int OFF_W2 = OFF_W1 + 64 * kS1 * 2;          // [64][kS2]  (out, in)
constexpr int OFF_W2T = OFF_W2 + 64 * kS2 * 2;         // [64][kS2]  (in, out)
constexpr int OFF_W3 = OFF_W2T + 64 * kS2 * 2;         // [16][kS2]  rows 4..15 zero
constexpr int OFF_W3T = OFF_W3 + 16 * kS2 * 2;         // [64][4]
constexpr int OFF_B = OFF_W3T + 64 * kS3T * 2;         // 132 floats
constexpr int OFF_G = OFF_B + 132 * 4;                 // gradient sums, kParams floats
constexpr int OFF_RED = OFF_G + ((kParams * 4 + 15) / 16) * 16;
constexpr int OFF_ACT = OFF_RED + 16;
constexpr int ACT_WAVE = (32 + 3 * 64) * kRS * 2;      // Xu, H1u, H2u, Du
constexpr int LDS_TOTAL = OFF_ACT + kTW * ACT_WAVE;
static_assert(OFF_G % 16 == 0 && OFF_ACT % 16 == 0, "LDS alignment");

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float sum16(float x) {       // over the 16 lanes of a row group
  x += __shfl_xor(x, 1, 64);
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 4, 64);
  x += __shfl_xor(x, 8, 64);
  return x;
}

__device__ __forceinline__ float nan_max(float a, float b) {   // NaN wins
  return (b > a || b != b) ? b : a;
}

// Data exchanged between the workgroups of a slot is written with stores
// coherent at device scope (they write through the non-coherent cache
// levels), so a barrier needs no writeback of whole caches: only that those
// stores have completed before the arrival is counted, and, after the wait,
// one invalidation of the workgroup's cached lines before plain loads read
// what the others wrote.
__device__ __forceinline__ void st_dev(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (one thread) until *w >= target; false after `limit` polls.
__device__ __forceinline__ bool spin_until(uint32_t* w, uint32_t target, uint32_t limit) {
  for (uint32_t i = 0; i < limit; ++i) {
    if (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}

// Barrier of a slot's workgroups on one counter: every workgroup adds one per
// barrier, so the b-th barrier of n workgroups ends when the counter reaches
// n * b.  Each wave first waits for its own coherent stores to complete.
// False when the wait gave up (the workgroup agrees through the LDS word `flag`).
__device__ __forceinline__ bool group_barrier(uint32_t* counter, uint32_t target, uint32_t limit,
                                              uint32_t* flag, int tid) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    flag[0] = spin_until(counter, target, limit) ? 0u : 1u;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");     // drop stale cached lines
  }
  __syncthreads();
  const bool ok = flag[0] == 0u;
  __syncthreads();                       // every thread has read the flag before it is reused
  return ok;
}

struct Lds {
  _Float16 *w1, *w2, *w2t, *w3, *w3t;
  float *b, *g, *red;
  uint32_t* flag;                        // one word: a wait of the step failed
  _Float16* act;
};

__device__ __forceinline__ Lds lds_layout(unsigned char* base) {
  Lds L;
  L.w1 = reinterpret_cast<_Float16*>(base + OFF_W1);
  L.w2 = reinterpret_cast<_Float16*>(base + OFF_W2);
  L.w2t = reinterpret_cast<_Float16*>(base + OFF_W2T);
  L.w3 = reinterpret_cast<_Float16*>(base + OFF_W3);
  L.w3t = reinterpret_cast<_Float16*>(base + OFF_W3T);
  L.b = reinterpret_cast<float*>(base + OFF_B);
  L.g = reinterpret_cast<float*>(base + OFF_G);
  L.red = reinterpret_cast<float*>(base + OFF_RED);
  L.flag = reinterpret_cast<uint32_t*>(base + OFF_RED + 8);
  L.act = reinterpret_cast<_Float16*>(base + OFF_ACT);
  return L;
}

// One master parameter -> its binary16 copies (weights) or FP32 copy (biases).
__device__ __forceinline__ void store_param(const Lds& L, int p, float w) {
  const _Float16 h = (_Float16)w;
  if (p < P_B1) {
    L.w1[(p >> 5) * kS1 + (p & 31)] = h;
  } else if (p < P_W2) {
    L.b[p - P_B1] = w;
  } else if (p < P_B2) {
    const int q = p - P_W2, r = q >> 6, c = q & 63;
    L.w2[r * kS2 + c] = h;
    L.w2t[c * kS2 + r] = h;
  } else if (p < P_W3) {
    L.b[64 + p - P_B2] = w;
  } else if (p < P_B3) {
    const int q = p - P_W3, o = q >> 6, c = q & 63;
    L.w3[o * kS2 + c] = h;
    L.w3t[c * kS3T + o] = h;
  } else {
    L.b[128 + p - P_B3] = w;
  }
}

// Inference copy of a slot from its master weights.
__device__ __forceinline__ void export_params(const float* P, SurrW* w, int tid, int nt) {
  for (int p = tid; p < kParams; p += nt) {
    const float x = P[p];
    if (p < P_B1) w->w1[p] = (_Float16)x;
    else if (p < P_W2) w->b1[p - P_B1] = x;
    else if (p < P_B2) w->w2[p - P_W2] = (_Float16)x;
    else if (p < P_W3) w->b2[p - P_B2] = x;
    else if (p < P_B3) w->w3[p - P_W3] = (_Float16)x;
    else w->b3[p - P_B3] = x;
  }
  for (int q = tid; q < 12 * 64; q += nt) w->w3[4 * 64 + q] = (_Float16)0.0f;
}

__device__ __forceinline__ h4 ld_h4(const _Float16* p) { return *reinterpret_cast<const h4*>(p); }

__device__ __forceinline__ void record_target(const pmc_log_record& R, const SurrState* st,
                                              float tg[4], float mk[4]) {
  uint32_t om = R.ordinal < 8u ? st->ordmap[R.ordinal] : 0u;
  const uint32_t base = om & 0xFu, width = (om >> 4) & 0xFu;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint32_t k = (uint32_t)c - base;       // wraps for c < base
    const bool used = k < width;
    mk[c] = used ? 1.0f : 0.0f;
    tg[c] = used ? (k == 0u ? R.value[0] : (k == 1u ? R.value[1] : R.value[2])) : 0.0f;
  }
}

__device__ __forceinline__ pmc_log_record load_record(const pmc_log_record* p) {
  const uint4* q = reinterpret_cast<const uint4*>(p);
  const uint4 a = q[0], b = q[1];
  pmc_log_record R;
  R.material = a.x;
  R.ordinal = a.y;
  R.u = __uint_as_float(a.z);
  R.v = __uint_as_float(a.w);
  R.value[0] = __uint_as_float(b.x);
  R.value[1] = __uint_as_float(b.y);
  R.value[2] = __uint_as_float(b.z);
  R.value[3] = __uint_as_float(b.w);
  return R;
}

}  // namespace

size_t surr_train_lds_bytes() { return (size_t)LDS_TOTAL; }

__global__ __launch_bounds__(256) void k_surr_train(TrainArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Lds L = lds_layout(lds_raw);
  const int tid = (int)threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, g = lane >> 4;

  // replicas > 1: the workgroups r = 0 .. replicas-1 of a slot take the
  // chunks r*4 + wave, r*4 + wave + 4*replicas, ... of each step's batch (the
  // single workgroup's samples, split) and publish their gradient sums; each
  // workgroup then adds the sums of a 1/replicas share of the parameters in
  // replica order and takes the Adam step there, and all read the new
  // parameters back.  The launch is cooperative (every workgroup resident),
  // and every wait is bounded: past its limit a workgroup marks the slot
  // failed (loss NaN) and leaves.
  const uint32_t nrep = a.replicas > 1u ? a.replicas : 1u;
  const uint32_t rep = blockIdx.x % nrep;
  uint32_t slot, begin, n_train;
  if (a.slot_begin) {
    slot = blockIdx.x / nrep;
    begin = a.slot_begin[slot];
    const uint32_t n_total = a.slot_count[slot];
    const uint32_t held = min(a.holdout, n_total / 4u);
    n_train = n_total - held;
    if (tid == 0 && rep == 0u) {
      a.state[slot].n_train = n_train;
      a.state[slot].n_heldout = held;
    }
    if (n_train < a.min_records || n_train == 0u) return;     // uniform over the block
  } else {
    slot = a.slot_fixed;
    begin = 0u;
    n_train = a.n_fixed;
    if (n_train == 0u) return;
  }
  SurrState* st = a.state + slot;
  const pmc_log_record* rec = a.rec + begin;
  // the slot's place in the exchange buffers (one slot per launch without grouping)
  const uint32_t xs = a.slot_begin ? slot : 0u;
  float* P = a.master + (size_t)slot * 3 * kParamStride;
  float* M1 = P + kParamStride;
  float* V1 = P + 2 * kParamStride;

  for (int p = tid; p < kParams; p += 256) store_param(L, p, P[p]);
  for (int q = tid; q < 12 * 64; q += 256) L.w3[(4 + (q >> 6)) * kS2 + (q & 63)] = (_Float16)0.0f;
  const uint32_t step0 = st->steps;
  __syncthreads();

  _Float16* Xu = L.act + wave * (ACT_WAVE / 2);
  _Float16* H1u = Xu + 32 * kRS;
  _Float16* H2u = H1u + 64 * kRS;
  _Float16* Du = H2u + 64 * kRS;
  const h4 z4 = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
  const f4 zf = {0.f, 0.f, 0.f, 0.f};

  const uint32_t steps = a.sample ? a.steps : 1u;
  float last_loss = 0.0f;
  for (uint32_t s = 0; s < steps; ++s) {
    const uint32_t t_step = step0 + s + 1u;
    f4 gw1[4][2], gw2[4][4], gw3[4];
    float gb1[4][4], gb2[4][4], gb3[4];
    float loss = 0.0f, nused = 0.0f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int n = 0; n < 2; ++n) gw1[m][n] = zf;
#pragma unroll
      for (int n = 0; n < 4; ++n) gw2[m][n] = zf;
      gw3[m] = zf;
#pragma unroll
      for (int r = 0; r < 4; ++r) { gb1[m][r] = 0.0f; gb2[m][r] = 0.0f; }
      gb3[m] = 0.0f;
    }
    const uint32_t n_chunks = a.sample ? a.batch / 32u : (n_train + 31u) / 32u;
    // lanes 0..31 hold a chunk's 32 samples (lanes 32..63 repeat them); the
    // records of the wave's next chunk are loaded while this one is processed
    auto record_of = [&](uint32_t c, bool* valid) -> uint32_t {
      const uint32_t i = c * 32u + (uint32_t)(lane & 31);
      if (a.sample) {
        *valid = true;
        return (uint32_t)(mix64(a.seed ^ (((uint64_t)t_step << 32) | i)) % n_train);
      }
      *valid = i < n_train;
      return *valid ? i : 0u;
    };
    bool valid_next = false;
    pmc_log_record R_next;
    if (rep * kTW + (uint32_t)wave < n_chunks)
      R_next = load_record(rec + record_of(rep * kTW + (uint32_t)wave, &valid_next));
    const uint32_t c_first = rep * kTW + (uint32_t)wave, c_step = kTW * nrep;
    for (uint32_t c = c_first; c < n_chunks; c += c_step) {
      const pmc_log_record R = R_next;
      const bool valid = valid_next;
      if (c + c_step < n_chunks) R_next = load_record(rec + record_of(c + c_step, &valid_next));
      float tg[4], mk[4];
      record_target(R, st, tg, mk);
      if (!valid) {
#pragma unroll
        for (int q = 0; q < 4; ++q) mk[q] = 0.0f;
      }
      // ---- forward: features, two hidden layers, output (tile n = samples 16n..16n+15)
      h4 X[2][2];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const float un = __shfl(R.u, 16 * n + j, 64), vn = __shfl(R.v, 16 * n + j, 64);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          X[t][n] = fourier4(un, vn, 4 * t + g);
#pragma unroll
          for (int q = 0; q < 4; ++q) Xu[(16 * t + 4 * g + q) * kRS + 16 * n + j] = X[t][n][q];
        }
      }
      h4 H1[4][2];
      uint32_t mask1 = 0u;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const h4 a0 = ld_h4(L.w1 + (16 * m + j) * kS1 + 4 * g);
        const h4 a1 = ld_h4(L.w1 + (16 * m + j) * kS1 + 16 + 4 * g);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const f4 acc = mfma16(a1, X[1][n], mfma16(a0, X[0][n], zf));
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float zz = acc[q] + L.b[16 * m + 4 * g + q];
            mask1 |= (zz > 0.0f ? 1u : 0u) << ((m * 2 + n) * 4 + q);
            const _Float16 h = (_Float16)fmaxf(zz, 0.0f);
            H1[m][n][q] = h;
            H1u[(16 * m + 4 * g + q) * kRS + 16 * n + j] = h;
          }
        }
      }
      h4 H2[4][2];
      uint32_t mask2 = 0u;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        h4 aw[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) aw[t] = ld_h4(L.w2 + (16 * m + j) * kS2 + 16 * t + 4 * g);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          f4 acc = zf;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc = mfma16(aw[t], H1[t][n], acc);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float zz = acc[q] + L.b[64 + 16 * m + 4 * g + q];
            mask2 |= (zz > 0.0f ? 1u : 0u) << ((m * 2 + n) * 4 + q);
            const _Float16 h = (_Float16)fmaxf(zz, 0.0f);
            H2[m][n][q] = h;
            H2u[(16 * m + 4 * g + q) * kRS + 16 * n + j] = h;
          }
        }
      }
      h4 a3[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a3[t] = ld_h4(L.w3 + j * kS2 + 16 * t + 4 * g);
      // ---- output gradient dY = 2 (y - t) mask (rows 0..3 of the output tile: lanes g = 0)
      h4 dY[2];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        f4 acc = zf;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = mfma16(a3[t], H2[t][n], acc);
        dY[n] = z4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float tn = __shfl(tg[q], 16 * n + j, 64), mn = __shfl(mk[q], 16 * n + j, 64);
          const float y = acc[q] + L.b[128 + q];
          const float d = g == 0 ? mn * (y - tn) : 0.0f;
          loss += d * d;
          nused += g == 0 ? mn : 0.0f;
          const _Float16 dh = (_Float16)(2.0f * d);
          dY[n][q] = dh;
          gb3[q] += (float)dh;
          if (g == 0) Du[q * kRS + 16 * n + j] = dh;
        }
      }
      wave_lds_sync();
      // gW3 += dY^T H2 (K = samples)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const h4 A = j < 4 ? ld_h4(Du + j * kRS + 16 * kb + 4 * g) : z4;
#pragma unroll
        for (int nn = 0; nn < 4; ++nn)
          gw3[nn] = mfma16(A, ld_h4(H2u + (16 * nn + j) * kRS + 16 * kb + 4 * g), gw3[nn]);
      }
      // dH2 = (W3^T dY) * [a2 > 0]
      h4 dH2[4][2];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const h4 A = g == 0 ? ld_h4(L.w3t + (16 * m + j) * kS3T) : z4;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const f4 acc = mfma16(A, dY[n], zf);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool on = (mask2 >> ((m * 2 + n) * 4 + q)) & 1u;
            const _Float16 dh = (_Float16)(on ? acc[q] : 0.0f);
            dH2[m][n][q] = dh;
            gb2[m][q] += (float)dh;
          }
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int q = 0; q < 4; ++q) Du[(16 * m + 4 * g + q) * kRS + 16 * n + j] = dH2[m][n][q];
      wave_lds_sync();
      // gW2 += dH2^T H1
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        h4 B[4];
#pragma unroll
        for (int nn = 0; nn < 4; ++nn) B[nn] = ld_h4(H1u + (16 * nn + j) * kRS + 16 * kb + 4 * g);
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          const h4 A = ld_h4(Du + (16 * mm + j) * kRS + 16 * kb + 4 * g);
#pragma unroll
          for (int nn = 0; nn < 4; ++nn) gw2[mm][nn] = mfma16(A, B[nn], gw2[mm][nn]);
        }
      }
      // dH1 = (W2^T dH2) * [a1 > 0]
      h4 dH1[4][2];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        h4 aw[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) aw[t] = ld_h4(L.w2t + (16 * m + j) * kS2 + 16 * t + 4 * g);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          f4 acc = zf;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc = mfma16(aw[t], dH2[t][n], acc);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool on = (mask1 >> ((m * 2 + n) * 4 + q)) & 1u;
            const _Float16 dh = (_Float16)(on ? acc[q] : 0.0f);
            dH1[m][n][q] = dh;
            gb1[m][q] += (float)dh;
          }
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int q = 0; q < 4; ++q) Du[(16 * m + 4 * g + q) * kRS + 16 * n + j] = dH1[m][n][q];
      wave_lds_sync();
      // gW1 += dH1^T X
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        h4 B[2];
#pragma unroll
        for (int nn = 0; nn < 2; ++nn) B[nn] = ld_h4(Xu + (16 * nn + j) * kRS + 16 * kb + 4 * g);
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          const h4 A = ld_h4(Du + (16 * mm + j) * kRS + 16 * kb + 4 * g);
#pragma unroll
          for (int nn = 0; nn < 2; ++nn) gw1[mm][nn] = mfma16(A, B[nn], gw1[mm][nn]);
        }
      }
      wave_lds_sync();
    }

    // ---- sum the waves' gradients into LDS, wave 0 first (deterministic order)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        gb1[m][q] = sum16(gb1[m][q]);
        gb2[m][q] = sum16(gb2[m][q]);
      }
      gb3[m] = sum16(gb3[m]);
    }
    loss = wave_sum_f(loss);
    nused = wave_sum_f(nused);
    for (int w = 0; w < kTW; ++w) {
      if (wave == w) {
        const bool first = w == 0;
        auto add = [&](int idx, float v) { L.g[idx] = first ? v : L.g[idx] + v; };
#pragma unroll
        for (int mm = 0; mm < 4; ++mm)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = 16 * mm + 4 * g + q;
#pragma unroll
            for (int nn = 0; nn < 2; ++nn) add(P_W1 + row * 32 + 16 * nn + j, gw1[mm][nn][q]);
#pragma unroll
            for (int nn = 0; nn < 4; ++nn) add(P_W2 + row * 64 + 16 * nn + j, gw2[mm][nn][q]);
          }
        if (g == 0) {
#pragma unroll
          for (int nn = 0; nn < 4; ++nn)
#pragma unroll
            for (int q = 0; q < 4; ++q) add(P_W3 + q * 64 + 16 * nn + j, gw3[nn][q]);
        }
        if (j == 0) {
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              add(P_B1 + 16 * m + 4 * g + q, gb1[m][q]);
              add(P_B2 + 16 * m + 4 * g + q, gb2[m][q]);
            }
        }
        if (lane == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) add(P_B3 + q, gb3[q]);
          L.red[0] = first ? loss : L.red[0] + loss;
          L.red[1] = first ? nused : L.red[1] + nused;
        }
      }
      __syncthreads();
    }
    // ---- Adam on the master weights (or the gradient itself)
    const float inv = 1.0f / fmaxf(L.red[1], 1.0f);
    if (!a.sample) {
      for (int p = tid; p < kParams; p += 256) a.grad_out[p] = L.g[p] * inv;
      if (tid == 0) *a.loss_out = L.red[0] * inv;
    } else if (nrep > 1u) {
      // ---- data parallel: every workgroup publishes its sums; each then adds,
      // in replica order, the sums of its own share of the parameters, takes
      // the Adam step there, and reads the whole step back after all are done
      const float lr = a.lr_end > 0.0f && steps > 1u
                           ? a.lr * powf(a.lr_end / a.lr, (float)s / (float)(steps - 1u))
                           : a.lr;
      const float bc1 = 1.0f - powf(0.9f, (float)t_step);
      const float bc2 = 1.0f - powf(0.999f, (float)t_step);
      float* part = a.partial + ((size_t)xs * nrep + rep) * kPartial;
      for (int p = tid; p < kParams; p += 256) st_dev(part + p, L.g[p]);
      if (tid < 2) st_dev(part + kParams + tid, L.red[tid]);
      if (!group_barrier(a.sync + 2 * xs, nrep * (2u * s + 1u), a.spin_limit, L.flag, tid)) {
        if (tid == 0) st->loss = __int_as_float(0x7FC00000);
        return;
      }
      const float* base = a.partial + (size_t)xs * nrep * kPartial;
      float lsum = 0.0f, nsum = 0.0f;
      for (uint32_t r = 0; r < nrep; ++r) {
        lsum += base[(size_t)r * kPartial + kParams];
        nsum += base[(size_t)r * kPartial + kParams + 1];
      }
      const float dinv = 1.0f / fmaxf(nsum, 1.0f);
      const int per = (kParams + (int)nrep - 1) / (int)nrep;
      const int p0 = (int)rep * per, p1 = min(kParams, p0 + per);
      for (int p = p0 + tid; p < p1; p += 256) {
        float sum = 0.0f;
#pragma unroll
        for (int r = 0; r < kMaxReplicas; ++r)
          if ((uint32_t)r < nrep) sum += base[(size_t)r * kPartial + p];
        const float gr = sum * dinv;
        const float m = 0.9f * M1[p] + 0.1f * gr;
        const float v = 0.999f * V1[p] + 0.001f * gr * gr;
        st_dev(P + p, P[p] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f));
        M1[p] = m;
        V1[p] = v;
      }
      last_loss = lsum * dinv;
      if (!group_barrier(a.sync + 2 * xs, nrep * (2u * s + 2u), a.spin_limit, L.flag, tid)) {
        if (tid == 0) st->loss = __int_as_float(0x7FC00000);
        return;
      }
      for (int p = tid; p < kParams; p += 256) store_param(L, p, P[p]);
    } else {
      const float lr = a.lr_end > 0.0f && steps > 1u
                           ? a.lr * powf(a.lr_end / a.lr, (float)s / (float)(steps - 1u))
                           : a.lr;
      const float bc1 = 1.0f - powf(0.9f, (float)t_step);
      const float bc2 = 1.0f - powf(0.999f, (float)t_step);
      for (int p = tid; p < kParams; p += 256) {
        const float gr = L.g[p] * inv;
        const float m = 0.9f * M1[p] + 0.1f * gr;
        const float v = 0.999f * V1[p] + 0.001f * gr * gr;
        const float w = P[p] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
        P[p] = w;
        M1[p] = m;
        V1[p] = v;
        store_param(L, p, w);
      }
      last_loss = L.red[0] * inv;
    }
    __syncthreads();
  }
  if (rep != 0u) return;
  // the other workgroups' parameter stores: drop any stale cached copy first
  if (nrep > 1u) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (a.sample) {
    export_params(P, a.w + slot, tid, 256);
    if (tid == 0) {
      st->steps = step0 + steps;
      st->loss = last_loss;
    }
  }
}

hipError_t prepare_surrogate_kernels() {
  return hipFuncSetAttribute((const void*)k_surr_train,
                             hipFuncAttributeMaxDynamicSharedMemorySize, LDS_TOTAL);
}

hipError_t launch_surr_train(const TrainArgs& a, uint32_t n_blocks, hipStream_t s) {
  if (a.replicas > 1u) {
    // every workgroup of a slot must be resident for its waits to end
    TrainArgs args = a;
    void* params[] = {&args};
    return hipLaunchCooperativeKernel((const void*)k_surr_train, dim3(n_blocks * a.replicas),
                                      dim3(256), params, LDS_TOTAL, s);
  }
  hipLaunchKernelGGL(k_surr_train, dim3(n_blocks), dim3(256), LDS_TOTAL, s, a);
  return hipGetLastError();
}

uint32_t surr_train_capacity() {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0u;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0u;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_surr_train, 256,
                                                   LDS_TOTAL) != hipSuccess)
    return 0u;
  return (uint32_t)(per_cu * cus);
}

__global__ __launch_bounds__(256) void k_surr_export(const float* master, SurrW* w) {
  export_params(master + (size_t)blockIdx.x * 3 * kParamStride, w + blockIdx.x, (int)threadIdx.x,
                256);
}

hipError_t launch_surr_export(const float* master, SurrW* w, uint32_t n_slots, hipStream_t s) {
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_surr_export, dim3(n_slots), dim3(256), 0, s, master, w);
  return hipGetLastError();
}

// Held-out error of each slot (block per slot): max and mean absolute error
// over the used channels of the last `held` records of its group; sets trust.
__global__ __launch_bounds__(256) void k_surr_probe(const pmc_log_record* rec,
                                                     const uint32_t* slot_begin,
                                                     const uint32_t* slot_count, uint32_t holdout,
                                                     uint32_t min_records, const SurrW* w,
                                                     SurrState* state) {
  __shared__ float s_max[4], s_sum[4], s_cnt[4];
  const uint32_t slot = blockIdx.x;
  const int tid = (int)threadIdx.x, wave = tid >> 6, lane = tid & 63;
  SurrState* st = state + slot;
  const uint32_t n_total = slot_count[slot];
  const uint32_t held = min(holdout, n_total / 4u);
  const uint32_t n_train = n_total - held;
  if (n_train < min_records || n_train == 0u || held == 0u) {
    if (tid == 0) {
      st->trusted = 0u;
      st->max_err = -1.0f;
      st->mean_err = -1.0f;
      st->live_err_bits = 0u;
      st->live_n = 0u;
    }
    return;
  }
  const pmc_log_record* base = rec + slot_begin[slot] + n_train;
  float emax = 0.0f, esum = 0.0f, ecnt = 0.0f;
  NetRegs N;
  load_net(w + slot, N);
  for (uint32_t c = (uint32_t)wave; c * 64u < held; c += 4u) {
    const uint32_t i = c * 64u + (uint32_t)lane;
    const bool valid = i < held;
    const pmc_log_record R = load_record(base + (valid ? i : 0u));
    float y[4];
    net_wave(N, R.u, R.v, y);
    float tg[4], mk[4];
    record_target(R, st, tg, mk);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (valid && mk[q] != 0.0f) {
        const float e = fabsf(y[q] - tg[q]);
        emax = nan_max(emax, e);
        esum += e;
        ecnt += 1.0f;
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) emax = nan_max(emax, __shfl_xor(emax, o, 64));
  esum = wave_sum_f(esum);
  ecnt = wave_sum_f(ecnt);
  if (lane == 0) {
    s_max[wave] = emax;
    s_sum[wave] = esum;
    s_cnt[wave] = ecnt;
  }
  __syncthreads();
  if (tid == 0) {
    float mx = s_max[0], sm = s_sum[0], ct = s_cnt[0];
    for (int q = 1; q < 4; ++q) {
      mx = nan_max(mx, s_max[q]);
      sm += s_sum[q];
      ct += s_cnt[q];
    }
    st->max_err = mx;
    st->mean_err = ct > 0.0f ? sm / ct : -1.0f;
    st->trusted = (ct > 0.0f && mx <= st->thresh) ? 1u : 0u;
    st->live_err_bits = 0u;
    st->live_n = 0u;
  }
}

hipError_t launch_surr_probe(const pmc_log_record* rec, const uint32_t* slot_begin,
                             const uint32_t* slot_count, uint32_t holdout, uint32_t min_records,
                             const SurrW* w, SurrState* state, uint32_t n_slots, hipStream_t s) {
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_surr_probe, dim3(n_slots), dim3(256), 0, s, rec, slot_begin, slot_count,
                     holdout, min_records, w, state);
  return hipGetLastError();
}

// Network outputs at n points: a grid of waves, each holding the network in
// its registers and striding over 16-point tiles.
constexpr uint32_t kInferMaxBlocks = 1024;

__global__ __launch_bounds__(256) void k_surr_infer(const SurrW* w, const float* uv, uint32_t n,
                                                    float* y) {
  const uint32_t tiles = (n + 15u) / 16u;
  const uint32_t waves = gridDim.x * 4u;
  uint32_t t = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (t >= tiles) return;                            // whole waves only
  NetRegs N;
  load_net(w, N);
  const uint32_t j = threadIdx.x & 15u;
  const bool lead = (threadIdx.x & 63u) < 16u;
  const float2* uv2 = reinterpret_cast<const float2*>(uv);
  // two tiles per step (t and t + waves): their products and the vector work
  // of their features and activations are independent, so the matrix core
  // works on one tile while the vector ALU works on the other
  const uint32_t step = 2u * waves;
#pragma unroll 1
  for (; t < tiles; t += step) {
    const uint32_t ia = t * 16u + j, ib = (t + waves) * 16u + j;
    const bool has_b = t + waves < tiles;
    const float2 pa = ia < n ? uv2[ia] : make_float2(0.f, 0.f);
    const float2 pb = has_b && ib < n ? uv2[ib] : make_float2(0.f, 0.f);
    const f4 Ya = net_tile(N, pa.x, pa.y);
    const f4 Yb = net_tile(N, pb.x, pb.y);
    if (lead && ia < n) reinterpret_cast<float4*>(y)[ia] = make_float4(Ya.x, Ya.y, Ya.z, Ya.w);
    if (lead && has_b && ib < n)
      reinterpret_cast<float4*>(y)[ib] = make_float4(Yb.x, Yb.y, Yb.z, Yb.w);
  }
}

hipError_t launch_surr_infer(const SurrW* w, const float* uv, uint32_t n, float* y,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t tiles = (n + 15u) / 16u;
  const uint32_t blocks = min((tiles + 3u) / 4u, kInferMaxBlocks);
  hipLaunchKernelGGL(k_surr_infer, dim3(blocks), dim3(256), 0, s, w, uv, n, y);
  return hipGetLastError();
}

__global__ void k_surr_set_trust(SurrState* state, uint32_t slot, uint32_t trusted,
                                 uint32_t reset_steps) {
  if (threadIdx.x == 0) {
    state[slot].trusted = trusted;
    if (reset_steps) state[slot].steps = 0u;
    state[slot].live_err_bits = 0u;
    state[slot].live_n = 0u;
  }
}

hipError_t launch_surr_set_trust(SurrState* state, uint32_t slot, uint32_t trusted,
                                 uint32_t reset_steps, hipStream_t s) {
  hipLaunchKernelGGL(k_surr_set_trust, dim3(1), dim3(64), 0, s, state, slot, trusted,
                     reset_steps);
  return hipGetLastError();
}

// After a shading call: a slot whose audited error exceeds its threshold
// (or is not a number) loses its trust.
__global__ void k_surr_live_update(SurrState* state, uint32_t n_slots) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slots) return;
  SurrState* st = state + s;
  if (st->trusted && st->live_n && !(__uint_as_float(st->live_err_bits) <= st->thresh))
    st->trusted = 0u;
}

hipError_t launch_surr_live_update(SurrState* state, uint32_t n_slots, hipStream_t s) {
  if (n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_surr_live_update, dim3((n_slots + 255) / 256), dim3(256), 0, s, state,
                     n_slots);
  return hipGetLastError();
}

// ------------------------------------------------------ grouping the log ---
// One block per log region.  Counts per network are kept in LDS and reach
// global memory with one atomic per (region, network); the scatter reserves a
// range per (region, network) the same way and places records with LDS atomics.

constexpr uint32_t kGroupThreads = 1024;
constexpr uint32_t kGroupMaxSlots = 16384;           // 64 KiB of LDS counters

__global__ __launch_bounds__(1024) void k_log_count(const pmc_log_record* log,
                                                     const uint32_t* region_count,
                                                     uint32_t region_cap, const uint32_t* mat_slot,
                                                     uint32_t n_mats, uint32_t n_slots,
                                                     uint32_t* slot_count) {
  extern __shared__ uint32_t cnt[];
  for (uint32_t k = threadIdx.x; k < n_slots; k += blockDim.x) cnt[k] = 0u;
  __syncthreads();
  const uint32_t region = blockIdx.x;
  const uint32_t n = min(region_count[region], region_cap);
  const pmc_log_record* base = log + (uint64_t)region * region_cap;
  for (uint32_t p = threadIdx.x; p < n; p += blockDim.x) {
    const uint32_t mat = base[p].material;
    const uint32_t sl = mat < n_mats ? mat_slot[mat] : 0xFFFFFFFFu;
    if (sl < n_slots) atomicAdd(cnt + sl, 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < n_slots; k += blockDim.x)
    if (cnt[k]) atomicAdd(slot_count + k, cnt[k]);
}

__global__ __launch_bounds__(1024) void k_log_scatter(const pmc_log_record* log,
                                                       const uint32_t* region_count,
                                                       uint32_t region_cap, const uint32_t* mat_slot,
                                                       uint32_t n_mats, uint32_t n_slots,
                                                       uint32_t* cursor, pmc_log_record* grouped) {
  extern __shared__ uint32_t cnt[];
  for (uint32_t k = threadIdx.x; k < n_slots; k += blockDim.x) cnt[k] = 0u;
  __syncthreads();
  const uint32_t region = blockIdx.x;
  const uint32_t n = min(region_count[region], region_cap);
  const pmc_log_record* base = log + (uint64_t)region * region_cap;
  for (uint32_t p = threadIdx.x; p < n; p += blockDim.x) {
    const uint32_t mat = base[p].material;
    const uint32_t sl = mat < n_mats ? mat_slot[mat] : 0xFFFFFFFFu;
    if (sl < n_slots) atomicAdd(cnt + sl, 1u);
  }
  __syncthreads();
  // reserve this region's range of every network; cnt becomes the local cursor
  for (uint32_t k = threadIdx.x; k < n_slots; k += blockDim.x)
    if (cnt[k]) cnt[k] = atomicAdd(cursor + k, cnt[k]);
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < n; p += blockDim.x) {
    const pmc_log_record* src = base + p;
    const uint32_t mat = src->material;
    const uint32_t sl = mat < n_mats ? mat_slot[mat] : 0xFFFFFFFFu;
    if (sl >= n_slots) continue;
    const uint32_t pos = atomicAdd(cnt + sl, 1u);
    const uint4* q = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(grouped + pos);
    d[0] = q[0];
    d[1] = q[1];
  }
}

hipError_t launch_log_group(const pmc_log_record* log, const uint32_t* region_count,
                            uint32_t region_cap, const uint32_t* mat_slot, uint32_t n_mats,
                            uint32_t n_slots, uint32_t* slot_count, uint32_t* slot_begin,
                            uint32_t* slot_cursor, uint32_t* scan_sums, pmc_log_record* grouped,
                            hipStream_t s) {
  if (n_slots == 0) return hipSuccess;
  if (n_slots > kGroupMaxSlots) return hipErrorInvalidValue;
  hipError_t e = launch_fill_u32(slot_count, 0u, n_slots, s);
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)n_slots * 4;
  hipLaunchKernelGGL(k_log_count, dim3(64), dim3(kGroupThreads), lds, s, log, region_count,
                     region_cap, mat_slot, n_mats, n_slots, slot_count);
  e = launch_exclusive_scan(slot_count, n_slots, slot_begin, slot_cursor, scan_sums, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_log_scatter, dim3(64), dim3(kGroupThreads), lds, s, log, region_count,
                     region_cap, mat_slot, n_mats, n_slots, slot_cursor, grouped);
  return hipGetLastError();
}

}  // namespace pmc
