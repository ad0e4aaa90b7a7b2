// surrogate.h - the per-material surrogate network: device layout, the
// wave-wide forward pass on the matrix cores, and host launchers.
//
// Beyond the paper (which stores exact sub-graph values only, Sec. 3): a
// 32 -> 64 -> 64 -> 4 ReLU network of Fourier features of UV may replace the
// deepest cacheable sub-graphs of a material on a cache miss.
//
// Matrix-core mapping (gfx950, wave64).  For a 16x16 tile with K = 16
// (v_mfma_f32_16x16x16_f16) the operand layouts are
//   A[i][k]: lane i + 16 (k / 4), element k % 4
//   B[k][j]: lane j + 16 (k / 4), element k % 4
//   D[i][j]: lane j + 16 (i / 4), element i % 4
// so D of one product is, lane for lane, the B operand of the next one when
// the samples run along j.  Every layer is therefore computed transposed,
// H^T = W X^T: weights are the A operand, activations stay in registers from
// layer to layer.  Inference uses the K = 32 product (NetRegs below); training
// keeps the K = 16 one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pmc.h"

namespace pmc {

constexpr int kFeat = 32, kHid = 64, kOut = 4;
constexpr int kParams = 6532;
// offsets of the flat parameter vector
constexpr int P_W1 = 0, P_B1 = 2048, P_W2 = 2112, P_B2 = 6208, P_W3 = 6272, P_B3 = 6528;
constexpr int kParamStride = 6656;   // floats per parameter block (params, m, v) of a slot
constexpr uint64_t kSeedAudit = 0xD6E8FEB86659FD93ull;

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Inference copy of one slot: binary16 weights [out][in] row-major, FP32 biases.
struct SurrW {
  _Float16 w1[64 * 32];
  _Float16 w2[64 * 64];
  _Float16 w3[16 * 64];        // rows 4..15 zero (the output tile is 16 rows)
  float b1[64], b2[64], b3[4];
  float pad[124];
};
static_assert(sizeof(SurrW) == 15360, "SurrW layout");

// Per-slot state (device), 128 bytes.
struct SurrState {
  uint32_t trusted, steps, n_train, n_heldout;
  float max_err, mean_err, loss;
  uint32_t live_err_bits;      // largest audited error (bits of a float >= 0)
  uint32_t live_n;             // audited outputs
  uint32_t material;
  uint32_t ordmap[8];          // per ordinal: bits 0-3 first channel, bits 4-7 width (0: none)
  float thresh;                // trust threshold
  uint32_t pad[13];
};
static_assert(sizeof(SurrState) == 128, "SurrState layout");


__device__ __forceinline__ f4 mfma16(h4 a, h4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// Features 4q .. 4q+3: sin and cos of w_q u and of w_q v, w_q = 2 pi 2^(q-4).
// sin(2 pi 2^(q-4) u) = sinpi(2^(q-3) u); the scaling by a power of two is exact.
__device__ __forceinline__ h4 fourier4(float u, float v, int q) {
  const float s = __builtin_ldexpf(1.0f, q - 3);
  float su, cu, sv, cv;
  sincospif(u * s, &su, &cu);
  sincospif(v * s, &sv, &cv);
  h4 r;
  r.x = (_Float16)su;
  r.y = (_Float16)cu;
  r.z = (_Float16)sv;
  r.w = (_Float16)cv;
  return r;
}

// One network held in the registers of a wave (loaded once, used for many
// 16-point tiles), for v_mfma_f32_16x16x32_f16.  A K = 32 product pairs two
// 16-row blocks of its input: lane group g = lane / 16 supplies, as its 8 K
// elements, rows 4g .. 4g+3 of the first block and rows 4g .. 4g+3 of the
// second, which is exactly what the D layout of the previous product leaves in
// its registers.  The weights are loaded with the same pairing, and since the
// A and B operands of a product index K the same way, each product still sums
// over all 32 rows.  (Layer 1 reads features: there lane group g supplies
// features 8g .. 8g+7, and W1 is read with the same columns.)  Per tile: 4 products for layer 1, 8 for layer 2, 2 for
// layer 3.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma32(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ h8 cat8(h4 lo, h4 hi) {
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

struct NetRegs {
  h8 w1[4];        // layer 1, M tile m: W1[16m + j][8g .. 8g+7] (the features of fourier8)
  h8 w2[4][2];     // layer 2, M tile m, K step t: input blocks 2t and 2t+1
  h8 w3[2];        // layer 3 (rows 4..15 zero), K step t
  f4 b1[4], b2[4]; // biases of rows 16m + 4g .. 16m + 4g+3
  float b3[4];
};

__device__ __forceinline__ h8 load_pair(const _Float16* row, int b0, int b1, int g) {
  return cat8(*reinterpret_cast<const h4*>(row + 16 * b0 + 4 * g),
              *reinterpret_cast<const h4*>(row + 16 * b1 + 4 * g));
}

__device__ __forceinline__ void load_net(const SurrW* __restrict__ W, NetRegs& N) {
  const int lane = (int)(threadIdx.x & 63u);
  const int j = lane & 15, g = lane >> 4;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    N.w1[m] = *reinterpret_cast<const h8*>(W->w1 + (16 * m + j) * 32 + 8 * g);
    N.w2[m][0] = load_pair(W->w2 + (16 * m + j) * 64, 0, 1, g);
    N.w2[m][1] = load_pair(W->w2 + (16 * m + j) * 64, 2, 3, g);
    N.b1[m] = *reinterpret_cast<const f4*>(W->b1 + 16 * m + 4 * g);
    N.b2[m] = *reinterpret_cast<const f4*>(W->b2 + 16 * m + 4 * g);
  }
  N.w3[0] = load_pair(W->w3 + j * 64, 0, 1, g);
  N.w3[1] = load_pair(W->w3 + j * 64, 2, 3, g);
#pragma unroll
  for (int c = 0; c < 4; ++c) N.b3[c] = W->b3[c];
}

// Features 8g .. 8g+7 (frequencies q = 2g and 2g + 1) for inference: the sines
// and cosines of the higher frequency come from the lower one by the double
// angle, sin 2x = 2 sin x cos x and cos 2x = (cos x - sin x)(cos x + sin x),
// one sin/cos pair per coordinate instead of two.  In binary32 the doubled
// values carry a few units in the last place more error than direct ones; after
// rounding to binary16 a feature rarely moves, and then by one binary16 unit.
__device__ __forceinline__ h8 fourier8(float u, float v, int g) {
  const float s = __builtin_ldexpf(1.0f, 2 * g - 3);
  float su, cu, sv, cv;
  sincospif(u * s, &su, &cu);
  sincospif(v * s, &sv, &cv);
  h8 r;
  r[0] = (_Float16)su;
  r[1] = (_Float16)cu;
  r[2] = (_Float16)sv;
  r[3] = (_Float16)cv;
  r[4] = (_Float16)(2.0f * su * cu);
  r[5] = (_Float16)((cu - su) * (cu + su));
  r[6] = (_Float16)(2.0f * sv * cv);
  r[7] = (_Float16)((cv - sv) * (cv + sv));
  return r;
}

// relu(acc) rounded to binary16 (round to nearest even).  Rounding is
// monotone and keeps zero, so the ReLU is taken after the rounding, on packed
// halves (a negative input may become -0, which adds nothing to the products).
__device__ __forceinline__ h4 relu_h4(f4 acc) {
  const h4 r = __builtin_convertvector(acc, h4);
  const h4 z = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
  return __builtin_elementwise_max(r, z);
}

// The network at 16 points: lane (j, g) gives the coordinates of point j; lanes
// 0..15 receive their point's 4 outputs (rows 0..3 of the output tile).
__device__ __forceinline__ f4 net_tile(const NetRegs& N, float un, float vn) {
  const int g = (int)((threadIdx.x & 63u) >> 4);
  const h8 x = fourier8(un, vn, g);
  // the biases start the accumulators (the D layout of row i is that of bias i)
  h4 H1[4], H2[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) H1[m] = relu_h4(mfma32(N.w1[m], x, N.b1[m]));
  const h8 p0 = cat8(H1[0], H1[1]), p1 = cat8(H1[2], H1[3]);
#pragma unroll
  for (int m = 0; m < 4; ++m)
    H2[m] = relu_h4(mfma32(N.w2[m][1], p1, mfma32(N.w2[m][0], p0, N.b2[m])));
  const f4 b3 = {N.b3[0], N.b3[1], N.b3[2], N.b3[3]};
  return mfma32(N.w3[1], cat8(H2[2], H2[3]), mfma32(N.w3[0], cat8(H2[0], H2[1]), b3));
}

// The network at 64 points, one per lane (all 64 lanes must be active): lane l
// gives (u, v) and receives y[0..3] of its own point.
__device__ __forceinline__ void net_wave(const NetRegs& N, float u, float v, float y[4]) {
  const int lane = (int)(threadIdx.x & 63u);
  const int j = lane & 15, g = lane >> 4;
  y[0] = y[1] = y[2] = y[3] = 0.0f;
#pragma unroll 1
  for (int n = 0; n < 4; ++n) {
    const float un = __shfl(u, 16 * n + j, 64), vn = __shfl(v, 16 * n + j, 64);
    const f4 Y = net_tile(N, un, vn);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float t = __shfl(Y[c], j, 64);
      y[c] = (g == n) ? t : y[c];
    }
  }
}

__device__ __forceinline__ float pick4(const float y[4], uint32_t c) {
  return c == 0u ? y[0] : (c == 1u ? y[1] : (c == 2u ? y[2] : y[3]));
}

// Audit rule: 1 in 64 surrogate-eligible hits are evaluated by the graph.
__device__ __forceinline__ bool surrogate_audited(uint32_t frame, uint32_t h) {
  uint64_t z = ((((uint64_t)frame) << 32) | (uint64_t)h) ^ kSeedAudit;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (z >> 58) == 0ull;
}

// ------------------------------------------------------------- launchers ---

struct TrainArgs {
  const pmc_log_record* rec;   // records (grouped by slot when slot_begin is set)
  const uint32_t* slot_begin;  // per slot: first record; NULL: 0
  const uint32_t* slot_count;  // per slot: records; NULL: n_fixed
  uint32_t n_fixed;
  uint32_t slot_fixed;         // slot of block 0 when slot_begin is NULL
  uint32_t holdout;            // grouped mode: held-out records per slot (capped at a quarter)
  uint32_t min_records;        // grouped mode: fewer training records -> slot skipped
  float* master;               // [slot][3][kParamStride]: params, Adam m, Adam v
  SurrW* w;                    // [slot] inference copies (written at the end)
  SurrState* state;            // [slot]
  uint32_t steps, batch;       // batch: multiple of 128
  float lr, lr_end;             // lr_end > 0: geometric decay over the call's steps
  uint64_t seed;
  uint32_t sample;             // 1: Adam steps on sampled batches; 0: one gradient pass
  float* grad_out;             // gradient pass: 6532 FP32
  float* loss_out;             // gradient pass: loss
  // data parallel (replicas > 1, sample = 1 only): workgroups per slot, their
  // published gradient sums [slot][replica][kPartial], and per slot two
  // words, zero at launch: arrivals and the published step
  uint32_t replicas;
  float* partial;
  uint32_t* sync;
  uint32_t spin_limit;         // polls before a wait gives up
};
constexpr int kPartial = 6536;   // kParams gradient sums, loss, samples, padding

size_t surr_train_lds_bytes();
// n_blocks slots (replicas workgroups each, launched cooperatively when more than one)
hipError_t launch_surr_train(const TrainArgs& a, uint32_t n_blocks, hipStream_t s);
// training workgroups that can be resident at once on the current device
uint32_t surr_train_capacity();
hipError_t launch_surr_export(const float* master, SurrW* w, uint32_t n_slots, hipStream_t s);
// held-out error -> trust, per slot (grouped records)
hipError_t launch_surr_probe(const pmc_log_record* rec, const uint32_t* slot_begin,
                             const uint32_t* slot_count, uint32_t holdout, uint32_t min_records,
                             const SurrW* w, SurrState* state, uint32_t n_slots, hipStream_t s);
hipError_t launch_surr_infer(const SurrW* w, const float* uv, uint32_t n, float* y,
                             hipStream_t s);
// trust flag of one slot (and its audit record cleared); reset_steps also zeroes the step count
hipError_t launch_surr_set_trust(SurrState* state, uint32_t slot, uint32_t trusted,
                                 uint32_t reset_steps, hipStream_t s);
hipError_t launch_surr_live_update(SurrState* state, uint32_t n_slots, hipStream_t s);
// group the insert log by slot: counts, offsets (exclusive scan) and the grouped copy
hipError_t launch_log_group(const pmc_log_record* log, const uint32_t* region_count,
                            uint32_t region_cap, const uint32_t* mat_slot, uint32_t n_mats,
                            uint32_t n_slots, uint32_t* slot_count, uint32_t* slot_begin,
                            uint32_t* slot_cursor, uint32_t* scan_sums, pmc_log_record* grouped,
                            hipStream_t s);

}  // namespace pmc
