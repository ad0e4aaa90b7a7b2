// snapshot.hip - deterministic application of a batch's insert candidates.
//
// In snapshot mode every lookup of a batch sees the table as it was before the
// batch; each miss leaves a candidate {cell, seq = hit * 32 + ordinal, code,
// hash2}.  Applying the candidates one after another in ascending seq with
// Algorithm 1 gives a unique table.  Cells are independent, so the candidates
// are grouped by cell (count -> scan -> scatter) and one thread per cell
// applies its own candidates in seq order.
#include "device_common.h"
#include "shade.h"

namespace pmc {

__global__ __launch_bounds__(256) void k_cand_count(SnapshotArgs a) {
  const uint32_t n = min(*a.cand_count, a.cand_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicAdd(&a.cell_count[a.cand[i].x], 1u);
}

__global__ __launch_bounds__(256) void k_cand_scatter(SnapshotArgs a) {
  const uint32_t n = min(*a.cand_count, a.cand_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint4 c = a.cand[i];
    uint32_t pos = atomicAdd(&a.cell_cursor[c.x], 1u);
    a.sorted[pos] = c;
  }
}

// Algorithm 1 on one cell for one candidate key (FIRST; OVERWRITE or PRIORITY
// with 16-byte entries); returns 0 inserted, 1 present, 2 full, 3 overwritten.
// PRIORITY: the victim is the entry of the largest path depth (aux), then the
// smallest stamp, then the lowest index; it is replaced when its depth exceeds
// the candidate's, or equals it and the entry predates this frame.
__device__ __forceinline__ int apply_one(uint64_t* w0, const SnapshotArgs& a, uint32_t hash2,
                                         uint32_t code, uint32_t stamp, uint32_t bounce) {
  const uint64_t neu = ((uint64_t)hash2 << 32) | code;
  const bool prio = a.policy == PMC_POLICY_PRIORITY;
  // the first entry holding the key or empty (entries fill front to back)
  uint32_t e = 0u;
  while (e < a.n_entries && (uint32_t)(w0[(uint64_t)e * a.entry_words] >> 32) != hash2 &&
         (uint32_t)(w0[(uint64_t)e * a.entry_words] >> 32) != 0u)
    ++e;
  if (e < a.n_entries) {
    uint64_t* p = w0 + (uint64_t)e * a.entry_words;
    if (*p != 0ull) return 1;
    *p = neu;
    if (a.entry_words == 2) {
      ((uint32_t*)p)[2] = stamp;
      if (prio) ((uint32_t*)p)[3] = bounce;
    }
    return 0;
  }
  if ((a.policy == PMC_POLICY_OVERWRITE || prio) && a.entry_words == 2) {
    uint32_t bs = 0xFFFFFFFFu, bb = 0u;
    int victim = -1;
    for (uint32_t i = 0; i < a.n_entries; ++i) {
      const uint32_t* e = (const uint32_t*)(w0 + (uint64_t)i * 2);
      const uint32_t st = e[2], b = prio ? e[3] : 0u;
      if (victim < 0 || b > bb || (b == bb && st < bs)) { bs = st; bb = b; victim = (int)i; }
    }
    const bool replace = prio ? (bb > bounce || (bb == bounce && bs < stamp)) : bs < stamp;
    if (victim >= 0 && replace) {
      uint64_t* p = w0 + (uint64_t)victim * 2;
      *p = neu;
      ((uint32_t*)p)[2] = stamp;
      if (prio) ((uint32_t*)p)[3] = bounce;
      return 3;
    }
  }
  return 2;
}

__device__ __forceinline__ uint32_t cand_bounce(const SnapshotArgs& a, uint32_t seq) {
  return (a.policy == PMC_POLICY_PRIORITY && a.bounce) ? a.bounce[seq >> 5] : 0u;
}

// One thread per cell applies its candidates as Algorithm 1 would in
// ascending seq, with stamps = frame + 1; it also clears the cell's count.
// Candidates of a key after its first (lowest seq) one never change the
// cell: the key is then present, or the cell was full and stays full (under
// FIRST nothing leaves a cell; under OVERWRITE a failed attempt means every
// entry was written in this frame, so later ones fail too).  So the distinct
// keys are applied in order of their lowest seq and the rest only counted;
// with more distinct keys than kDistinct the candidates are taken one by one.
// Under PRIORITY a later candidate of a key may carry a smaller path depth and
// succeed where the first failed, so there every candidate is taken in turn.
constexpr int kDistinct = 8;

__global__ __launch_bounds__(256) void k_cell_apply(SnapshotArgs a) {
  uint32_t c_ins = 0, c_present = 0, c_full = 0, c_over = 0;
  const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell < a.n_cells) {
    const uint32_t n = a.cell_count[cell];
    if (n) {
      a.cell_count[cell] = 0u;
      const uint32_t base = a.cell_start[cell];
      uint64_t* w0 = a.table + (uint64_t)cell * a.n_entries * a.entry_words;
      const uint32_t stamp = a.frame + 1u;
      // distinct keys: hash2, lowest seq, its code, candidate count
      uint32_t kh[kDistinct], ks[kDistinct], kc[kDistinct], kn[kDistinct];
      uint32_t d = 0;
      bool overflow = a.policy == PMC_POLICY_PRIORITY;
      for (uint32_t j = 0; j < n && !overflow; ++j) {
        const uint4 c = a.sorted[base + j];
        bool seen = false;
#pragma unroll
        for (int k = 0; k < kDistinct; ++k) {
          if ((uint32_t)k < d && kh[k] == c.w) {
            seen = true;
            kn[k] += 1u;
            if (c.y < ks[k]) { ks[k] = c.y; kc[k] = c.z; }
          }
        }
        if (!seen) {
          if (d == (uint32_t)kDistinct) {
            overflow = true;
          } else {
#pragma unroll
            for (int k = 0; k < kDistinct; ++k)
              if ((uint32_t)k == d) { kh[k] = c.w; ks[k] = c.y; kc[k] = c.z; kn[k] = 1u; }
            ++d;
          }
        }
      }
      if (!overflow) {
        for (uint32_t step = 0; step < d; ++step) {
          // the distinct key with the next lowest seq
          uint32_t best = 0xFFFFFFFFu;
          int bi = 0;
#pragma unroll
          for (int k = 0; k < kDistinct; ++k)
            if ((uint32_t)k < d && ks[k] < best) { best = ks[k]; bi = k; }
          uint32_t h2 = 0, code = 0, cntk = 0;
#pragma unroll
          for (int k = 0; k < kDistinct; ++k)
            if (k == bi) { h2 = kh[k]; code = kc[k]; cntk = kn[k]; ks[k] = 0xFFFFFFFFu; }
          const int o = apply_one(w0, a, h2, code, stamp, 0u);
          c_ins += o == 0;
          c_over += o == 3;
          c_present += o == 1;
          c_full += o == 2;
          // the key's later candidates
          if (o == 2) c_full += cntk - 1u;
          else c_present += cntk - 1u;
        }
      } else {
        int64_t last = -1;
        for (uint32_t step = 0; step < n; ++step) {
          uint32_t best = 0xFFFFFFFFu, bi = 0;
          for (uint32_t j = 0; j < n; ++j) {
            uint32_t sq = a.sorted[base + j].y;
            if ((int64_t)sq > last && sq <= best) { best = sq; bi = j; }
          }
          last = best;
          const uint4 c = a.sorted[base + bi];
          const int o = apply_one(w0, a, c.w, c.z, stamp, cand_bounce(a, c.y));
          c_ins += o == 0;
          c_over += o == 3;
          c_present += o == 1;
          c_full += o == 2;
        }
      }
    }
  }
  if (a.stat_slots) {
    unsigned long long* slot = a.stat_slots + (uint64_t)(blockIdx.x % kStatSlots) * kStatStride;
    uint32_t v[4] = {wave_sum(c_ins), wave_sum(c_present), wave_sum(c_full), wave_sum(c_over)};
    const int q[4] = {CNT_INSERTS, CNT_PRESENT, CNT_FULL, CNT_OVERWRITES};
    if (lane_id() == 0)
      for (int k = 0; k < 4; ++k)
        if (v[k]) atomicAdd(slot + q[k], (unsigned long long)v[k]);
  }
}

hipError_t launch_snapshot_apply(const SnapshotArgs& a, hipStream_t s) {
  const unsigned cgrid = 2048;
  hipLaunchKernelGGL(k_cand_count, dim3(cgrid), dim3(256), 0, s, a);
  hipError_t e = launch_exclusive_scan(a.cell_count, a.n_cells, a.cell_start, a.cell_cursor,
                                       a.block_sums, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cand_scatter, dim3(cgrid), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_cell_apply, dim3((a.n_cells + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pmc
