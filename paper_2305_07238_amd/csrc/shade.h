// shade.h - kernel arguments and host launchers of libpmc's HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pmc.h"
#include "device_common.h"
#include "program.h"
#include "surrogate.h"

namespace pmc {

// Counter slots, in the order of pmc_stats.
enum {
  CNT_HITS = 0, CNT_PROBES, CNT_CACHE_HITS, CNT_BYPASSES, CNT_INSERTS, CNT_CAS_FAIL,
  CNT_PRESENT, CNT_FULL, CNT_OVERWRITES, CNT_NONFINITE, CNT_CANDIDATES, CNT_NODES_EXEC,
  CNT_NODES_TOTAL, CNT_INVALID, CNT_TEX_EVALS, CNT_DEFERRED, CNT_INS_TRIED, CNT_TEX_DEFERRED,
  CNT_INS_TRIED_DEFERRED, CNT_PROBES_DEFERRED, CNT_SURR_USED, CNT_LOGGED, CNT_AUDITED,
  kNumCounters
};
enum { KIND_FULL = 0, KIND_PROBE = 1 };   // shade kernel variants
constexpr int kStatSlots = 1024;     // counters are spread over slots to limit atomic contention
constexpr int kStatStride = 32;      // u64 per slot (= sizeof(pmc_stats) / 8)

struct ShadeArgs {
  // compiled program
  const MatHeader* hdr;
  const Instr* instr;
  const CachDesc* cach;
  const float* pool;
  const TexDesc* tex;
  const uint32_t* texels;
  uint32_t n_mats;
  uint32_t n_regs;               // LDS registers per lane (max over materials)
  // hits
  const uint32_t* material;
  const float* uv;
  const float* duv;
  const float* normal;
  const uint32_t* bounce;        // path depth per hit (PRIORITY policy), NULL = all 0
  const float* position;         // [n][3] world positions, NULL when no graph reads them
  const float* width;            // [n] world footprint widths (with position)
  const uint32_t* perm;          // processing order (material-sorted), NULL = identity
  uint32_t n;
  uint32_t mode;
  // outputs
  float* out_base;
  float* out_rough;
  float* out_normal;
  // cache
  uint64_t* table;
  uint32_t n_cells;
  CellMap cells;                 // x -> x mod n_cells
  uint32_t n_entries;
  uint32_t entry_words;          // 64-bit words per entry: 1 (8 B) or 2 (16 B)
  uint32_t policy;
  uint32_t hash2_mask;           // bits of the verification hash kept (all 32 in the method)
  int32_t level_bias;
  int32_t level_max;
  uint32_t frame;
  uint32_t chunk_waves;          // consecutive 64-hit chunks per wave run
  // snapshot candidates {cell, seq, code, hash2}
  uint4* cand;
  uint32_t* cand_count;
  uint32_t cand_cap;
  // stats and diagnostics
  unsigned long long* stat_slots;
  uint8_t* dbg_state;
  float* dbg_value;
  uint32_t defer_max;            // a chunk with more missing lanes is evaluated in place
  // surrogate networks (PMC_FLAG_SURROGATE) and the insert log (PMC_FLAG_LOG)
  const SurrW* surr_w;
  SurrState* surr_state;
  pmc_log_record* log;           // NULL: no logging
  uint32_t* log_count;           // 64 region counters
  uint32_t log_region_cap;       // records per region
  uint2* surr_queue;             // parked hits {hit, surrogated ordinals | audited << 8},
                                 // kQueueRegions regions of surr_queue_cap entries
  uint32_t* surr_queue_count;    // [r] plain entries of region r (from its front),
                                 // [kQueueRegions + r] audited ones (from its back)
  uint32_t surr_queue_cap;       // entries per region
  float4* surr_val;              // the networks' outputs for the parked hits
  uint32_t surr_insert;          // 1: the networks' values are inserted as well
};

// The queue of parked hits is split into regions so that its counters are not
// one hot address: the run of chunks r (chunk_waves chunks handled by one wave)
// parks into region r % kQueueRegions, and a region holds every hit of its runs.
constexpr uint32_t kQueueRegions = 64;

inline uint32_t resolve_chunk_waves(uint32_t requested, bool probe_first) {
  return requested ? requested : (probe_first ? 4u : 1u);
}

inline uint32_t queue_region_cap(uint32_t n, uint32_t chunk_waves) {
  const uint64_t runs = ((uint64_t)(n + 63u) / 64u + chunk_waves - 1u) / chunk_waves;
  const uint64_t cap = (runs + kQueueRegions - 1u) / kQueueRegions * chunk_waves * 64u;
  return (uint32_t)(cap < 0xFFFFFFFFull / kQueueRegions ? cap : 0u);
}

// surr: the variant that consults the surrogate networks (cached modes only).
// block_waves: waves per workgroup of the flat grid (the persistent grid uses 4).
hipError_t launch_shade(const ShadeArgs& a, int kind, bool persistent, bool surr, uint32_t grid,
                        uint32_t block_waves, hipStream_t s);
// LDS of a workgroup of `waves` waves: per wave the register file and 64 staging ids.
size_t shade_lds_bytes(uint32_t n_regs, uint32_t waves = 4);
// After a surrogate first pass: the networks over the parked hits, then their finish
// pass (both size themselves from the queue count on the device).
hipError_t launch_surr_queue(const ShadeArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_surr_finish(const ShadeArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_debug_keys(const ShadeArgs& a, pmc_key_record* out, hipStream_t s);
hipError_t launch_insert_raw(const ShadeArgs& a, const uint64_t* k0, const uint64_t* k1,
                             const uint32_t* enc, uint64_t n, hipStream_t s);
hipError_t launch_lookup_raw(const ShadeArgs& a, const uint64_t* k0, const uint64_t* k1,
                             uint64_t n, uint32_t* enc_out, uint8_t* hit, hipStream_t s);

// util.hip
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t value, uint64_t n, hipStream_t s);
hipError_t launch_stats_reduce(unsigned long long* slots, pmc_stats* out, hipStream_t s);
// exclusive scan of n u32 -> out (and out_copy if not null); *total = sum (if not null).
// block_sums needs scan_blocks(n) + 1 entries.
uint32_t scan_blocks(uint32_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t n, uint32_t* out, uint32_t* out_copy,
                                 uint32_t* block_sums, uint32_t* total, hipStream_t s);

// Counting sort over tiles of the batch: buckets in rank order (rank[m] =
// position of material m by decreasing program length; invalid ids last).
// mat_counts / offsets need n_mats + 1 entries; scan_sums is unused.
// reset[0..n_reset) is zeroed.  At most 16383 materials and 1024 reset words.
// Kernel attributes (large dynamic LDS) set once per device, at context creation.
hipError_t prepare_sort_kernels();
hipError_t prepare_surrogate_kernels();
hipError_t launch_material_sort_tiled(const uint32_t* material, uint32_t n, uint32_t n_mats,
                                      const uint32_t* rank, uint32_t* mat_counts,
                                      uint32_t* offsets, uint32_t* scan_sums, uint32_t* perm,
                                      uint32_t* reset, uint32_t n_reset, hipStream_t s);

// snapshot.hip: apply the candidates of one batch in (hit, ordinal) order.
struct SnapshotArgs {
  uint64_t* table;
  uint32_t n_cells, n_entries, entry_words, policy, frame;
  const uint32_t* bounce;        // path depth of hit seq >> 5 (PRIORITY policy), NULL = all 0
  const uint4* cand;
  uint4* sorted;
  const uint32_t* cand_count;
  uint32_t cand_cap;
  uint32_t* cell_count;          // n_cells
  uint32_t* cell_start;          // n_cells
  uint32_t* cell_cursor;         // n_cells
  uint32_t* block_sums;          // scan scratch
  unsigned long long* stat_slots;
};
hipError_t launch_snapshot_apply(const SnapshotArgs& a, hipStream_t s);

}  // namespace pmc
