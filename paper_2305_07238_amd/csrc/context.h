// context.h - library-internal state of a pmc context and its caches, and the
// helpers shared by the C entry points (abi.cpp) and the frame graphs (frame.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pmc.h"
#include "compiler.h"
#include "shade.h"

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Surrogate networks and the insert log (pmc_surrogate_setup).
struct SurrHost {
  bool ready = false;
  uint32_t n_slots = 0;
  uint32_t log_cap = 0;                     // records, 64 regions of log_cap / 64
  float max_err = 1e-2f;
  std::vector<pmc_surrogate_slot> slots;
  std::vector<uint32_t> mat_slot;           // per material, 0xFFFFFFFF = none
  DevBuf w, master, state, mat_slot_dev, log, log_count;
  DevBuf slot_count, slot_begin, slot_cursor, scan_sums, grouped;
  DevBuf partial, sync;                     // data-parallel training exchange
};

struct pmc_ctx {
  int device = -1;
  bool host_only = true;
  int num_cus = 0;
  std::string err;
  pmc::Program prog;
  bool compiled = false;
  // program on the device
  DevBuf hdr, instr, cach, pool, lpt, lpt_rank;
  // textures
  DevBuf texels, texdesc;
  uint32_t n_tex = 0;
  // workspace
  // perm (+ perm2) and misc: the sorted order and device counters of a batch,
  // in kWorkSets sets (set 0 for single batches; frame graphs use all of them,
  // frame f set f % kWorkSets, so that sorts can run ahead of the shading)
  DevBuf perm, perm2, misc, cand, stat_slots;
  DevBuf surr_queue, surr_val;                   // parked hits of the surrogate passes
  DevBuf sort_counts, sort_offsets, sort_sums;   // tiled material sort
  SurrHost surr;
  void* static_scratch = nullptr;  // this device's fixed scratch array (pmc_shade_static)
  bool no_alloc = false;       // set while a frame graph is captured
  // Frame graphs bake this context's buffers and program into their launches:
  // while any exists, nothing they use may move or change shape, and
  // pmc_destroy only marks the context (freed with its last graph).
  uint32_t live_graphs = 0;
  bool orphaned = false;
  // phase timing: events recorded in pairs per phase
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_records;
  pmc_status fail(pmc_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
};

struct pmc_cache {
  pmc_ctx* ctx = nullptr;
  int device = 0;                // kept here so destruction never reads the context
  pmc_cache_params params{};
  void* mem = nullptr;
  bool owned = false;
  size_t bytes = 0;
  DevBuf cell_count, cell_start, cell_cursor, block_sums, sorted;
  uint32_t live_graphs = 0;      // frame graphs replaying into this table
  bool orphaned = false;         // pmc_cache_destroy called while graphs live
};

#define HIP_TRY(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return (ctx)->fail(PMC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
  } while (0)

namespace pmc {

void free_buf(DevBuf& b);
// Release a context or a table now (pmc_destroy / pmc_cache_destroy defer to
// these until no frame graph uses the object).
void destroy_context(pmc_ctx* ctx);
void destroy_cache(pmc_cache* c);
// PMC_ERR_STATE while frame graphs use the context's program or buffers.
pmc_status no_live_graphs(pmc_ctx* ctx, const char* what);
// grow-only device buffer; contents are not preserved.  Fails with
// PMC_ERR_STATE when it would allocate while ctx->no_alloc is set, or replace
// an existing buffer while frame graphs may use it.
pmc_status ensure(pmc_ctx* ctx, DevBuf& b, size_t bytes);
pmc_status need_device(pmc_ctx* ctx);
hipEvent_t next_event(pmc_ctx* ctx);

// Records a start event on construction and an end event on finish().
struct PhaseTimer {
  pmc_ctx* ctx;
  int phase;
  hipStream_t s;
  hipEvent_t start = nullptr;
  PhaseTimer(pmc_ctx* c, int ph, hipStream_t st);
  void finish();
};

// Argument checks of pmc_shade (host side, nothing enqueued).
pmc_status check_shade_args(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                            const pmc_bsdf_out* out, const pmc_shade_params* params);
// Device workspace for batches of up to n hits (all allocations and first-use
// clears, enqueued on s).  After this, shade_batch for such batches allocates
// nothing.  all_sets: every workspace set, not only set 0 (frame graphs).
constexpr int kWorkSets = 8;
pmc_status reserve_batch(pmc_ctx* ctx, pmc_cache* cache, uint32_t n, uint32_t mode,
                         uint32_t flags, uint32_t chunk_waves, bool all_sets, hipStream_t s);
// Per-batch device workspace of the modes without snapshot candidates or
// surrogate queues: the sorted order, the sort's tile matrix and scan sums,
// the batch counters and the statistics slots.  NULL members are taken from
// the context's buffers (workspace set `set`).
struct Workspace {
  uint32_t* perm = nullptr;
  uint32_t* sort_counts = nullptr;
  uint32_t* sort_offsets = nullptr;
  uint32_t* sort_sums = nullptr;
  uint32_t* misc = nullptr;                  // kMiscWords words
  unsigned long long* stat_slots = nullptr;  // kStatSlots * kStatStride, zero between batches
};
constexpr uint32_t kMiscQueue = 64, kMiscWords = 256;
// The two stages of a batch, for workspace set `set` (< kWorkSets): the material
// sort (or, unsorted, the reset of the set's counters), then shade -> surrogate
// passes -> snapshot apply -> stats.  The workspace must be reserved, or given
// in ws (its members replace the context's).
pmc_status sort_stage(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                      const pmc_shade_params* params, int set, hipStream_t s,
                      const Workspace* ws = nullptr);
pmc_status shade_stage(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                       const pmc_bsdf_out* out, const pmc_shade_params* params, pmc_stats* stats,
                       const pmc_debug_out* dbg, int set, hipStream_t s,
                       const Workspace* ws = nullptr);
// Address of this device's fixed scratch array (static_shade.cpp), looked up
// once per device with the device current; kept in ctx->static_scratch.
pmc_status static_scratch_init(pmc_ctx* ctx);
// The per-batch pipeline: reserve, then both stages on s with set 0.
pmc_status shade_batch(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                       const pmc_bsdf_out* out, const pmc_shade_params* params, pmc_stats* stats,
                       const pmc_debug_out* dbg, hipStream_t s);

}  // namespace pmc
