// static_shade.cpp - pmc_shade_static: the shading pipeline of pmc_shade with
// its per-batch workspace in a fixed device array instead of context
// buffers, for callers that cannot allocate device memory.
//
// The array `scratch` is a file-scope __device__ object: every device the
// library runs on holds its own copy, at its own address, until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host it is only a stand-in for the symbol); the device address comes
// from hipGetSymbolAddress, taken once per device with that device current
// (at pmc_create) and kept per device.
#include <mutex>

#include "context.h"

namespace {

__device__ __align__(256) unsigned char scratch[PMC_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the array for a batch of n hits over n_mats materials: statistics
// slots, batch counters, then (sorted batches) the order and the sort's tile
// matrix.  Returns the bytes used.
size_t carve(unsigned char* base, uint32_t n, uint32_t n_mats, bool sort, pmc::Workspace* ws) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  auto* slots = (unsigned long long*)take(sizeof(unsigned long long) * pmc::kStatSlots *
                                          pmc::kStatStride);
  auto* misc = (uint32_t*)take(pmc::kMiscWords * 4);
  if (ws) {
    ws->stat_slots = slots;
    ws->misc = misc;
  }
  if (sort) {
    const size_t cells = (size_t)n_mats + 1;                      // bucket counts
    auto* perm = (uint32_t*)take((size_t)n * 4);
    auto* counts = (uint32_t*)take(cells * 4);
    auto* offsets = (uint32_t*)take(cells * 4);
    auto* sums = (uint32_t*)take(((size_t)pmc::scan_blocks((uint32_t)cells) + 1) * 4);
    if (ws) {
      ws->perm = perm;
      ws->sort_counts = counts;
      ws->sort_offsets = offsets;
      ws->sort_sums = sums;
    }
  }
  return off;
}

}  // namespace

namespace pmc {

pmc_status static_scratch_init(pmc_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return ctx->fail(PMC_ERR_UNSUPPORTED, "device %d beyond the static scratch table",
                     ctx->device);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[ctx->device]) {
    void* p = nullptr;
    HIP_TRY(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return ctx->fail(PMC_ERR_HIP, "hipGetSymbolAddress returned no address");
    g_scratch[ctx->device] = p;
  }
  ctx->static_scratch = g_scratch[ctx->device];
  return PMC_OK;
}

}  // namespace pmc

using namespace pmc;

extern "C" {

pmc_status pmc_shade_static(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                            const pmc_bsdf_out* out, const pmc_shade_params* params,
                            pmc_stats* stats, const pmc_debug_out* dbg, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = check_shade_args(ctx, cache, hits, out, params)) return st;
  const uint32_t mode = cache ? params->mode : (uint32_t)PMC_MODE_UNCACHED;
  if (mode == PMC_MODE_SNAPSHOT)
    return ctx->fail(PMC_ERR_UNSUPPORTED,
                     "pmc_shade_static: SNAPSHOT mode needs workspace sized by the table");
  if (params->flags & (PMC_FLAG_LOG | PMC_FLAG_SURROGATE | PMC_FLAG_SURROGATE_INSERT))
    return ctx->fail(PMC_ERR_UNSUPPORTED,
                     "pmc_shade_static: the insert log and the networks need their own buffers");
  if (hits->n > PMC_STATIC_MAX_HITS)
    return ctx->fail(PMC_ERR_UNSUPPORTED, "pmc_shade_static: %llu hits, at most %u per call",
                     (unsigned long long)hits->n, (unsigned)PMC_STATIC_MAX_HITS);
  if (!ctx->static_scratch) return ctx->fail(PMC_ERR_STATE, "no static scratch on this device");
  const uint32_t n = (uint32_t)hits->n;
  if (n == 0) return PMC_OK;
  const uint32_t n_mats = (uint32_t)ctx->prog.headers.size();
  const bool sort = params->flags & PMC_FLAG_SORT;
  if (sort && n_mats + 1 > 16384)
    return ctx->fail(PMC_ERR_UNSUPPORTED, "material sort handles at most 16383 materials");
  const size_t need = carve(nullptr, n, n_mats, sort, nullptr);
  if (need > (size_t)PMC_STATIC_SCRATCH_BYTES)
    return ctx->fail(PMC_ERR_UNSUPPORTED,
                     "pmc_shade_static: %u hits over %u materials need %zu bytes of scratch, "
                     "the array holds %zu",
                     n, n_mats, need, (size_t)PMC_STATIC_SCRATCH_BYTES);
  Workspace ws;
  carve((unsigned char*)ctx->static_scratch, n, n_mats, sort, &ws);
  hipStream_t s = (hipStream_t)stream;
  // phase timing would create HIP events: not recorded by this entry point
  struct NoProfile {
    pmc_ctx* c;
    bool was;
    ~NoProfile() { c->profiling = was; }
  } guard{ctx, ctx->profiling};
  ctx->profiling = false;
  // the statistics slots must start at zero; an earlier call (of any context on
  // this device) leaves them zero only if it ran to its reduction
  if (stats)
    HIP_TRY(ctx, launch_fill_u64((uint64_t*)ws.stat_slots, 0ull,
                                 (uint64_t)kStatSlots * kStatStride, s));
  if (pmc_status st = sort_stage(ctx, cache, hits, params, 0, s, &ws)) return st;
  return shade_stage(ctx, cache, hits, out, params, stats, dbg, 0, s, &ws);
}

}  // extern "C"
