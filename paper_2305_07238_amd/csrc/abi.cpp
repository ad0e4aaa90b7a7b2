// abi.cpp - the C entry points of libpmc: context, textures, graph
// compilation, cache tables, and the per-batch shading pipeline
// (material sort -> shade -> snapshot apply -> statistics).
#include <cstring>

#include "context.h"

using namespace pmc;

namespace pmc {

hipEvent_t next_event(pmc_ctx* ctx) {
  if (ctx->ev_used == ctx->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->ev_pool.push_back(e);
  }
  return ctx->ev_pool[ctx->ev_used++];
}

PhaseTimer::PhaseTimer(pmc_ctx* c, int ph, hipStream_t st) : ctx(c), phase(ph), s(st) {
  if (ctx->profiling && (start = next_event(ctx))) (void)hipEventRecord(start, s);
}

void PhaseTimer::finish() {
  if (!start) return;
  hipEvent_t end = next_event(ctx);
  if (!end) return;
  (void)hipEventRecord(end, s);
  ctx->ev_records.push_back({phase, {start, end}});
  start = nullptr;
}

void free_buf(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

pmc_status ensure(pmc_ctx* ctx, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return PMC_OK;
  if (ctx->no_alloc)
    return ctx->fail(PMC_ERR_STATE, "workspace of %zu bytes not reserved before capture", bytes);
  if (b.p && ctx->live_graphs)
    return ctx->fail(PMC_ERR_STATE,
                     "a buffer of %zu bytes would replace one that %u frame graph(s) may use; "
                     "destroy them first or create them for the larger batch",
                     bytes, ctx->live_graphs);
  free_buf(b);
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return ctx->fail(e == hipErrorOutOfMemory ? PMC_ERR_OOM : PMC_ERR_HIP,
                     "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  return PMC_OK;
}

pmc_status need_device(pmc_ctx* ctx) {
  if (ctx->host_only) return ctx->fail(PMC_ERR_STATE, "host-only context has no device");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  return PMC_OK;
}

void destroy_context(pmc_ctx* ctx) {
  if (!ctx->host_only) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&ctx->hdr, &ctx->instr, &ctx->cach, &ctx->pool, &ctx->lpt, &ctx->lpt_rank,
                      &ctx->sort_counts, &ctx->sort_offsets, &ctx->sort_sums, &ctx->texels,
                      &ctx->texdesc, &ctx->perm, &ctx->perm2, &ctx->misc,
                      &ctx->cand, &ctx->stat_slots, &ctx->surr_queue, &ctx->surr_val,
                      &ctx->surr.w, &ctx->surr.master,
                      &ctx->surr.state, &ctx->surr.mat_slot_dev, &ctx->surr.log,
                      &ctx->surr.log_count, &ctx->surr.slot_count, &ctx->surr.slot_begin,
                      &ctx->surr.slot_cursor, &ctx->surr.scan_sums, &ctx->surr.grouped,
                      &ctx->surr.partial, &ctx->surr.sync})
      free_buf(*b);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  }
  delete ctx;
}

void destroy_cache(pmc_cache* c) {
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->owned && c->mem) (void)hipFree(c->mem);
  for (DevBuf* b : {&c->cell_count, &c->cell_start, &c->cell_cursor, &c->block_sums, &c->sorted})
    free_buf(*b);
  delete c;
}

pmc_status no_live_graphs(pmc_ctx* ctx, const char* what) {
  if (ctx->live_graphs)
    return ctx->fail(PMC_ERR_STATE, "%s: %u frame graph(s) use the current program and buffers",
                     what, ctx->live_graphs);
  return PMC_OK;
}

}  // namespace pmc

namespace {

// Small per-context device words, kWorkSets sets of kMiscWords: [1] the snapshot
// candidate count, [kMiscQueue, kMiscQueue + 2 kQueueRegions) the surrogate
// queue's counters.
static_assert(kMiscQueue + 2 * kQueueRegions <= kMiscWords, "misc words");

template <typename T>
pmc_status upload(pmc_ctx* ctx, DevBuf& b, const std::vector<T>& v) {
  size_t bytes = v.size() * sizeof(T);
  pmc_status st = ensure(ctx, b, bytes ? bytes : 256);
  if (st) return st;
  if (bytes) HIP_TRY(ctx, hipMemcpy(b.p, v.data(), bytes, hipMemcpyHostToDevice));
  return PMC_OK;
}

}  // namespace

extern "C" {

uint32_t pmc_abi_version(void) { return PMC_ABI_VERSION; }

size_t pmc_abi_sizeof(uint32_t which) {
  switch (which) {
    case 0: return sizeof(pmc_node_desc);
    case 1: return sizeof(pmc_input);
    case 2: return sizeof(pmc_texture_desc);
    case 3: return sizeof(pmc_compile_opts);
    case 4: return sizeof(pmc_material_info);
    case 5: return sizeof(pmc_cache_params);
    case 6: return sizeof(pmc_shade_params);
    case 7: return sizeof(pmc_stats);
    case 8: return sizeof(pmc_hits);
    case 9: return sizeof(pmc_bsdf_out);
    case 10: return sizeof(pmc_debug_out);
    case 11: return sizeof(pmc_key_record);
    case 12: return sizeof(pmc_frame_plan);
    case 13: return sizeof(pmc_tune_result);
    case 14: return sizeof(pmc_profile);
    case 15: return sizeof(pmc_surrogate_opts);
    case 16: return sizeof(pmc_surrogate_slot);
    case 17: return sizeof(pmc_log_record);
    case 18: return sizeof(pmc_train_params);
    case 19: return sizeof(pmc_surrogate_stat);
    case 20: return sizeof(pmc_cone_hits);
    default: return 0;
  }
}

pmc_status pmc_create(int device, pmc_ctx** out) {
  if (!out) return PMC_ERR_INVALID;
  *out = nullptr;
  pmc_ctx* ctx = new (std::nothrow) pmc_ctx();
  if (!ctx) return PMC_ERR_OOM;
  if (device >= 0) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
      delete ctx;
      return PMC_ERR_INVALID;
    }
    ctx->device = device;
    ctx->host_only = false;
    if (hipSetDevice(device) != hipSuccess) {
      delete ctx;
      return PMC_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
      delete ctx;
      return PMC_ERR_HIP;
    }
    ctx->num_cus = prop.multiProcessorCount;
    if (ensure(ctx, ctx->stat_slots, sizeof(unsigned long long) * kStatSlots * kStatStride) ||
        ensure(ctx, ctx->misc, kWorkSets * kMiscWords * 4) ||
        hipMemset(ctx->stat_slots.p, 0, ctx->stat_slots.bytes) != hipSuccess ||
        hipMemset(ctx->misc.p, 0, ctx->misc.bytes) != hipSuccess ||
        prepare_sort_kernels() != hipSuccess || prepare_surrogate_kernels() != hipSuccess ||
        static_scratch_init(ctx) != PMC_OK) {
      pmc_destroy(ctx);
      return PMC_ERR_HIP;
    }
  } else if (device != -1) {
    delete ctx;
    return PMC_ERR_INVALID;
  }
  *out = ctx;
  return PMC_OK;
}

void pmc_destroy(pmc_ctx* ctx) {
  if (!ctx) return;
  if (ctx->live_graphs) {
    ctx->orphaned = true;
    return;
  }
  destroy_context(ctx);
}

pmc_status pmc_profile_enable(pmc_ctx* ctx, int on) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_device(ctx)) return st;
  HIP_TRY(ctx, hipDeviceSynchronize());
  ctx->profiling = on != 0;
  ctx->ev_records.clear();
  ctx->ev_used = 0;
  return PMC_OK;
}

pmc_status pmc_profile_read(pmc_ctx* ctx, pmc_profile* out, int reset) {
  if (!ctx || !out) return PMC_ERR_INVALID;
  if (pmc_status st = need_device(ctx)) return st;
  std::memset(out, 0, sizeof *out);
  for (auto& r : ctx->ev_records) {
    HIP_TRY(ctx, hipEventSynchronize(r.second.second));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, r.second.first, r.second.second));
    out->ms[r.first] += ms;
    out->launches[r.first] += 1;
  }
  if (reset) {
    ctx->ev_records.clear();
    ctx->ev_used = 0;
  }
  return PMC_OK;
}

const char* pmc_last_error(const pmc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

pmc_status pmc_set_textures(pmc_ctx* ctx, const pmc_texture_desc* tex, uint32_t n_tex) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = no_live_graphs(ctx, "set_textures")) return st;
  if (n_tex && !tex) return ctx->fail(PMC_ERR_INVALID, "set_textures: null texture array");
  if (pmc_status st = need_device(ctx)) return st;
  std::vector<TexDesc> desc(n_tex);
  uint64_t total = 0;
  for (uint32_t t = 0; t < n_tex; ++t) {
    if (!tex[t].texels || tex[t].width == 0 || tex[t].height == 0 || tex[t].width > 65536 ||
        tex[t].height > 65536)
      return ctx->fail(PMC_ERR_INVALID, "texture %u: null texels or bad size", t);
    desc[t].offset = total;
    desc[t].w = tex[t].width;
    desc[t].h = tex[t].height;
    total += (uint64_t)tex[t].width * tex[t].height;
  }
  if (pmc_status st = ensure(ctx, ctx->texels, total * 4 + 256)) return st;
  for (uint32_t t = 0; t < n_tex; ++t)
    HIP_TRY(ctx, hipMemcpy((uint32_t*)ctx->texels.p + desc[t].offset, tex[t].texels,
                           (size_t)tex[t].width * tex[t].height * 4, hipMemcpyHostToDevice));
  if (pmc_status st = upload(ctx, ctx->texdesc, desc)) return st;
  ctx->n_tex = n_tex;
  return PMC_OK;
}

pmc_status pmc_compile_materials(pmc_ctx* ctx, const pmc_node_desc* nodes,
                                 const uint32_t* node_offsets, uint32_t n_mats,
                                 const pmc_compile_opts* opts) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = no_live_graphs(ctx, "compile_materials")) return st;
  Program prog;
  std::string err;
  pmc_status st = compile_program(nodes, node_offsets, n_mats, opts, prog, err);
  if (st != PMC_OK) return ctx->fail(st, "%s", err.c_str());
  if (prog.max_regs > 64)
    return ctx->fail(PMC_ERR_UNSUPPORTED, "a material needs %u registers (limit 64)",
                     prog.max_regs);
  if (!ctx->host_only) {
    if (pmc_status s2 = need_device(ctx)) return s2;
    HIP_TRY(ctx, hipDeviceSynchronize());   // no batch may still read the old program
    if ((st = upload(ctx, ctx->hdr, prog.headers)) || (st = upload(ctx, ctx->instr, prog.instrs)) ||
        (st = upload(ctx, ctx->cach, prog.cach)) || (st = upload(ctx, ctx->pool, prog.pool)) ||
        (st = upload(ctx, ctx->lpt, prog.lpt_order)) ||
        (st = upload(ctx, ctx->lpt_rank, prog.lpt_rank)))
      return st;
  }
  ctx->prog = std::move(prog);
  ctx->compiled = true;
  ctx->surr.ready = false;     // slots refer to the old graph set: set up again
  ctx->surr.n_slots = 0;
  ctx->surr.slots.clear();
  return PMC_OK;
}

pmc_status pmc_get_material_info(const pmc_ctx* ctx, uint32_t mat, pmc_material_info* out) {
  if (!ctx || !out) return PMC_ERR_INVALID;
  if (!ctx->compiled) return PMC_ERR_STATE;
  if (mat >= ctx->prog.info.size()) return PMC_ERR_INVALID;
  *out = ctx->prog.info[mat];
  return PMC_OK;
}

// ------------------------------------------------------------------ cache ---

pmc_status pmc_cache_create(pmc_ctx* ctx, const pmc_cache_params* p, void* device_mem,
                            pmc_cache** out) {
  if (!ctx || !p || !out) return PMC_ERR_INVALID;
  *out = nullptr;
  if (pmc_status st = need_device(ctx)) return st;
  if (p->n_cells == 0 || p->n_cells >= (1ull << 32))
    return ctx->fail(PMC_ERR_INVALID, "n_cells must be in [1, 2^32)");
  if (p->n_entries == 0 || p->n_entries > 64)
    return ctx->fail(PMC_ERR_INVALID, "n_entries must be in [1, 64]");
  if (p->entry_bytes != 8 && p->entry_bytes != 16)
    return ctx->fail(PMC_ERR_INVALID, "entry_bytes must be 8 or 16");
  if (p->policy > PMC_POLICY_PRIORITY) return ctx->fail(PMC_ERR_INVALID, "unknown policy");
  if (p->policy != PMC_POLICY_FIRST && p->entry_bytes != 16)
    return ctx->fail(PMC_ERR_INVALID, "OVERWRITE and PRIORITY need 16-byte entries (stamps)");
  if (p->level_max > 30) return ctx->fail(PMC_ERR_INVALID, "level_max must be <= 30");
  pmc_cache* c = new (std::nothrow) pmc_cache();
  if (!c) return PMC_ERR_OOM;
  c->ctx = ctx;
  c->device = ctx->device;
  c->params = *p;
  if (c->params.level_max == 0) c->params.level_max = 20;
  if (c->params.hash2_mask == 0) c->params.hash2_mask = 0xFFFFFFFFu;
  c->bytes = (size_t)p->n_cells * p->n_entries * p->entry_bytes;
  if (device_mem) {
    if (((uintptr_t)device_mem & 255u) != 0) {
      delete c;
      return ctx->fail(PMC_ERR_INVALID, "device_mem must be 256-byte aligned");
    }
    c->mem = device_mem;
  } else {
    hipError_t e = hipMalloc(&c->mem, c->bytes);
    if (e != hipSuccess) {
      delete c;
      return ctx->fail(PMC_ERR_OOM, "hipMalloc(%zu) for the table failed", c->bytes);
    }
    c->owned = true;
  }
  hipError_t e = hipMemset(c->mem, 0, c->bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    pmc_cache_destroy(c);
    return ctx->fail(PMC_ERR_HIP, "clearing the table failed: %s", hipGetErrorString(e));
  }
  *out = c;
  return PMC_OK;
}

void pmc_cache_destroy(pmc_cache* c) {
  if (!c) return;
  if (c->live_graphs) {
    c->orphaned = true;
    return;
  }
  destroy_cache(c);
}

pmc_status pmc_cache_clear(pmc_cache* c, void* stream) {
  if (!c) return PMC_ERR_INVALID;
  pmc_ctx* ctx = c->ctx;
  if (pmc_status st = need_device(ctx)) return st;
  HIP_TRY(ctx, launch_fill_u64((uint64_t*)c->mem, 0ull, c->bytes / 8, (hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_cache_device_ptr(pmc_cache* c, void** ptr, size_t* bytes) {
  if (!c || !ptr || !bytes) return PMC_ERR_INVALID;
  *ptr = c->mem;
  *bytes = c->bytes;
  return PMC_OK;
}

pmc_status pmc_cache_export(pmc_cache* c, void* host_dst, size_t bytes, void* stream) {
  if (!c || !host_dst) return PMC_ERR_INVALID;
  pmc_ctx* ctx = c->ctx;
  if (bytes != c->bytes) return ctx->fail(PMC_ERR_INVALID, "export: size %zu != table %zu", bytes, c->bytes);
  if (pmc_status st = need_device(ctx)) return st;
  HIP_TRY(ctx, hipMemcpyAsync(host_dst, c->mem, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(ctx, hipStreamSynchronize((hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_cache_import(pmc_cache* c, const void* host_src, size_t bytes, void* stream) {
  if (!c || !host_src) return PMC_ERR_INVALID;
  pmc_ctx* ctx = c->ctx;
  if (bytes != c->bytes) return ctx->fail(PMC_ERR_INVALID, "import: size %zu != table %zu", bytes, c->bytes);
  if (pmc_status st = need_device(ctx)) return st;
  HIP_TRY(ctx, hipMemcpyAsync(c->mem, host_src, bytes, hipMemcpyHostToDevice, (hipStream_t)stream));
  HIP_TRY(ctx, hipStreamSynchronize((hipStream_t)stream));
  return PMC_OK;
}

// ---------------------------------------------------------------- shading ---

static void fill_program_args(pmc_ctx* ctx, ShadeArgs& a) {
  std::memset(&a, 0, sizeof a);
  a.hdr = (const MatHeader*)ctx->hdr.p;
  a.instr = (const Instr*)ctx->instr.p;
  a.cach = (const CachDesc*)ctx->cach.p;
  a.pool = (const float*)ctx->pool.p;
  a.tex = (const TexDesc*)ctx->texdesc.p;
  a.texels = (const uint32_t*)ctx->texels.p;
  a.n_mats = (uint32_t)ctx->prog.headers.size();
  a.n_regs = ctx->prog.max_regs ? ctx->prog.max_regs : 1;
}

static void fill_cache_args(pmc_cache* c, ShadeArgs& a) {
  a.table = (uint64_t*)c->mem;
  a.n_cells = (uint32_t)c->params.n_cells;
  a.cells = make_cell_map(a.n_cells);
  a.n_entries = c->params.n_entries;
  a.entry_words = c->params.entry_bytes / 8;
  a.policy = c->params.policy;
  a.hash2_mask = c->params.hash2_mask;
  a.level_bias = c->params.level_bias;
  a.level_max = (int32_t)c->params.level_max;
}

static pmc_status check_hits(pmc_ctx* ctx, const pmc_hits* h) {
  if (!h) return ctx->fail(PMC_ERR_INVALID, "null hits");
  if (h->n >= (1ull << 27)) return ctx->fail(PMC_ERR_INVALID, "at most 2^27 - 1 hits per call");
  if (h->n && (!h->material || !h->uv || !h->duv || !h->normal))
    return ctx->fail(PMC_ERR_INVALID, "null hit array");
  if (((uintptr_t)h->uv & 7u) || ((uintptr_t)h->duv & 15u))
    return ctx->fail(PMC_ERR_INVALID, "uv must be 8-byte and duv 16-byte aligned");
  if (!h->position != !h->width)
    return ctx->fail(PMC_ERR_INVALID, "position and width go together");
  if (h->n && ctx->compiled && ctx->prog.uses_position && !h->position)
    return ctx->fail(PMC_ERR_INVALID, "the compiled graphs read the world position");
  return PMC_OK;
}

static pmc_status ready(pmc_ctx* ctx) {
  if (pmc_status st = need_device(ctx)) return st;
  if (!ctx->compiled) return ctx->fail(PMC_ERR_STATE, "no compiled graph set");
  if (ctx->prog.max_texture >= (int32_t)ctx->n_tex)
    return ctx->fail(PMC_ERR_STATE, "graphs use texture %d but %u are set",
                     ctx->prog.max_texture, ctx->n_tex);
  return PMC_OK;
}

}  // extern "C"

namespace pmc {

pmc_status check_shade_args(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                            const pmc_bsdf_out* out, const pmc_shade_params* params) {
  if (pmc_status st = ready(ctx)) return st;
  if (pmc_status st = check_hits(ctx, hits)) return st;
  if (!params) return ctx->fail(PMC_ERR_INVALID, "null params");
  if (params->mode > PMC_MODE_SNAPSHOT) return ctx->fail(PMC_ERR_INVALID, "unknown mode");
  if (params->flags & ~(uint32_t)(PMC_FLAG_SORT | PMC_FLAG_PERSISTENT | PMC_FLAG_DEFER |
                                  PMC_FLAG_LOG | PMC_FLAG_SURROGATE | PMC_FLAG_SURROGATE_INSERT))
    return ctx->fail(PMC_ERR_INVALID, "unknown flags");
  if ((params->flags & (PMC_FLAG_LOG | PMC_FLAG_SURROGATE)) && !ctx->surr.ready)
    return ctx->fail(PMC_ERR_STATE, "PMC_FLAG_LOG / PMC_FLAG_SURROGATE need pmc_surrogate_setup");
  if (params->waves_per_block != 0 && params->waves_per_block != 1 &&
      params->waves_per_block != 2 && params->waves_per_block != 4)
    return ctx->fail(PMC_ERR_INVALID, "waves_per_block must be 0, 1, 2 or 4");
  if (hits->n && (!out || !out->base_color || !out->roughness || !out->normal))
    return ctx->fail(PMC_ERR_INVALID, "null output array");
  if (cache && cache->ctx != ctx) return ctx->fail(PMC_ERR_INVALID, "cache of another context");
  return PMC_OK;
}

pmc_status reserve_batch(pmc_ctx* ctx, pmc_cache* cache, uint32_t n, uint32_t mode,
                         uint32_t flags, uint32_t chunk_waves, bool all_sets, hipStream_t s) {
  const uint32_t n_mats = (uint32_t)ctx->prog.headers.size();
  pmc_status st;
  if (flags & PMC_FLAG_SORT) {
    if (n_mats + 1 > 16384)
      return ctx->fail(PMC_ERR_UNSUPPORTED, "material sort handles at most 16383 materials");
    const size_t cells = (size_t)n_mats + 1;                      // bucket counts
    if ((st = ensure(ctx, ctx->perm, (size_t)n * 4)) ||
        (all_sets && (st = ensure(ctx, ctx->perm2, (size_t)n * 4 * (kWorkSets - 1)))) ||
        (st = ensure(ctx, ctx->sort_counts, cells * 4)) ||
        (st = ensure(ctx, ctx->sort_offsets, cells * 4)) ||
        (st = ensure(ctx, ctx->sort_sums, ((size_t)scan_blocks((uint32_t)cells) + 1) * 4)))
      return st;
  }
  if ((flags & PMC_FLAG_SURROGATE) && mode != PMC_MODE_UNCACHED && cache) {
    const uint32_t cap = queue_region_cap(n, chunk_waves);
    if (cap == 0) return ctx->fail(PMC_ERR_UNSUPPORTED, "batch too large for the surrogate queue");
    const size_t entries = (size_t)cap * kQueueRegions;
    if ((st = ensure(ctx, ctx->surr_queue, entries * 8)) ||
        (st = ensure(ctx, ctx->surr_val, entries * 16)))
      return st;
  }
  if (mode == PMC_MODE_SNAPSHOT && cache) {
    const size_t cap = (size_t)n * (ctx->prog.max_cach ? ctx->prog.max_cach : 1);
    if ((st = ensure(ctx, ctx->cand, cap * 16)) || (st = ensure(ctx, cache->sorted, cap * 16)))
      return st;
    const uint32_t ncell = (uint32_t)cache->params.n_cells;
    if (!cache->cell_count.p) {
      if ((st = ensure(ctx, cache->cell_count, (size_t)ncell * 4))) return st;
      HIP_TRY(ctx, launch_fill_u32((uint32_t*)cache->cell_count.p, 0u, ncell, s));
    }
    if ((st = ensure(ctx, cache->cell_start, (size_t)ncell * 4)) ||
        (st = ensure(ctx, cache->cell_cursor, (size_t)ncell * 4)) ||
        (st = ensure(ctx, cache->block_sums, (size_t)scan_blocks(ncell) * 4 + 4)))
      return st;
  }
  return PMC_OK;
}

namespace {

uint32_t batch_mode(const pmc_shade_params* params, const pmc_cache* cache) {
  return cache ? params->mode : (uint32_t)PMC_MODE_UNCACHED;
}

bool batch_surr(const pmc_shade_params* params, uint32_t mode) {
  return (params->flags & PMC_FLAG_SURROGATE) && mode != PMC_MODE_UNCACHED;
}

uint32_t* misc_set(pmc_ctx* ctx, int set) { return (uint32_t*)ctx->misc.p + set * kMiscWords; }

// set k > 0 of a batch of n hits: entries [(k - 1) n, k n) of perm2
uint32_t* perm_set(pmc_ctx* ctx, int set, uint32_t n) {
  return set ? (uint32_t*)ctx->perm2.p + (size_t)(set - 1) * n : (uint32_t*)ctx->perm.p;
}

}  // namespace

pmc_status sort_stage(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                      const pmc_shade_params* params, int set, hipStream_t s,
                      const Workspace* ws) {
  const uint32_t n = (uint32_t)hits->n;
  if (n == 0) return PMC_OK;
  const uint32_t mode = batch_mode(params, cache);
  uint32_t* misc = ws && ws->misc ? ws->misc : misc_set(ctx, set);
  // misc[1]: snapshot candidate count; misc[kMiscQueue ..]: the queue's region
  // counters (reset by the sort's scan, or filled here)
  const uint32_t n_reset = batch_surr(params, mode) ? kMiscQueue + 2u * kQueueRegions : 4u;
  if (params->flags & PMC_FLAG_SORT) {
    PhaseTimer t0(ctx, 0, s);
    const bool own = ws && ws->perm;
    HIP_TRY(ctx, launch_material_sort_tiled(
                     hits->material, n, (uint32_t)ctx->prog.headers.size(),
                     (const uint32_t*)ctx->lpt_rank.p,
                     own ? ws->sort_counts : (uint32_t*)ctx->sort_counts.p,
                     own ? ws->sort_offsets : (uint32_t*)ctx->sort_offsets.p,
                     own ? ws->sort_sums : (uint32_t*)ctx->sort_sums.p,
                     own ? ws->perm : perm_set(ctx, set, n), misc, n_reset, s));
    t0.finish();
  } else {
    HIP_TRY(ctx, launch_fill_u32(misc, 0u, n_reset, s));
  }
  return PMC_OK;
}

pmc_status shade_batch(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                       const pmc_bsdf_out* out, const pmc_shade_params* params, pmc_stats* stats,
                       const pmc_debug_out* dbg, hipStream_t s) {
  const uint32_t n = (uint32_t)hits->n;
  if (n == 0) return PMC_OK;
  const uint32_t mode = batch_mode(params, cache);
  const bool probe_first = mode != PMC_MODE_UNCACHED && (params->flags & PMC_FLAG_DEFER);
  const uint32_t chunk_waves = resolve_chunk_waves(params->chunk_waves, probe_first);
  if (pmc_status st = reserve_batch(ctx, cache, n, mode, params->flags, chunk_waves, false, s))
    return st;
  if (pmc_status st = sort_stage(ctx, cache, hits, params, 0, s)) return st;
  return shade_stage(ctx, cache, hits, out, params, stats, dbg, 0, s);
}

pmc_status shade_stage(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                       const pmc_bsdf_out* out, const pmc_shade_params* params, pmc_stats* stats,
                       const pmc_debug_out* dbg, int set, hipStream_t s, const Workspace* ws) {
  const uint32_t n = (uint32_t)hits->n;
  if (n == 0) return PMC_OK;
  const uint32_t mode = batch_mode(params, cache);
  const bool sort = params->flags & PMC_FLAG_SORT;
  const bool persistent = params->flags & PMC_FLAG_PERSISTENT;
  const bool probe_first = mode != PMC_MODE_UNCACHED && (params->flags & PMC_FLAG_DEFER);
  const uint32_t chunk_waves = resolve_chunk_waves(params->chunk_waves, probe_first);

  ShadeArgs a;
  fill_program_args(ctx, a);
  a.material = hits->material;
  a.uv = hits->uv;
  a.duv = hits->duv;
  a.normal = hits->normal;
  a.bounce = hits->bounce;
  a.position = hits->position;
  a.width = hits->width;
  a.n = n;
  a.mode = mode;
  a.out_base = out->base_color;
  a.out_rough = out->roughness;
  a.out_normal = out->normal;
  a.frame = params->frame;
  unsigned long long* slots = ws && ws->stat_slots ? ws->stat_slots
                                                   : (unsigned long long*)ctx->stat_slots.p;
  a.stat_slots = stats ? slots : nullptr;
  a.dbg_state = dbg ? dbg->state : nullptr;
  a.dbg_value = dbg ? dbg->value : nullptr;
  uint32_t* misc = ws && ws->misc ? ws->misc : misc_set(ctx, set);
  if (mode != PMC_MODE_UNCACHED) fill_cache_args(cache, a);
  const bool surr = batch_surr(params, mode);
  const bool logged = (params->flags & PMC_FLAG_LOG) && mode != PMC_MODE_UNCACHED;
  if (surr || logged) {
    a.surr_w = (const SurrW*)ctx->surr.w.p;
    a.surr_state = (SurrState*)ctx->surr.state.p;
  }
  if (surr) {
    a.surr_insert = (params->flags & PMC_FLAG_SURROGATE_INSERT) ? 1u : 0u;
    a.surr_queue = (uint2*)ctx->surr_queue.p;
    a.surr_val = (float4*)ctx->surr_val.p;
    a.surr_queue_cap = queue_region_cap(n, chunk_waves);
    a.surr_queue_count = misc + kMiscQueue;
  }
  if (logged) {
    a.log = (pmc_log_record*)ctx->surr.log.p;
    a.log_count = (uint32_t*)ctx->surr.log_count.p;
    a.log_region_cap = ctx->surr.log_cap / 64u;
  }

  if (sort) a.perm = ws && ws->perm ? ws->perm : perm_set(ctx, set, n);
  if (mode == PMC_MODE_SNAPSHOT) {
    a.cand = (uint4*)ctx->cand.p;
    a.cand_count = misc + 1;
    a.cand_cap = (uint32_t)((size_t)n * (ctx->prog.max_cach ? ctx->prog.max_cach : 1));
  }
  const uint32_t n_chunks = (n + 63) / 64;
  a.chunk_waves = chunk_waves;
  a.defer_max = params->defer_max ? params->defer_max : 48u;
  const uint32_t runs = (n_chunks + a.chunk_waves - 1) / a.chunk_waves;
  const uint32_t block_waves = params->waves_per_block ? params->waves_per_block : 4u;
  uint32_t grid;
  if (persistent) {
    uint32_t bpc = params->blocks_per_cu;
    if (bpc == 0) {
      size_t lds_per_block = shade_lds_bytes(a.n_regs);
      bpc = (uint32_t)((160 * 1024) / (lds_per_block ? lds_per_block : 1));
      bpc = bpc < 1 ? 1 : (bpc > 8 ? 8 : bpc);
    }
    grid = (uint32_t)ctx->num_cus * bpc;
    const uint32_t max_useful = (runs + 3) / 4;
    if (grid > max_useful) grid = max_useful ? max_useful : 1;
  } else {
    grid = (runs + block_waves - 1) / block_waves;
  }
  PhaseTimer t1(ctx, 1, s);
  HIP_TRY(ctx,
          launch_shade(a, probe_first ? KIND_PROBE : KIND_FULL, persistent, surr, grid,
                       block_waves, s));
  if (surr) {
    const uint32_t qgrid = (uint32_t)ctx->num_cus * 4u;
    HIP_TRY(ctx, launch_surr_queue(a, qgrid, s));
    HIP_TRY(ctx, launch_surr_finish(a, qgrid, s));
  }
  t1.finish();
  if (mode == PMC_MODE_SNAPSHOT) {
    SnapshotArgs sa;
    sa.table = a.table;
    sa.n_cells = a.n_cells;
    sa.n_entries = a.n_entries;
    sa.entry_words = a.entry_words;
    sa.policy = a.policy;
    sa.frame = a.frame;
    sa.bounce = a.bounce;
    sa.cand = a.cand;
    sa.sorted = (uint4*)cache->sorted.p;
    sa.cand_count = a.cand_count;
    sa.cand_cap = a.cand_cap;
    sa.cell_count = (uint32_t*)cache->cell_count.p;
    sa.cell_start = (uint32_t*)cache->cell_start.p;
    sa.cell_cursor = (uint32_t*)cache->cell_cursor.p;
    sa.block_sums = (uint32_t*)cache->block_sums.p;
    sa.stat_slots = a.stat_slots;
    PhaseTimer t2(ctx, 2, s);
    HIP_TRY(ctx, launch_snapshot_apply(sa, s));
    t2.finish();
  }
  if (surr) HIP_TRY(ctx, launch_surr_live_update((SurrState*)ctx->surr.state.p,
                                                 ctx->surr.n_slots, s));
  if (stats) {
    PhaseTimer t3(ctx, 3, s);
    HIP_TRY(ctx, launch_stats_reduce(slots, stats, s));
    t3.finish();
  }
  return PMC_OK;
}

}  // namespace pmc

extern "C" {

pmc_status pmc_shade(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                     const pmc_bsdf_out* out, const pmc_shade_params* params, pmc_stats* stats,
                     const pmc_debug_out* dbg, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = check_shade_args(ctx, cache, hits, out, params)) return st;
  return shade_batch(ctx, cache, hits, out, params, stats, dbg, (hipStream_t)stream);
}

pmc_status pmc_debug_keys(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                          pmc_key_record* out, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = ready(ctx)) return st;
  if (pmc_status st = check_hits(ctx, hits)) return st;
  if (!cache || !out) return ctx->fail(PMC_ERR_INVALID, "null cache or output");
  if (hits->n == 0) return PMC_OK;
  ShadeArgs a;
  fill_program_args(ctx, a);
  fill_cache_args(cache, a);
  a.material = hits->material;
  a.uv = hits->uv;
  a.duv = hits->duv;
  a.position = hits->position;
  a.width = hits->width;
  a.n = (uint32_t)hits->n;
  HIP_TRY(ctx, launch_debug_keys(a, out, (hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_cache_insert_raw(pmc_cache* c, const uint64_t* k0, const uint64_t* k1,
                                const uint32_t* enc, uint64_t n, uint32_t frame,
                                pmc_stats* stats, void* stream) {
  if (!c) return PMC_ERR_INVALID;
  pmc_ctx* ctx = c->ctx;
  if (pmc_status st = need_device(ctx)) return st;
  if (n && (!k0 || !k1 || !enc)) return ctx->fail(PMC_ERR_INVALID, "null raw arrays");
  if (n >= (1ull << 32)) return ctx->fail(PMC_ERR_INVALID, "too many raw inserts");
  if (n == 0) return PMC_OK;
  ShadeArgs a;
  std::memset(&a, 0, sizeof a);
  fill_cache_args(c, a);
  a.frame = frame;
  a.stat_slots = stats ? (unsigned long long*)ctx->stat_slots.p : nullptr;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(ctx, launch_insert_raw(a, k0, k1, enc, n, s));
  if (stats) HIP_TRY(ctx, launch_stats_reduce((unsigned long long*)ctx->stat_slots.p, stats, s));
  return PMC_OK;
}

pmc_status pmc_cache_lookup_raw(pmc_cache* c, const uint64_t* k0, const uint64_t* k1, uint64_t n,
                                uint32_t* enc_out, uint8_t* hit, void* stream) {
  if (!c) return PMC_ERR_INVALID;
  pmc_ctx* ctx = c->ctx;
  if (pmc_status st = need_device(ctx)) return st;
  if (n && (!k0 || !k1 || !enc_out || !hit)) return ctx->fail(PMC_ERR_INVALID, "null raw arrays");
  if (n >= (1ull << 32)) return ctx->fail(PMC_ERR_INVALID, "too many raw lookups");
  if (n == 0) return PMC_OK;
  ShadeArgs a;
  std::memset(&a, 0, sizeof a);
  fill_cache_args(c, a);
  HIP_TRY(ctx, launch_lookup_raw(a, k0, k1, n, enc_out, hit, (hipStream_t)stream));
  return PMC_OK;
}

}  // extern "C"
