// frame.cpp - progressive frames as one HIP graph, and the launch-parameter
// autotuner.
//
// A progressive render shades frame after frame against one table (Sec. 1,
// Sec. 3: values inserted while rendering are reused by later frames).  The
// whole sequence is captured once into a HIP graph and replayed: every
// per-frame parameter (frame index, hit and output offsets) is baked into
// the captured kernel arguments, and all workspace is reserved before
// capture so that replays allocate nothing.
#include <chrono>
#include <cstring>
#include <string>

#include "context.h"

using namespace pmc;

struct pmc_frame_graph {
  pmc_ctx* ctx = nullptr;
  pmc_cache* cache = nullptr;    // the table it replays into (NULL: uncached)
  int device = 0;
  bool counted = false;          // registered with ctx (and cache)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

pmc_hits frame_hits(const pmc_frame_plan* p, uint32_t f) {
  pmc_hits h = p->hits;
  const uint64_t o = (uint64_t)f * p->hits_per_frame;
  h.material = p->hits.material + o;
  h.uv = p->hits.uv + 2 * o;
  h.duv = p->hits.duv + 4 * o;
  h.normal = p->hits.normal + 3 * o;
  h.bounce = p->hits.bounce ? p->hits.bounce + o : nullptr;
  h.position = p->hits.position ? p->hits.position + 3 * o : nullptr;
  h.width = p->hits.width ? p->hits.width + o : nullptr;
  h.n = p->hits_per_frame;
  return h;
}

pmc_bsdf_out frame_out(const pmc_frame_plan* p, uint32_t f) {
  pmc_bsdf_out o = p->out;
  const uint64_t k = p->out_per_frame ? (uint64_t)f * p->hits_per_frame : 0;
  o.base_color = p->out.base_color + 3 * k;
  o.roughness = p->out.roughness + k;
  o.normal = p->out.normal + 3 * k;
  return o;
}

pmc_status check_plan(pmc_ctx* ctx, pmc_cache* cache, const pmc_frame_plan* p) {
  if (!p) return ctx->fail(PMC_ERR_INVALID, "null plan");
  if (p->n_frames == 0 || p->hits_per_frame == 0)
    return ctx->fail(PMC_ERR_INVALID, "plan needs frames and hits");
  pmc_hits h0 = frame_hits(p, 0);
  pmc_bsdf_out o0 = frame_out(p, 0);
  if (pmc_status st = check_shade_args(ctx, cache, &h0, &o0, &p->params)) return st;
  if (p->params.mode != PMC_MODE_UNCACHED && !cache)
    return ctx->fail(PMC_ERR_INVALID, "cached plan without a cache");
  if (p->late_frame) {
    if (p->late_frame >= p->n_frames)
      return ctx->fail(PMC_ERR_INVALID, "late_frame must be below n_frames");
    if (p->late_params.mode != p->params.mode)
      return ctx->fail(PMC_ERR_INVALID, "late_params must keep the plan's mode");
    if (pmc_status st = check_shade_args(ctx, cache, &h0, &o0, &p->late_params)) return st;
  }
  return PMC_OK;
}

// Workspace for every setting the plan uses (eight sets each, for a frame graph).
pmc_status reserve_plan(pmc_ctx* ctx, pmc_cache* cache, const pmc_frame_plan* p,
                        const pmc_shade_params& early, const pmc_shade_params& late,
                        bool all_sets, hipStream_t s) {
  const uint32_t mode = cache ? early.mode : PMC_MODE_UNCACHED;
  for (int k = 0; k < (p->late_frame ? 2 : 1); ++k) {
    const pmc_shade_params& q = k ? late : early;
    const bool probe_first = mode != PMC_MODE_UNCACHED && (q.flags & PMC_FLAG_DEFER);
    if (pmc_status st = reserve_batch(ctx, cache, (uint32_t)p->hits_per_frame, mode, q.flags,
                                      resolve_chunk_waves(q.chunk_waves, probe_first), all_sets,
                                      s))
      return st;
  }
  return PMC_OK;
}

// Streams and events of a pipelined capture: the material sorts run on `side`,
// one group of frames ahead of the shading on the origin stream.
struct Pipe {
  hipStream_t side = nullptr;
  hipEvent_t start = nullptr, join = nullptr;
  hipEvent_t sorted[2] = {nullptr, nullptr}, shaded[2] = {nullptr, nullptr};
};

// Enqueue the plan's work on s (no validation).  With a pipe (and a sorted,
// multi-frame plan) the frames are taken in groups, {0}, then kPipeGroup frames
// at a time; frame f uses workspace set f % kWorkSets, and
//   the sorts of group g+1 run on the side stream after those of group g
//   (stream order) and after the shading of group g-1, the last user of their
//   sets (two consecutive groups span at most kWorkSets frames);
//   the shading of group g on s waits once, for the sorts of group g;
// so the sorts of the next group overlap the shading of the current one, and
// only the first frame of a group waits on the other stream.  The workspace
// must be reserved for all sets.
constexpr uint32_t kPipeGroup = kWorkSets / 2;

pmc_status enqueue_plan(pmc_ctx* ctx, pmc_cache* cache, const pmc_frame_plan* p,
                        const pmc_shade_params& early, const pmc_shade_params& late,
                        hipStream_t s, const Pipe* pipe) {
  // frames from late_frame on use `late` (when the plan sets late_frame)
  auto params_of = [&](uint32_t f) {
    pmc_shade_params q = (p->late_frame && f >= p->late_frame) ? late : early;
    q.frame = p->first_frame + f;
    return q;
  };
  // the sort stream runs ahead only when every frame is sorted
  const bool all_sorted = (early.flags & PMC_FLAG_SORT) &&
                          (!p->late_frame || (late.flags & PMC_FLAG_SORT));
  const bool piped = pipe && all_sorted && p->n_frames >= 2;
  if (piped) {
    // fork before the table clear: the first sort does not wait for it
    HIP_TRY(ctx, hipEventRecord(pipe->start, s));
    HIP_TRY(ctx, hipStreamWaitEvent(pipe->side, pipe->start, 0));
  }
  if (p->clear_cache && cache) {
    const hipError_t e = launch_fill_u64((uint64_t*)cache->mem, 0ull, cache->bytes / 8, s);
    if (e != hipSuccess && piped) {
      (void)hipEventRecord(pipe->join, pipe->side);
      (void)hipStreamWaitEvent(s, pipe->join, 0);
    }
    HIP_TRY(ctx, e);
  }
  if (!piped) {
    for (uint32_t f = 0; f < p->n_frames; ++f) {
      pmc_hits h = frame_hits(p, f);
      pmc_bsdf_out o = frame_out(p, f);
      const pmc_shade_params q = params_of(f);
      if (pmc_status st = shade_batch(ctx, cache, &h, &o, &q, p->stats, nullptr, s)) return st;
    }
    return PMC_OK;
  }
  const hipStream_t side = pipe->side;
  const uint32_t F = p->n_frames;
  const uint32_t n_groups = 1u + (F - 1u + kPipeGroup - 1u) / kPipeGroup;
  auto group_begin = [&](uint32_t g) { return g == 0 ? 0u : 1u + (g - 1u) * kPipeGroup; };
  auto group_end = [&](uint32_t g) { return g + 1 >= n_groups ? F : group_begin(g + 1); };
  auto sort_group = [&](uint32_t g) -> pmc_status {
    for (uint32_t f = group_begin(g); f < group_end(g); ++f) {
      pmc_hits h = frame_hits(p, f);
      const pmc_shade_params q = params_of(f);
      if (pmc_status st = sort_stage(ctx, cache, &h, &q, (int)(f % kWorkSets), side)) return st;
    }
    if (hipEventRecord(pipe->sorted[g & 1u], side) != hipSuccess)
      return ctx->fail(PMC_ERR_HIP, "hipEventRecord failed");
    return PMC_OK;
  };
  pmc_status st = sort_group(0);
  for (uint32_t g = 0; st == PMC_OK && g < n_groups; ++g) {
    if (hipStreamWaitEvent(s, pipe->sorted[g & 1u], 0) != hipSuccess) {
      st = ctx->fail(PMC_ERR_HIP, "hipStreamWaitEvent failed");
      break;
    }
    for (uint32_t f = group_begin(g); st == PMC_OK && f < group_end(g); ++f) {
      pmc_hits h = frame_hits(p, f);
      pmc_bsdf_out o = frame_out(p, f);
      const pmc_shade_params q = params_of(f);
      st = shade_stage(ctx, cache, &h, &o, &q, p->stats, nullptr, (int)(f % kWorkSets), s);
    }
    if (st == PMC_OK && hipEventRecord(pipe->shaded[g & 1u], s) != hipSuccess)
      st = ctx->fail(PMC_ERR_HIP, "hipEventRecord failed");
    if (st != PMC_OK || g + 1 == n_groups) break;
    if (g >= 1 && hipStreamWaitEvent(side, pipe->shaded[(g - 1u) & 1u], 0) != hipSuccess) {
      st = ctx->fail(PMC_ERR_HIP, "hipStreamWaitEvent failed");
      break;
    }
    st = sort_group(g + 1);
  }
  // the side stream joins the origin stream again, on every path
  if (hipEventRecord(pipe->join, side) != hipSuccess ||
      hipStreamWaitEvent(s, pipe->join, 0) != hipSuccess) {
    if (st == PMC_OK) st = ctx->fail(PMC_ERR_HIP, "joining the sort stream failed");
  }
  return st;
}

}  // namespace

extern "C" {

pmc_status pmc_frame_graph_create(pmc_ctx* ctx, pmc_cache* cache, const pmc_frame_plan* plan,
                                  pmc_frame_graph** out) {
  if (!ctx || !out) return PMC_ERR_INVALID;
  *out = nullptr;
  if (pmc_status st = check_plan(ctx, cache, plan)) return st;
  hipStream_t cs = nullptr;
  HIP_TRY(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  pmc_status st = reserve_plan(ctx, cache, plan, plan->params, plan->late_params, true, cs);
  Pipe pipe;
  if (st == PMC_OK) {
    bool ok = hipStreamCreateWithFlags(&pipe.side, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t* e : {&pipe.start, &pipe.join, &pipe.sorted[0], &pipe.sorted[1],
                          &pipe.shaded[0], &pipe.shaded[1]})
      ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    if (!ok) st = ctx->fail(PMC_ERR_HIP, "stream or event creation failed");
  }
  if (st == PMC_OK && hipStreamSynchronize(cs) != hipSuccess)
    st = ctx->fail(PMC_ERR_HIP, "workspace reservation failed");
  pmc_frame_graph* g = nullptr;
  if (st == PMC_OK) {
    g = new (std::nothrow) pmc_frame_graph();
    if (!g) st = PMC_ERR_OOM;
  }
  if (st == PMC_OK) {
    g->ctx = ctx;
    g->device = ctx->device;
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    ctx->no_alloc = true;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      st = ctx->fail(PMC_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    } else {
      st = enqueue_plan(ctx, cache, plan, plan->params, plan->late_params, cs, &pipe);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(cs, &graph);
      if (st == PMC_OK && e != hipSuccess)
        st = ctx->fail(PMC_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
      g->graph = graph;
    }
    ctx->no_alloc = false;
    ctx->profiling = prof;
    if (st == PMC_OK) {
      e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (e != hipSuccess)
        st = ctx->fail(PMC_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
  }
  (void)hipStreamDestroy(cs);
  for (hipEvent_t e : {pipe.start, pipe.join, pipe.sorted[0], pipe.sorted[1], pipe.shaded[0],
                       pipe.shaded[1]})
    if (e) (void)hipEventDestroy(e);
  if (pipe.side) (void)hipStreamDestroy(pipe.side);
  if (st != PMC_OK) {
    pmc_frame_graph_destroy(g);
    return st;
  }
  g->counted = true;
  ++ctx->live_graphs;
  if (cache) {
    g->cache = cache;
    ++cache->live_graphs;
  }
  *out = g;
  return PMC_OK;
}

pmc_status pmc_frame_graph_launch(pmc_frame_graph* g, void* stream) {
  if (!g || !g->exec) return PMC_ERR_INVALID;
  pmc_ctx* ctx = g->ctx;
  HIP_TRY(ctx, hipSetDevice(g->device));
  HIP_TRY(ctx, hipGraphLaunch(g->exec, (hipStream_t)stream));
  return PMC_OK;
}

void pmc_frame_graph_destroy(pmc_frame_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->exec) {
    (void)hipDeviceSynchronize();                 // no replay may still be running
    (void)hipGraphExecDestroy(g->exec);
  }
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->counted) {
    pmc_cache* c = g->cache;
    if (c && --c->live_graphs == 0 && c->orphaned) destroy_cache(c);
    pmc_ctx* ctx = g->ctx;
    if (--ctx->live_graphs == 0 && ctx->orphaned) destroy_context(ctx);
  }
  delete g;
}

pmc_status pmc_autotune(pmc_ctx* ctx, pmc_cache* cache, const pmc_frame_plan* plan,
                        pmc_tune_result* out, const char* json_path) {
  if (!ctx || !out) return PMC_ERR_INVALID;
  if (pmc_status st = check_plan(ctx, cache, plan)) return st;
  std::memset(out, 0, sizeof *out);
  hipStream_t s = nullptr;
  HIP_TRY(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const bool cached = cache && plan->params.mode != PMC_MODE_UNCACHED;
  pmc_frame_plan p = *plan;
  p.clear_cache = cached ? 1u : 0u;
  p.stats = nullptr;

  struct Cand { uint32_t flags, chunk_waves, defer_max, bpc, wpb; double ms; };
  std::vector<Cand> cands;
  // the surrogate choice is the caller's (it changes results); logging is not
  // wanted while tuning
  const uint32_t base =
      PMC_FLAG_SORT | (plan->params.flags & (PMC_FLAG_SURROGATE | PMC_FLAG_SURROGATE_INSERT));
  for (uint32_t pers = 0; pers < 2; ++pers) {
    const uint32_t pf = pers ? PMC_FLAG_PERSISTENT : 0u;
    for (uint32_t cw : {1u, 2u, 4u}) cands.push_back({base | pf, cw, 0u, 0u, 0u, 0.0});
    if (cached)
      for (uint32_t cw : {2u, 4u, 8u})
        for (uint32_t dm : {32u, 48u})
          cands.push_back({base | pf | PMC_FLAG_DEFER, cw, dm, 0u, 0u, 0.0});
  }
  for (uint32_t bpc : {2u, 4u}) cands.push_back({base | PMC_FLAG_PERSISTENT, 1u, 0u, bpc, 0u, 0.0});
  if (cached)
    for (uint32_t cw : {1u, 2u, 4u})
      cands.push_back({base | PMC_FLAG_PERSISTENT | PMC_FLAG_DEFER, cw, 48u, 4u, 0u, 0.0});
  // (smaller workgroups, waves_per_block 1 or 2, measured within 0.3% of 4 on
  // the 64-material scene and are left to the caller)

  pmc_status st = PMC_OK;
  auto time_one = [&](const pmc_shade_params& prm, double* ms) -> pmc_status {
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {           // first run warms up
      HIP_TRY(ctx, hipEventRecord(e0, s));
      // with late_frame, the candidate is the late setting; the early frames keep the plan's
      const pmc_shade_params& early = p.late_frame ? plan->params : prm;
      if (pmc_status r = enqueue_plan(ctx, cache, &p, early, prm, s, nullptr)) return r;
      HIP_TRY(ctx, hipEventRecord(e1, s));
      HIP_TRY(ctx, hipEventSynchronize(e1));
      float t = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&t, e0, e1));
      if (rep > 0 && t < best) best = t;
    }
    *ms = best;
    return PMC_OK;
  };
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  pmc_shade_params def = plan->params;
  def.flags = base;
  def.chunk_waves = def.defer_max = def.blocks_per_cu = def.waves_per_block = 0;
  st = time_one(def, &out->default_ms);
  double best_ms = 1e30;
  size_t best_i = 0;
  for (size_t i = 0; st == PMC_OK && i < cands.size(); ++i) {
    pmc_shade_params prm = plan->params;
    prm.flags = cands[i].flags;
    prm.chunk_waves = cands[i].chunk_waves;
    prm.defer_max = cands[i].defer_max;
    prm.blocks_per_cu = cands[i].bpc;
    prm.waves_per_block = cands[i].wpb;
    st = time_one(prm, &cands[i].ms);
    if (st == PMC_OK && cands[i].ms < best_ms) {
      best_ms = cands[i].ms;
      best_i = i;
    }
  }
  ctx->profiling = prof;
  if (st == PMC_OK && cached) {
    (void)launch_fill_u64((uint64_t*)cache->mem, 0ull, cache->bytes / 8, s);
    (void)hipStreamSynchronize(s);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (st != PMC_OK) return st;
  out->best = plan->params;
  out->best.flags = cands[best_i].flags;
  out->best.chunk_waves = cands[best_i].chunk_waves;
  out->best.defer_max = cands[best_i].defer_max;
  out->best.blocks_per_cu = cands[best_i].bpc;
  out->best.waves_per_block = cands[best_i].wpb;
  out->best_ms = best_ms;
  out->n_tried = (uint32_t)cands.size();
  if (json_path) {
    FILE* fp = std::fopen(json_path, "w");
    if (!fp) return ctx->fail(PMC_ERR_INVALID, "cannot write %s", json_path);
    std::fprintf(fp, "{\"default_ms\": %.6f, \"best\": %zu, \"candidates\": [", out->default_ms,
                 best_i);
    for (size_t i = 0; i < cands.size(); ++i)
      std::fprintf(fp, "%s{\"flags\": %u, \"chunk_waves\": %u, \"defer_max\": %u, "
                   "\"blocks_per_cu\": %u, \"waves_per_block\": %u, \"ms\": %.6f}",
                   i ? ", " : "", cands[i].flags, cands[i].chunk_waves, cands[i].defer_max,
                   cands[i].bpc, cands[i].wpb, cands[i].ms);
    std::fprintf(fp, "]}\n");
    std::fclose(fp);
  }
  return PMC_OK;
}

}  // extern "C"
