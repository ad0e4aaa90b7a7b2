// surrogate_api.cpp - C entry points of the surrogate networks and the insert
// log (host side; the kernels are in surrogate.hip and shade.hip).
#include <cmath>
#include <cstring>
#include <vector>

#include "context.h"
#include "surrogate.h"

using namespace pmc;

namespace {

// SplitMix64 output mix (Steele, Lea and Flood, OOPSLA 2014), host copy.
uint64_t mix64_host(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// He-uniform weights, zero biases: w = (2 U - 1) sqrt(6 / fan_in) with U the
// top 53 bits of mix64(seed ^ (slot << 40 | layer << 32 | index)) / 2^53.
void init_params(uint64_t seed, uint32_t slot, float* p) {
  struct Layer { int off, n, fan_in; } layers[3] = {{P_W1, 64 * 32, 32}, {P_W2, 64 * 64, 64},
                                                    {P_W3, 4 * 64, 64}};
  std::memset(p, 0, sizeof(float) * kParams);
  for (int l = 0; l < 3; ++l) {
    const double lim = std::sqrt(6.0 / layers[l].fan_in);
    for (int i = 0; i < layers[l].n; ++i) {
      const uint64_t z = mix64_host(seed ^ (((uint64_t)slot << 40) | ((uint64_t)l << 32) | (uint64_t)i));
      const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
      p[layers[l].off + i] = (float)((2.0 * u - 1.0) * lim);
    }
  }
}

pmc_status need_setup(pmc_ctx* ctx) {
  if (pmc_status st = need_device(ctx)) return st;
  if (!ctx->surr.ready) return ctx->fail(PMC_ERR_STATE, "pmc_surrogate_setup was not called");
  return PMC_OK;
}

pmc_status check_slot(pmc_ctx* ctx, uint32_t slot) {
  if (slot >= ctx->surr.n_slots)
    return ctx->fail(PMC_ERR_INVALID, "slot %u out of range (%u slots)", slot, ctx->surr.n_slots);
  return PMC_OK;
}

pmc_status check_train(pmc_ctx* ctx, const pmc_train_params* p, pmc_train_params* out) {
  pmc_train_params q{};
  if (p) q = *p;
  if (q.steps == 0) q.steps = 2000;
  if (q.batch == 0) q.batch = 4096;
  if (q.lr == 0.0f) q.lr = 1e-3f;
  if (q.holdout == 0) q.holdout = 4096;
  if (q.min_records == 0) q.min_records = 1024;
  if (q.batch % 128u != 0u || q.batch > (1u << 20))
    return ctx->fail(PMC_ERR_INVALID, "batch must be a multiple of 128, at most 2^20");
  if (q.steps > 1000000u) return ctx->fail(PMC_ERR_INVALID, "at most 10^6 steps per call");
  if (!(q.lr > 0.0f) || !std::isfinite(q.lr)) return ctx->fail(PMC_ERR_INVALID, "bad lr");
  if (!(q.lr_end >= 0.0f) || !std::isfinite(q.lr_end))
    return ctx->fail(PMC_ERR_INVALID, "bad lr_end");
  if (q.workgroups > 64u || q.workgroups > q.batch / 128u)
    return ctx->fail(PMC_ERR_INVALID, "workgroups: at most 64 and batch / 128");
  *out = q;
  return PMC_OK;
}

// Workgroups per slot for a launch over n_blocks slots: the caller's choice,
// else as many as can be resident together (at most batch / 128 and 16); the
// buffers of the data-parallel exchange are sized and the step words cleared.
pmc_status train_replicas(pmc_ctx* ctx, const pmc_train_params& q, uint32_t n_blocks,
                          TrainArgs& a, hipStream_t s) {
  uint32_t r = q.workgroups;
  if (r == 0u) {
    const uint32_t cap = surr_train_capacity();
    r = n_blocks ? cap / n_blocks : 1u;
    r = std::min(r, std::min(q.batch / 128u, 16u));
  }
  if (r < 1u) r = 1u;
  a.replicas = r;
  if (r == 1u) return PMC_OK;
  SurrHost& S = ctx->surr;
  if (pmc_status st = ensure(ctx, S.partial, (size_t)n_blocks * r * kPartial * sizeof(float)))
    return st;
  if (pmc_status st = ensure(ctx, S.sync, (size_t)n_blocks * 2 * sizeof(uint32_t))) return st;
  a.partial = (float*)S.partial.p;
  a.sync = (uint32_t*)S.sync.p;
  a.spin_limit = 1u << 22;
  HIP_TRY(ctx, launch_fill_u32(a.sync, 0u, (uint64_t)n_blocks * 2, s));
  return PMC_OK;
}

SurrW* slot_w(pmc_ctx* ctx, uint32_t slot) { return (SurrW*)ctx->surr.w.p + slot; }
float* slot_master(pmc_ctx* ctx, uint32_t slot) {
  return (float*)ctx->surr.master.p + (size_t)slot * 3 * kParamStride;
}
SurrState* states(pmc_ctx* ctx) { return (SurrState*)ctx->surr.state.p; }

}  // namespace

extern "C" {

pmc_status pmc_surrogate_setup(pmc_ctx* ctx, const pmc_surrogate_opts* opts, uint32_t* n_slots) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = no_live_graphs(ctx, "surrogate_setup")) return st;
  if (!ctx->compiled) return ctx->fail(PMC_ERR_STATE, "no compiled graph set");
  pmc_surrogate_opts o{};
  if (opts) o = *opts;
  if (o.min_subgraph_nodes == 0) o.min_subgraph_nodes = 32;
  if (o.log_capacity == 0) o.log_capacity = 1u << 20;
  if (o.max_err == 0.0f) o.max_err = 1e-2f;
  if (o.log_capacity % 64u != 0u || o.log_capacity > (1u << 26))
    return ctx->fail(PMC_ERR_INVALID, "log_capacity must be a multiple of 64, at most 2^26");
  if (!(o.max_err > 0.0f)) return ctx->fail(PMC_ERR_INVALID, "max_err must be positive");

  SurrHost& S = ctx->surr;
  Program& prog = ctx->prog;
  const uint32_t n_mats = (uint32_t)prog.headers.size();
  std::vector<pmc_surrogate_slot> slots;
  std::vector<uint32_t> mat_slot(n_mats, 0xFFFFFFFFu);
  for (uint32_t m = 0; m < n_mats; ++m) {
    const pmc_material_info& in = prog.info[m];
    pmc_surrogate_slot sl{};
    sl.material = m;
    uint32_t used = 0, chan = 0;
    for (uint32_t c = 0; c < in.n_cacheable && c < 8; ++c) {
      if (in.subgraph_nodes[c] <= o.min_subgraph_nodes) continue;
      if (in.cacheable_key[c] != 0u) continue;      // the networks read UV only
      const uint32_t w = in.cacheable_type[c] == 1u ? 3u : 1u;
      if (used + w > 4u) continue;
      sl.ordinal_mask |= 1u << c;
      sl.channel[c] = used;
      chan |= used << (4 * c);
      used += w;
    }
    MatHeader& h = prog.headers[m];
    h.surr_mask = sl.ordinal_mask;
    h.surr_chan = chan;
    h.surr_slot = 0;
    if (sl.ordinal_mask) {
      sl.n_channels = used;
      h.surr_slot = (uint32_t)slots.size();
      mat_slot[m] = h.surr_slot;
      slots.push_back(sl);
    }
  }
  const uint32_t n = (uint32_t)slots.size();
  if (n > 16384u) return ctx->fail(PMC_ERR_UNSUPPORTED, "at most 16384 surrogate networks");
  if (!ctx->host_only) {
    if (pmc_status st = need_device(ctx)) return st;
    HIP_TRY(ctx, hipDeviceSynchronize());
    pmc_status st;
    const size_t nn = n ? n : 1;
    if ((st = ensure(ctx, S.w, nn * sizeof(SurrW))) ||
        (st = ensure(ctx, S.master, nn * 3 * kParamStride * sizeof(float))) ||
        (st = ensure(ctx, S.state, nn * sizeof(SurrState))) ||
        (st = ensure(ctx, S.mat_slot_dev, (size_t)(n_mats ? n_mats : 1) * 4)) ||
        (st = ensure(ctx, S.log, (size_t)o.log_capacity * sizeof(pmc_log_record))) ||
        (st = ensure(ctx, S.log_count, 64 * 4)) ||
        (st = ensure(ctx, S.slot_count, nn * 4)) || (st = ensure(ctx, S.slot_begin, nn * 4)) ||
        (st = ensure(ctx, S.slot_cursor, nn * 4)) ||
        (st = ensure(ctx, S.scan_sums, ((size_t)scan_blocks((uint32_t)nn) + 1) * 4)) ||
        (st = ensure(ctx, S.grouped, (size_t)o.log_capacity * sizeof(pmc_log_record))))
      return st;
    std::vector<float> master((size_t)nn * 3 * kParamStride, 0.0f);
    std::vector<SurrState> state(nn);
    std::memset(state.data(), 0, state.size() * sizeof(SurrState));
    for (uint32_t k = 0; k < n; ++k) {
      init_params(o.seed, k, master.data() + (size_t)k * 3 * kParamStride);
      state[k].material = slots[k].material;
      state[k].thresh = o.max_err;
      for (int c = 0; c < 8; ++c) {
        if (!((slots[k].ordinal_mask >> c) & 1u)) continue;
        const uint32_t w = prog.info[slots[k].material].cacheable_type[c] == 1u ? 3u : 1u;
        state[k].ordmap[c] = slots[k].channel[c] | (w << 4);
      }
    }
    HIP_TRY(ctx, hipMemcpy(S.master.p, master.data(), master.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(S.state.p, state.data(), state.size() * sizeof(SurrState),
                           hipMemcpyHostToDevice));
    if (n_mats)
      HIP_TRY(ctx, hipMemcpy(S.mat_slot_dev.p, mat_slot.data(), (size_t)n_mats * 4,
                             hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(ctx->hdr.p, prog.headers.data(),
                           prog.headers.size() * sizeof(MatHeader), hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemset(S.log_count.p, 0, 64 * 4));
    HIP_TRY(ctx, launch_surr_export((const float*)S.master.p, (SurrW*)S.w.p, n, nullptr));
    HIP_TRY(ctx, hipDeviceSynchronize());
  }
  S.slots = std::move(slots);
  S.mat_slot = std::move(mat_slot);
  S.n_slots = n;
  S.log_cap = o.log_capacity;
  S.max_err = o.max_err;
  S.ready = true;
  if (n_slots) *n_slots = n;
  return PMC_OK;
}

pmc_status pmc_surrogate_get_slot(const pmc_ctx* ctx, uint32_t slot, pmc_surrogate_slot* out) {
  if (!ctx || !out || !ctx->surr.ready || slot >= ctx->surr.n_slots) return PMC_ERR_INVALID;
  *out = ctx->surr.slots[slot];
  return PMC_OK;
}

pmc_status pmc_log_clear(pmc_ctx* ctx, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  HIP_TRY(ctx, launch_fill_u32((uint32_t*)ctx->surr.log_count.p, 0u, 64, (hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_log_read(pmc_ctx* ctx, pmc_log_record* host_out, uint64_t max, uint64_t* n,
                        void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (max && !host_out) return ctx->fail(PMC_ERR_INVALID, "null output");
  hipStream_t s = (hipStream_t)stream;
  uint32_t counts[64];
  HIP_TRY(ctx, hipMemcpyAsync(counts, ctx->surr.log_count.p, sizeof counts,
                              hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  const uint32_t cap = ctx->surr.log_cap / 64u;
  uint64_t held = 0, copied = 0;
  for (int r = 0; r < 64; ++r) {
    const uint64_t k = counts[r] < cap ? counts[r] : cap;
    held += k;
    const uint64_t take = copied + k <= max ? k : max - copied;
    if (take) {
      HIP_TRY(ctx, hipMemcpyAsync(host_out + copied,
                                  (pmc_log_record*)ctx->surr.log.p + (uint64_t)r * cap,
                                  take * sizeof(pmc_log_record), hipMemcpyDeviceToHost, s));
      copied += take;
    }
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  if (n) *n = held;
  return PMC_OK;
}

pmc_status pmc_surrogate_set_params(pmc_ctx* ctx, uint32_t slot, const float* host_params) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (pmc_status st = check_slot(ctx, slot)) return st;
  if (!host_params) return ctx->fail(PMC_ERR_INVALID, "null params");
  std::vector<float> blk((size_t)3 * kParamStride, 0.0f);
  std::memcpy(blk.data(), host_params, kParams * sizeof(float));
  HIP_TRY(ctx, hipDeviceSynchronize());
  HIP_TRY(ctx, hipMemcpy(slot_master(ctx, slot), blk.data(), blk.size() * 4,
                         hipMemcpyHostToDevice));
  HIP_TRY(ctx, launch_surr_export(slot_master(ctx, slot), slot_w(ctx, slot), 1, nullptr));
  HIP_TRY(ctx, launch_surr_set_trust(states(ctx), slot, 0u, 1u, nullptr));
  HIP_TRY(ctx, hipDeviceSynchronize());
  return PMC_OK;
}

pmc_status pmc_surrogate_get_params(pmc_ctx* ctx, uint32_t slot, float* host_params) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (pmc_status st = check_slot(ctx, slot)) return st;
  if (!host_params) return ctx->fail(PMC_ERR_INVALID, "null params");
  HIP_TRY(ctx, hipDeviceSynchronize());
  HIP_TRY(ctx, hipMemcpy(host_params, slot_master(ctx, slot), kParams * sizeof(float),
                         hipMemcpyDeviceToHost));
  return PMC_OK;
}

pmc_status pmc_surrogate_set_trust(pmc_ctx* ctx, uint32_t slot, int trusted, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (pmc_status st = check_slot(ctx, slot)) return st;
  HIP_TRY(ctx, launch_surr_set_trust(states(ctx), slot, trusted ? 1u : 0u, 0u,
                                     (hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_surrogate_train(pmc_ctx* ctx, const pmc_train_params* params, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  pmc_train_params q;
  if (pmc_status st = check_train(ctx, params, &q)) return st;
  SurrHost& S = ctx->surr;
  if (S.n_slots == 0) return PMC_OK;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(ctx, launch_log_group((const pmc_log_record*)S.log.p, (const uint32_t*)S.log_count.p,
                                S.log_cap / 64u, (const uint32_t*)S.mat_slot_dev.p,
                                (uint32_t)ctx->prog.headers.size(), S.n_slots,
                                (uint32_t*)S.slot_count.p, (uint32_t*)S.slot_begin.p,
                                (uint32_t*)S.slot_cursor.p, (uint32_t*)S.scan_sums.p,
                                (pmc_log_record*)S.grouped.p, s));
  TrainArgs a;
  std::memset(&a, 0, sizeof a);
  a.rec = (const pmc_log_record*)S.grouped.p;
  a.slot_begin = (const uint32_t*)S.slot_begin.p;
  a.slot_count = (const uint32_t*)S.slot_count.p;
  a.holdout = q.holdout;
  a.min_records = q.min_records;
  a.master = (float*)S.master.p;
  a.w = (SurrW*)S.w.p;
  a.state = states(ctx);
  a.steps = q.steps;
  a.batch = q.batch;
  a.lr = q.lr;
  a.lr_end = q.lr_end;
  a.seed = q.seed;
  a.sample = 1;
  if (pmc_status st = train_replicas(ctx, q, S.n_slots, a, s)) return st;
  HIP_TRY(ctx, launch_surr_train(a, S.n_slots, s));
  HIP_TRY(ctx, launch_surr_probe(a.rec, a.slot_begin, a.slot_count, q.holdout, q.min_records,
                                 a.w, a.state, S.n_slots, s));
  return PMC_OK;
}

pmc_status pmc_surrogate_train_records(pmc_ctx* ctx, uint32_t slot, const pmc_log_record* records,
                                       uint32_t n, const pmc_train_params* params, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (pmc_status st = check_slot(ctx, slot)) return st;
  pmc_train_params q;
  if (pmc_status st = check_train(ctx, params, &q)) return st;
  if (n == 0 || !records) return ctx->fail(PMC_ERR_INVALID, "no records");
  TrainArgs a;
  std::memset(&a, 0, sizeof a);
  a.rec = records;
  a.n_fixed = n;
  a.slot_fixed = slot;
  a.master = (float*)ctx->surr.master.p;
  a.w = (SurrW*)ctx->surr.w.p;
  a.state = states(ctx);
  a.steps = q.steps;
  a.batch = q.batch;
  a.lr = q.lr;
  a.lr_end = q.lr_end;
  a.seed = q.seed;
  a.sample = 1;
  if (pmc_status st = train_replicas(ctx, q, 1, a, (hipStream_t)stream)) return st;
  HIP_TRY(ctx, launch_surr_train(a, 1, (hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_surrogate_grad(pmc_ctx* ctx, uint32_t slot, const pmc_log_record* records,
                              uint32_t n, float* grads, float* loss, void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (pmc_status st = check_slot(ctx, slot)) return st;
  if (n == 0 || !records || !grads || !loss)
    return ctx->fail(PMC_ERR_INVALID, "null argument or no records");
  TrainArgs a;
  std::memset(&a, 0, sizeof a);
  a.rec = records;
  a.n_fixed = n;
  a.slot_fixed = slot;
  a.master = (float*)ctx->surr.master.p;
  a.w = (SurrW*)ctx->surr.w.p;
  a.state = states(ctx);
  a.steps = 1;
  a.sample = 0;
  a.grad_out = grads;
  a.loss_out = loss;
  HIP_TRY(ctx, launch_surr_train(a, 1, (hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_surrogate_infer(pmc_ctx* ctx, uint32_t slot, const float* uv, uint32_t n, float* y,
                               void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (pmc_status st = check_slot(ctx, slot)) return st;
  if (n && (!uv || !y)) return ctx->fail(PMC_ERR_INVALID, "null uv or y");
  if (((uintptr_t)uv & 7u) || ((uintptr_t)y & 15u))
    return ctx->fail(PMC_ERR_INVALID, "uv must be 8-byte and y 16-byte aligned");
  HIP_TRY(ctx, launch_surr_infer(slot_w(ctx, slot), uv, n, y, (hipStream_t)stream));
  return PMC_OK;
}

pmc_status pmc_surrogate_report(pmc_ctx* ctx, pmc_surrogate_stat* host_out, uint32_t n,
                                void* stream) {
  if (!ctx) return PMC_ERR_INVALID;
  if (pmc_status st = need_setup(ctx)) return st;
  if (n > ctx->surr.n_slots) return ctx->fail(PMC_ERR_INVALID, "n beyond the slot count");
  if (n && !host_out) return ctx->fail(PMC_ERR_INVALID, "null output");
  if (n == 0) return PMC_OK;
  std::vector<SurrState> st(n);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(ctx, hipMemcpyAsync(st.data(), ctx->surr.state.p, n * sizeof(SurrState),
                              hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  for (uint32_t k = 0; k < n; ++k) {
    pmc_surrogate_stat& o = host_out[k];
    std::memset(&o, 0, sizeof o);
    o.material = st[k].material;
    o.trusted = st[k].trusted;
    o.n_train = st[k].n_train;
    o.n_heldout = st[k].n_heldout;
    o.max_err = st[k].max_err;
    o.mean_err = st[k].mean_err;
    o.loss = st[k].loss;
    uint32_t bits = st[k].live_err_bits;
    std::memcpy(&o.live_max_err, &bits, 4);
    o.steps = st[k].steps;
    o.live_checked = st[k].live_n;
  }
  return PMC_OK;
}

}  // extern "C"
