// compiler.cpp - validation, constant folding, cacheable marking, need masks,
// register allocation and bytecode emission for material graph sets.
//
// Paper passages followed:
//   Sec. 2   networks become data read and executed in storage order; simple
//            arithmetic nodes with constant inputs are pre-computed.
//   Sec. 3   cacheable nodes are marked by a bottom-to-top traversal during
//            that same optimisation pass, at the highest level whose
//            sub-graph depends on no shading-point datum other than UV; a
//            material can have several.
//   Sec. 3.1 sub-graphs reading other shading-point data are not cacheable.
//
// Rule used for "highest level": a node's class is the set of shading-point
// data its value depends on (UV; POS, the world position, which Sec. 3.1 names
// as other information a descriptor can hold; SP, any other datum).  An output
// socket of a node whose class is exactly UV or exactly POS is cacheable when
// one of its consumers has another class or is the BSDF sink, and its
// sub-graph has at least `min_subgraph_nodes` nodes besides UV inputs.  A UV
// output is keyed by a UV texel, a POS output by a world-space cell.
//
// Need masks: with miss_mask the per-lane set of cacheable outputs that were
// not found, a node runs for a lane iff (exec & kAlways) || (exec & miss_mask).
// exec is built top-down: a cacheable socket contributes its own bit (its
// sub-graph runs only when its lookup missed), any other socket contributes
// the union of its consumers' masks, the sink contributes kAlways.  Because
// every cacheable socket has an always-needed consumer, this one-level mask
// is exact.  With every lookup missing (cache off) all nodes run, so the
// cache-disabled path is plain evaluation.
#include "compiler.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace pmc {
namespace {

enum Cls { C_CONST = 0, C_UV = 1, C_POS = 2, C_SP = 4 };   // a class is a union of these

constexpr int kNumOps = 10;
const int kNumIn[kNumOps] = {0, 1, 1, 1, 3, 2, 1, 2, 3, 0};
const int kNumOut[kNumOps] = {1, 2, 1, 1, 1, 1, 2, 1, 0, 1};

uint8_t in_type(uint32_t op, int k) {
  switch (op) {
    case PMC_OP_IMAGE_TEXTURE: case PMC_OP_VALUE_NOISE: case PMC_OP_PERLIN_NOISE: return OT_UV;
    case PMC_OP_MIX: return k == 0 ? OT_FLOAT : OT_COLOR;
    case PMC_OP_MATH: return OT_FLOAT;
    case PMC_OP_COLOR_RAMP: return OT_FLOAT;
    case PMC_OP_NORMAL_MAP: return k == 0 ? OT_COLOR : OT_FLOAT;
    case PMC_OP_BSDF_OUTPUT: return k == 0 ? OT_COLOR : (k == 1 ? OT_FLOAT : OT_VECTOR);
    default: return OT_FLOAT;
  }
}

uint8_t out_type(uint32_t op, int s) {
  switch (op) {
    case PMC_OP_UV_INPUT: return OT_UV;
    case PMC_OP_IMAGE_TEXTURE: case PMC_OP_COLOR_RAMP: return s == 0 ? OT_COLOR : OT_FLOAT;
    case PMC_OP_MIX: return OT_COLOR;
    case PMC_OP_NORMAL_MAP: return OT_VECTOR;
    default: return OT_FLOAT;
  }
}

bool convertible(uint8_t src, uint8_t dst) {
  if (src == dst) return true;
  return (src == OT_FLOAT || src == OT_COLOR) && (dst == OT_FLOAT || dst == OT_COLOR);
}

int width_of(uint8_t t) { return t == OT_FLOAT ? 1 : 3; }

// ---- FP32 host evaluation of constant-foldable nodes ------------------------

struct Val { float v[3]; };

float clamp01(float x) { return x < 0.f ? 0.f : (x > 1.f ? 1.f : x); }

Val as_type(const Val& x, uint8_t src, uint8_t dst) {
  if (src == dst) return x;
  Val r{};
  if (src == OT_COLOR && dst == OT_FLOAT) {
    r.v[0] = (x.v[0] + x.v[1] + x.v[2]) / 3.0f;
  } else {
    r.v[0] = r.v[1] = r.v[2] = x.v[0];
  }
  return r;
}

void ramp_eval(const pmc_node_desc& n, float fac, float out[4]) {
  const float* p = n.ramp_pos;
  if (!(fac > p[0])) {
    for (int c = 0; c < 4; ++c) out[c] = n.ramp_rgba[0][c];
    return;
  }
  if (fac >= p[7]) {
    for (int c = 0; c < 4; ++c) out[c] = n.ramp_rgba[7][c];
    return;
  }
  int k = 0;
  while (k < 6 && fac >= p[k + 1]) ++k;
  float t = (fac - p[k]) / (p[k + 1] - p[k]);
  for (int c = 0; c < 4; ++c) {
    float a = n.ramp_rgba[k][c], b = n.ramp_rgba[k + 1][c];
    out[c] = a + t * (b - a);
  }
}

// Integer hash (C. Wellons' "lowbias32" finalizer) for scrambled visiting orders.
inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

constexpr uint32_t kOrderVariants = 32;   // alternative emission orders tried per material
constexpr uint32_t kRegsGoal = 24;        // registers at which no further order is tried

struct MatCompiler {
  uint32_t mat;
  const pmc_node_desc* nd;
  uint32_t n;
  uint32_t min_nodes;
  bool fold;
  bool world_keys = true;                 // outputs of the world position are cacheable
  std::string& err;

  std::vector<uint8_t> live, cls, folded;
  std::vector<int> order;                 // emission order (node ids)
  std::vector<int> need;                  // Sethi-Ullman register need per node
  std::vector<std::array<int, 3>> child_order;   // inputs in visiting order
  std::vector<int> pos;                   // emission position, -1 if not emitted
  std::vector<std::vector<std::pair<int, int>>> consumers;  // per (node): (consumer, input slot)
  std::vector<Val> fval[2];               // folded value per socket
  std::vector<std::pair<int, int>> cach;  // cacheable (node, socket)
  std::vector<int> cach_sub;              // sub-graph sizes
  std::vector<int> sock_ord[2];           // cacheable ordinal of (node, socket) or -1
  std::vector<uint32_t> exec;
  std::vector<int> reg[2];                // register base per socket, -1 if none
  int sink = -1;
  uint32_t n_regs = 0;

  MatCompiler(uint32_t m, const pmc_node_desc* nodes, uint32_t count, uint32_t min_n, bool f,
              std::string& e)
      : mat(m), nd(nodes), n(count), min_nodes(min_n), fold(f), err(e) {}

  bool fail(uint32_t node, const char* what) {
    char buf[256];
    snprintf(buf, sizeof buf, "material %u node %u: %s", mat, node, what);
    err = buf;
    return false;
  }

  bool validate() {
    if (n == 0) return fail(0, "material has no nodes");
    for (uint32_t i = 0; i < n; ++i) {
      const pmc_node_desc& d = nd[i];
      if (d.op >= kNumOps) return fail(i, "unknown op");
      if (d.op == PMC_OP_BSDF_OUTPUT) {
        if (sink >= 0) return fail(i, "more than one BSDF_OUTPUT");
        sink = int(i);
      }
      if ((d.op == PMC_OP_VALUE_NOISE || d.op == PMC_OP_PERLIN_NOISE ||
           d.op == PMC_OP_POSITION_NOISE) &&
          (d.octaves < 1 || d.octaves > 8 || !std::isfinite(d.freq)))
        return fail(i, "noise needs 1..8 octaves and a finite frequency");
      if (d.op == PMC_OP_MATH && d.variant > PMC_MATH_POW) return fail(i, "unknown math op");
      if (d.op == PMC_OP_COLOR_RAMP) {
        for (int k = 0; k < 7; ++k)
          if (!(d.ramp_pos[k] <= d.ramp_pos[k + 1])) return fail(i, "ramp stops not ascending");
      }
      for (int k = 0; k < kNumIn[d.op]; ++k) {
        const pmc_input& in = d.in[k];
        if (in.node < 0) continue;
        if (uint32_t(in.node) >= n) return fail(i, "input links past the end");
        uint32_t sop = nd[in.node].op;
        if (sop >= kNumOps) return fail(uint32_t(in.node), "unknown op");
        if (int(in.socket) >= kNumOut[sop]) return fail(i, "input names a missing socket");
        if (!convertible(out_type(sop, int(in.socket)), in_type(d.op, k)))
          return fail(i, "input type mismatch");
      }
    }
    if (sink < 0) return fail(0, "no BSDF_OUTPUT node");
    // acyclic (iterative DFS with colours)
    std::vector<uint8_t> colour(n, 0);
    std::vector<std::pair<int, int>> stack;
    for (uint32_t s = 0; s < n; ++s) {
      if (colour[s]) continue;
      stack.push_back({int(s), 0});
      colour[s] = 1;
      while (!stack.empty()) {
        auto& top = stack.back();
        const pmc_node_desc& d = nd[top.first];
        if (top.second < kNumIn[d.op]) {
          int k = top.second++;
          int j = d.in[k].node;
          if (j < 0) continue;
          if (colour[j] == 1) return fail(uint32_t(top.first), "cycle");
          if (colour[j] == 0) {
            colour[j] = 1;
            stack.push_back({j, 0});
          }
        } else {
          colour[top.first] = 2;
          stack.pop_back();
        }
      }
    }
    return true;
  }

  void analyse() {
    live.assign(n, 0);
    std::vector<int> st{sink};
    while (!st.empty()) {
      int i = st.back();
      st.pop_back();
      if (live[i]) continue;
      live[i] = 1;
      for (int k = 0; k < kNumIn[nd[i].op]; ++k)
        if (nd[i].in[k].node >= 0) st.push_back(nd[i].in[k].node);
    }
    // Emission order: post-order DFS from the sink.  Inputs are visited in
    // decreasing register need (Sethi-Ullman order, a heuristic on DAGs) so
    // that few values are live at once.
    std::vector<int> topo;                    // inputs before consumers (slot order)
    {
      std::vector<uint8_t> seen(n, 0);
      std::vector<std::pair<int, int>> st{{sink, 0}};
      seen[sink] = 1;
      while (!st.empty()) {
        auto& top = st.back();
        const pmc_node_desc& d = nd[top.first];
        if (top.second < kNumIn[d.op]) {
          int j = d.in[top.second++].node;
          if (j >= 0 && !seen[j]) {
            seen[j] = 1;
            st.push_back({j, 0});
          }
        } else {
          topo.push_back(top.first);
          st.pop_back();
        }
      }
    }
    std::vector<int> width(n, 0);
    need.assign(n, 0);
    child_order.assign(n, {-1, -1, -1});
    for (int i : topo) {
      const pmc_node_desc& d = nd[i];
      int w = 0;
      for (int s = 0; s < kNumOut[d.op]; ++s) w += d.op == PMC_OP_UV_INPUT ? 0 : width_of(out_type(d.op, s));
      width[i] = w;
      std::array<int, 3> ch{-1, -1, -1};
      int nc = 0;
      for (int k = 0; k < kNumIn[d.op]; ++k) {
        int j = d.in[k].node;
        if (j < 0) continue;
        bool dup = false;
        for (int q = 0; q < nc; ++q) dup |= ch[q] == j;
        if (!dup) ch[nc++] = j;
      }
      std::sort(ch.begin(), ch.begin() + nc, [&](int a, int b) { return need[a] > need[b]; });
      int nd_need = w, held = 0;
      for (int q = 0; q < nc; ++q) {
        nd_need = std::max(nd_need, held + need[ch[q]]);
        held += width[ch[q]];
      }
      need[i] = std::max(nd_need, held + w);
      child_order[i] = ch;
    }
    std::vector<uint8_t> done(n, 0);
    std::vector<std::pair<int, int>> stack{{sink, 0}};
    std::vector<int> post;
    done[sink] = 1;
    while (!stack.empty()) {
      auto& top = stack.back();
      if (top.second < 3) {
        int j = child_order[top.first][top.second++];
        if (j >= 0 && !done[j]) {
          done[j] = 1;
          stack.push_back({j, 0});
        }
      } else {
        post.push_back(top.first);
        stack.pop_back();
      }
    }
    // dependency classes, inputs first
    cls.assign(n, C_CONST);
    for (int i : post) {
      const pmc_node_desc& d = nd[i];
      int c = C_CONST;
      if (d.op == PMC_OP_UV_INPUT || d.op == PMC_OP_IMAGE_TEXTURE || d.op == PMC_OP_VALUE_NOISE ||
          d.op == PMC_OP_PERLIN_NOISE)
        c = C_UV;
      if (d.op == PMC_OP_POSITION_NOISE) c = C_POS;
      if (d.op == PMC_OP_NORMAL_MAP) c = C_SP;
      for (int k = 0; k < kNumIn[d.op]; ++k)
        if (d.in[k].node >= 0) c |= cls[d.in[k].node];
      cls[i] = uint8_t(c);
    }
    consumers.assign(n, {});
    for (int i : post)
      for (int k = 0; k < kNumIn[nd[i].op]; ++k)
        if (nd[i].in[k].node >= 0) consumers[nd[i].in[k].node].push_back({i, k});
    // constant folding (Sec. 2): MATH / MIX / COLOR_RAMP whose inputs are all constant
    folded.assign(n, 0);
    fval[0].assign(n, Val{});
    fval[1].assign(n, Val{});
    if (fold) {
      for (int i : post) {
        const pmc_node_desc& d = nd[i];
        if (cls[i] != C_CONST || i == sink) continue;
        if (d.op != PMC_OP_MATH && d.op != PMC_OP_MIX && d.op != PMC_OP_COLOR_RAMP) continue;
        Val in[3];
        for (int k = 0; k < kNumIn[d.op]; ++k) in[k] = const_input(i, k);
        if (d.op == PMC_OP_MATH) {
          float a = in[0].v[0], b = in[1].v[0], r;
          if (d.variant == PMC_MATH_ADD) r = a + b;
          else if (d.variant == PMC_MATH_MUL) r = a * b;
          else r = a > 0.f ? std::pow(a, b) : 0.f;
          if (d.flags & PMC_NODE_CLAMP) r = clamp01(r);
          fval[0][i].v[0] = r;
        } else if (d.op == PMC_OP_MIX) {
          float t = clamp01(in[0].v[0]);
          for (int c = 0; c < 3; ++c) fval[0][i].v[c] = in[1].v[c] + t * (in[2].v[c] - in[1].v[c]);
        } else {
          float o[4];
          ramp_eval(d, in[0].v[0], o);
          for (int c = 0; c < 3; ++c) fval[0][i].v[c] = o[c];
          fval[1][i].v[0] = o[3];
        }
        folded[i] = 1;
      }
    }
    pos.assign(n, -1);
    for (int i : post) {
      uint32_t op = nd[i].op;
      if (i == sink || op == PMC_OP_UV_INPUT || folded[i]) continue;
      pos[i] = int(order.size());
      order.push_back(i);
    }
  }

  // value of a constant input (unconnected, or a folded node), converted to the input type
  Val const_input(int i, int k) {
    const pmc_input& in = nd[i].in[k];
    uint8_t want = in_type(nd[i].op, k);
    if (in.node < 0) {
      Val r{};
      for (int c = 0; c < 3; ++c) r.v[c] = in.value[c];
      if (want == OT_FLOAT) r.v[1] = r.v[2] = 0.f;
      return r;
    }
    int s = int(in.socket);
    return as_type(fval[s][in.node], out_type(nd[in.node].op, s), want);
  }

  int subgraph_size(int root) {
    std::vector<uint8_t> seen(n, 0);
    std::vector<int> st{root};
    int count = 0;
    while (!st.empty()) {
      int i = st.back();
      st.pop_back();
      if (seen[i]) continue;
      seen[i] = 1;
      if (nd[i].op != PMC_OP_UV_INPUT) ++count;
      for (int k = 0; k < kNumIn[nd[i].op]; ++k)
        if (nd[i].in[k].node >= 0) st.push_back(nd[i].in[k].node);
    }
    return count;
  }

  void mark_cacheable() {
    sock_ord[0].assign(n, -1);
    sock_ord[1].assign(n, -1);
    for (uint32_t i = 0; i < n; ++i) {
      uint32_t op = nd[i].op;
      const bool keyable = cls[i] == C_UV || (cls[i] == C_POS && world_keys);
      if (!live[i] || !keyable || op == PMC_OP_UV_INPUT || op == PMC_OP_BSDF_OUTPUT) continue;
      int size = -1;
      for (int s = 0; s < kNumOut[op]; ++s) {
        bool boundary = false;
        for (auto& ck : consumers[i]) {
          if (int(nd[ck.first].in[ck.second].socket) != s) continue;
          if (ck.first == sink || cls[ck.first] != cls[i]) boundary = true;
        }
        if (!boundary) continue;
        if (size < 0) size = subgraph_size(int(i));
        if (size < int(min_nodes)) continue;
        if (int(cach.size()) >= kMaxCach) continue;  // beyond the cap: stays uncached
        sock_ord[s][i] = int(cach.size());
        cach.push_back({int(i), s});
        cach_sub.push_back(size);
      }
    }
  }

  void need_masks() {
    exec.assign(n, 0);
    for (int p = int(order.size()) - 1; p >= 0; --p) {
      int i = order[p];
      uint32_t m = 0;
      for (int s = 0; s < kNumOut[nd[i].op]; ++s) {
        if (sock_ord[s][i] >= 0) {
          m |= 1u << sock_ord[s][i];
          continue;
        }
        for (auto& ck : consumers[i]) {
          if (int(nd[ck.first].in[ck.second].socket) != s) continue;
          m |= (ck.first == sink) ? kAlways : exec[ck.first];
        }
      }
      exec[i] = m;
    }
  }

  bool socket_used(int i, int s) const {
    if (sock_ord[s][i] >= 0) return true;
    for (auto& ck : consumers[i])
      if (int(nd[ck.first].in[ck.second].socket) == s && (ck.first == sink || pos[ck.first] >= 0))
        return true;
    return false;
  }

  // Emission order: post-order of a depth-first walk from the sink that visits
  // each node's inputs in the order co gives.
  std::vector<int> emission_order(const std::vector<std::array<int, 3>>& co) const {
    std::vector<uint8_t> done(n, 0);
    std::vector<std::pair<int, int>> stack{{sink, 0}};
    std::vector<int> out;
    done[sink] = 1;
    while (!stack.empty()) {
      auto& top = stack.back();
      if (top.second < 3) {
        int j = co[top.first][top.second++];
        if (j >= 0 && !done[j]) {
          done[j] = 1;
          stack.push_back({j, 0});
        }
      } else {
        const int i = top.first;
        stack.pop_back();
        if (i != sink && nd[i].op != PMC_OP_UV_INPUT && !folded[i]) out.push_back(i);
      }
    }
    return out;
  }

  // Sethi-Ullman order is a heuristic on a DAG: shared values can stay live
  // across long stretches.  Variants of it that break ties between equally
  // needy inputs differently, or visit inputs in a scrambled order, are tried
  // too (a fixed number, with a fixed hash: the result is deterministic), and
  // the order whose allocation needs the fewest registers is emitted.
  bool allocate_registers() {
    const std::string err0 = err;
    bool ok = assign_registers();
    std::string best_err = err;
    std::vector<int> best_order = order, best_reg[2] = {reg[0], reg[1]};
    uint32_t best_regs = n_regs;
    if (ok && n_regs <= kRegsGoal) return true;
    for (uint32_t v = 1; v <= kOrderVariants; ++v) {
      std::vector<std::array<int, 3>> co = child_order;
      for (uint32_t i = 0; i < n; ++i) {
        auto& ch = co[i];
        int nc = 0;
        while (nc < 3 && ch[nc] >= 0) ++nc;
        auto key = [&](int j) { return mix32(v * 0x9E3779B9u ^ (uint32_t(i) << 12) ^ uint32_t(j)); };
        if (v & 1u)      // scrambled visiting order
          std::sort(ch.begin(), ch.begin() + nc, [&](int a, int b) { return key(a) < key(b); });
        else             // by need, ties scrambled
          std::sort(ch.begin(), ch.begin() + nc, [&](int a, int b) {
            return need[a] != need[b] ? need[a] > need[b] : key(a) < key(b);
          });
      }
      order = emission_order(co);
      for (size_t p = 0; p < order.size(); ++p) pos[order[p]] = int(p);
      n_regs = 0;
      const bool ok_v = assign_registers();
      if (ok_v && (!ok || n_regs < best_regs)) {
        ok = true;
        best_err = err0;
        best_order = order;
        best_reg[0] = reg[0];
        best_reg[1] = reg[1];
        best_regs = n_regs;
      }
      if (ok && best_regs <= kRegsGoal) break;
    }
    err = ok ? err0 : best_err;
    order = best_order;
    for (size_t p = 0; p < order.size(); ++p) pos[order[p]] = int(p);
    reg[0] = best_reg[0];
    reg[1] = best_reg[1];
    n_regs = best_regs;
    return ok;
  }

  bool assign_registers() {
    struct V { int node, sock, width, def, last; };
    std::vector<V> vals;
    int end = int(order.size());
    for (int i : order) {
      for (int s = 0; s < kNumOut[nd[i].op]; ++s) {
        if (!socket_used(i, s)) continue;
        int last = -1;
        for (auto& ck : consumers[i]) {
          if (int(nd[ck.first].in[ck.second].socket) != s) continue;
          last = std::max(last, ck.first == sink ? end : pos[ck.first]);
        }
        bool cachd = sock_ord[s][i] >= 0;
        // a cached value is written by its own instruction: it stays busy
        // there even when nothing reads it later
        if (cachd) last = std::max(last, pos[i] + 1);
        vals.push_back({i, s, width_of(out_type(nd[i].op, s)), cachd ? -1 : pos[i], last});
      }
    }
    std::stable_sort(vals.begin(), vals.end(), [](const V& a, const V& b) { return a.def < b.def; });
    std::vector<int> owner_last(kMaxRegs, -2);   // last use of the value holding each register
    reg[0].assign(n, -1);
    reg[1].assign(n, -1);
    for (const V& v : vals) {
      int base = -1;
      for (int r = 0; r + v.width <= kMaxRegs && base < 0; ++r) {
        bool ok = true;
        // a register whose value is last read by the defining instruction is
        // free for its result: the interpreter reads all operands of an
        // instruction before it writes any output
        for (int w = 0; w < v.width; ++w)
          if (owner_last[r + w] > v.def) { ok = false; break; }
        if (ok) base = r;
      }
      if (base < 0) {
        char buf[160];
        snprintf(buf, sizeof buf, "material %u: needs more than %d registers", mat, kMaxRegs);
        err = buf;
        return false;
      }
      for (int w = 0; w < v.width; ++w) owner_last[base + w] = v.last;
      reg[v.sock][v.node] = base;
      n_regs = std::max<uint32_t>(n_regs, uint32_t(base + v.width));
    }
    return true;
  }

  // operand for input k of node i; constants go to k[] at *kofs
  uint32_t operand(int i, int k, float* kbuf, int* kofs) {
    const pmc_input& in = nd[i].in[k];
    uint8_t want = in_type(nd[i].op, k);
    if (want == OT_UV) return make_operand(OPK_UV, 0, 0);
    if (want == OT_VECTOR && in.node < 0) return make_operand(OPK_NORMAL, 0, 0);
    if (in.node < 0 || folded[in.node]) {
      Val v = const_input(i, k);
      int w = want == OT_FLOAT ? 1 : 3;
      int o = *kofs;
      for (int c = 0; c < w; ++c) kbuf[o + c] = v.v[c];
      *kofs += w;
      return make_operand(w == 1 ? OPK_CONST_F : OPK_CONST_C, uint8_t(o), 0);
    }
    int s = int(in.socket);
    uint8_t have = out_type(nd[in.node].op, s);
    uint16_t r = uint16_t(reg[s][in.node]);
    uint8_t kind;
    if (have == want) kind = (want == OT_FLOAT) ? OPK_REG_F : OPK_REG_C;
    else if (have == OT_COLOR) kind = OPK_REG_C2F;
    else kind = OPK_REG_F2C;
    return make_operand(kind, 0, r);
  }

  void emit(Program& P, pmc_material_info& info) {
    MatHeader h{};
    h.instr_begin = uint32_t(P.instrs.size());
    h.n_instr = uint32_t(order.size());
    h.n_regs = n_regs;
    h.n_cach = uint32_t(cach.size());
    h.cach_begin = uint32_t(P.cach.size());
    for (int i : order) {
      const pmc_node_desc& d = nd[i];
      Instr I;
      std::memset(&I, 0, sizeof I);
      I.op = uint8_t(d.op);
      I.flags = uint8_t(d.flags & PMC_NODE_CLAMP);
      I.n_out = uint8_t(kNumOut[d.op]);
      I.exec = exec[i];
      for (int s = 0; s < 2; ++s) {
        I.dst[s] = kNoReg;
        I.cord[s] = kNoOrd;
        I.otype[s] = OT_FLOAT;
      }
      for (int s = 0; s < kNumOut[d.op]; ++s) {
        I.dst[s] = reg[s][i] >= 0 ? uint16_t(reg[s][i]) : kNoReg;
        I.cord[s] = sock_ord[s][i] >= 0 ? uint8_t(sock_ord[s][i]) : kNoOrd;
        I.otype[s] = out_type(d.op, s);
      }
      int kofs = 0;
      for (int k = 0; k < kNumIn[d.op]; ++k) I.src[k] = operand(i, k, I.k, &kofs);
      switch (d.op) {
        case PMC_OP_IMAGE_TEXTURE: I.param = d.variant;
          P.max_texture = std::max<int32_t>(P.max_texture, int32_t(d.variant)); break;
        case PMC_OP_VALUE_NOISE: case PMC_OP_PERLIN_NOISE: case PMC_OP_POSITION_NOISE:
          I.variant = uint8_t(d.octaves); I.param = d.seed; I.k[7] = d.freq;
          if (d.op == PMC_OP_POSITION_NOISE) P.uses_position = true;
          break;
        case PMC_OP_MATH: I.variant = uint8_t(d.variant); break;
        case PMC_OP_COLOR_RAMP:
          I.param = uint32_t(P.pool.size());
          for (int c = 0; c < 8; ++c) P.pool.push_back(d.ramp_pos[c]);
          for (int c = 0; c < 8; ++c)
            for (int q = 0; q < 4; ++q) P.pool.push_back(d.ramp_rgba[c][q]);
          break;
        default: break;
      }
      P.instrs.push_back(I);
    }
    // hit program: a lane whose lookups all hit runs only the always-needed nodes
    h.hit_begin = uint32_t(P.instrs.size());
    for (uint32_t q = h.instr_begin; q < h.instr_begin + h.n_instr; ++q) {
      Instr copy = P.instrs[q];
      if (copy.exec & kAlways) P.instrs.push_back(copy);
    }
    h.n_hit = uint32_t(P.instrs.size()) - h.hit_begin;
    int kofs = 0;
    for (int k = 0; k < 3; ++k) h.out_src[k] = operand(sink, k, h.out_k, &kofs);
    for (size_t c = 0; c < cach.size(); ++c) {
      CachDesc cd{};
      int i = cach[c].first, s = cach[c].second;
      cd.node_sock = (uint32_t(i) << 16) | (uint32_t(s) << 8);
      cd.reg = uint16_t(reg[s][i]);
      cd.otype = out_type(nd[i].op, s);
      cd.key = cls[i] == C_POS ? KEY_CELL : KEY_TEXEL;
      P.cach.push_back(cd);
    }
    P.headers.push_back(h);
    std::memset(&info, 0, sizeof info);
    info.n_nodes = n;
    for (uint32_t i = 0; i < n; ++i) {
      info.n_live += live[i];
      info.n_folded += folded[i];
    }
    info.n_instr = h.n_instr;
    info.n_regs = n_regs;
    info.n_cacheable = uint32_t(cach.size());
    for (size_t c = 0; c < cach.size(); ++c) {
      info.cacheable_node[c] = uint32_t(cach[c].first);
      info.cacheable_socket[c] = uint32_t(cach[c].second);
      info.subgraph_nodes[c] = uint32_t(cach_sub[c]);
      info.cacheable_type[c] = out_type(nd[cach[c].first].op, cach[c].second) == OT_COLOR ? 1u : 0u;
      info.cacheable_key[c] = cls[cach[c].first] == C_POS ? 1u : 0u;
    }
    P.max_regs = std::max(P.max_regs, n_regs);
    P.max_cach = std::max(P.max_cach, uint32_t(cach.size()));
  }
};

}  // namespace

pmc_status compile_program(const pmc_node_desc* nodes, const uint32_t* node_offsets,
                           uint32_t n_mats, const pmc_compile_opts* opts, Program& out,
                           std::string& err) {
  out = Program{};
  if (!nodes || !node_offsets || n_mats == 0) {
    err = "compile: null nodes/offsets or zero materials";
    return PMC_ERR_INVALID;
  }
  uint32_t min_nodes = (opts && opts->min_subgraph_nodes) ? opts->min_subgraph_nodes : 2;
  bool fold = !(opts && opts->no_fold);
  const bool world_keys = !(opts && opts->texel_keys_only);
  out.info.resize(n_mats);
  for (uint32_t m = 0; m < n_mats; ++m) {
    if (node_offsets[m + 1] < node_offsets[m]) {
      err = "compile: node_offsets not ascending";
      return PMC_ERR_INVALID;
    }
    MatCompiler mc(m, nodes + node_offsets[m], node_offsets[m + 1] - node_offsets[m], min_nodes,
                   fold, err);
    mc.world_keys = world_keys;
    if (!mc.validate()) return PMC_ERR_GRAPH;
    mc.analyse();
    mc.mark_cacheable();
    mc.need_masks();
    if (!mc.allocate_registers()) return PMC_ERR_GRAPH;
    mc.emit(out, out.info[m]);
  }
  out.lpt_order.resize(n_mats);
  for (uint32_t m = 0; m < n_mats; ++m) out.lpt_order[m] = m;
  std::stable_sort(out.lpt_order.begin(), out.lpt_order.end(), [&](uint32_t a, uint32_t b) {
    return out.headers[a].n_instr > out.headers[b].n_instr;
  });
  out.lpt_rank.resize(n_mats);
  for (uint32_t r = 0; r < n_mats; ++r) out.lpt_rank[out.lpt_order[r]] = r;
  return PMC_OK;
}

}  // namespace pmc
