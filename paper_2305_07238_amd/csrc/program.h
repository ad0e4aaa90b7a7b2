// program.h - compiled form of a material graph set (host compiler -> device interpreter).
//
// Sec. 2 of the paper evaluates material networks as a stack machine: nodes
// are turned into data that the GPU reads and executes in storage order.
// Here each live node becomes one 64-byte instruction, read wave-uniformly
// (scalar loads) because every wave shades hits of a single material.  Node
// outputs live in a per-lane register file in LDS, laid out [reg][lane] so a
// wave's access to one register is 64 consecutive dwords (no bank conflicts).
#pragma once
#include <cstdint>

namespace pmc {

constexpr int kMaxCach = 8;            // cacheable outputs per material
constexpr uint32_t kAlways = 1u << 31; // need-mask bit: needed whatever the lookups gave
constexpr uint16_t kNoReg = 0xFFFF;
constexpr uint8_t kNoOrd = 0xFF;
constexpr int kMaxRegs = 240;          // per-lane float registers (LDS budget)

// Operand kinds.  Conversions between FLOAT and COLOR are resolved at compile time.
enum : uint8_t {
  OPK_NONE = 0,
  OPK_CONST_F = 1,   // k[kofs]
  OPK_CONST_C = 2,   // k[kofs .. kofs+2]
  OPK_REG_F = 3,     // reg
  OPK_REG_C = 4,     // reg .. reg+2 (COLOR or VECTOR)
  OPK_REG_C2F = 5,   // (reg + reg+1 + reg+2) / 3
  OPK_REG_F2C = 6,   // (reg, reg, reg)
  OPK_UV = 7,        // the hit's UV
  OPK_NORMAL = 8     // the hit's normal
};

inline uint32_t make_operand(uint8_t kind, uint8_t kofs, uint16_t reg) {
  return uint32_t(kind) | (uint32_t(kofs) << 8) | (uint32_t(reg) << 16);
}
inline uint8_t operand_kind(uint32_t o) { return uint8_t(o & 0xFF); }
inline uint8_t operand_kofs(uint32_t o) { return uint8_t((o >> 8) & 0xFF); }
inline uint16_t operand_reg(uint32_t o) { return uint16_t(o >> 16); }

enum : uint8_t { OT_FLOAT = 0, OT_COLOR = 1, OT_VECTOR = 2, OT_UV = 3 };

struct Instr {              // 64 bytes, one per emitted node
  uint8_t op;               // pmc_op
  uint8_t variant;          // MATH op; noise octave count
  uint8_t flags;            // PMC_NODE_CLAMP
  uint8_t n_out;            // output sockets
  uint16_t dst[2];          // register base of each output socket, kNoReg if unused
  uint8_t cord[2];          // cacheable ordinal of each socket, kNoOrd if none
  uint8_t otype[2];         // OT_* of each socket
  uint32_t exec;            // need mask: kAlways | bit c for each cacheable ordinal c
  uint32_t src[3];          // operand descriptors
  uint32_t param;           // IMAGE: texture index; noise: seed; RAMP: offset into the float pool
  float k[8];               // constants of unconnected / folded inputs; noise: k[7] = f0
};
static_assert(sizeof(Instr) == 64, "Instr layout");

struct MatHeader {          // 128 bytes
  uint32_t instr_begin;     // full program: every live node
  uint32_t n_instr;
  uint32_t n_regs;
  uint32_t n_cach;
  uint32_t cach_begin;
  uint32_t out_src[3];      // operands of base colour, roughness, normal
  float out_k[8];           // their constants: base k[0..2], roughness k[3]
  uint32_t hit_begin;       // hit program: only the nodes needed when every lookup hit
  uint32_t n_hit;           // (the instructions whose need mask has kAlways)
  uint32_t surr_slot;       // surrogate network of the material (valid when surr_mask != 0)
  uint32_t surr_mask;       // cacheable ordinals the network can stand in for
  uint32_t surr_chan;       // first network channel of each ordinal, 4 bits per ordinal
  uint32_t pad[11];
};
static_assert(sizeof(MatHeader) == 128, "MatHeader layout");

enum : uint8_t { KEY_TEXEL = 0, KEY_CELL = 1 };   // UV texel, or world-space cell

struct CachDesc {           // 16 bytes, one per cacheable output
  uint32_t node_sock;       // node << 16 | socket << 8 (low byte: level)
  uint16_t reg;             // register that holds the value
  uint8_t otype;            // OT_FLOAT (raw float code) or OT_COLOR (RGB9E5)
  uint8_t key;              // KEY_TEXEL or KEY_CELL
  uint32_t pad2[2];
};
static_assert(sizeof(CachDesc) == 16, "CachDesc layout");

struct TexDesc {            // 16 bytes
  uint64_t offset;          // texel offset into the texel pool
  uint32_t w, h;
};

}  // namespace pmc
