// compiler.h - material graph set -> interpreter program (host only).
#pragma once
#include <string>
#include <vector>

#include "../../include/pmc.h"
#include "program.h"

namespace pmc {

struct Program {
  std::vector<MatHeader> headers;       // one per material
  std::vector<Instr> instrs;
  std::vector<CachDesc> cach;
  std::vector<float> pool;              // COLOR_RAMP stops (8 positions + 8 RGBA each)
  std::vector<uint32_t> lpt_order;      // materials by decreasing program length
  std::vector<uint32_t> lpt_rank;       // inverse: rank of each material in lpt_order
  std::vector<pmc_material_info> info;
  uint32_t max_regs = 0;
  uint32_t max_cach = 0;
  int32_t max_texture = -1;             // highest texture index referenced
  bool uses_position = false;           // some live node reads the world position
};

// Compile every material.  On failure returns PMC_ERR_GRAPH (or INVALID) and sets err.
pmc_status compile_program(const pmc_node_desc* nodes, const uint32_t* node_offsets,
                           uint32_t n_mats, const pmc_compile_opts* opts, Program& out,
                           std::string& err);

}  // namespace pmc
