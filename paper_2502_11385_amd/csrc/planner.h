// Host-side gate-fusion and tiling planner (pure C++, no device calls).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "program.h"

namespace qsv {

// A validated gate in normalised form.
struct HostGate {
  int k = 0, c = 0;
  int t[kMaxK] = {0};
  int ctl[kMaxQubits] = {0};
  std::vector<double> m;   // 2^k x 2^k complex, interleaved, row-major
  bool diagonal = false;   // off-diagonal entries are all exactly zero
  bool masked_phase = false;  // diagonal with every entry 1 except the last
  uint64_t tmask = 0, cmask = 0;
  // Commutation footprint: "dense" qubits are targets of a non-diagonal
  // gate; "touch" is every qubit the gate involves.  Two gates commute when
  // neither's dense set meets the other's touch set.
  uint64_t dense() const { return diagonal ? 0 : tmask; }
  uint64_t touch() const { return tmask | cmask; }
};

enum PassKind : int32_t { kPassPlain = 1, kPassTile = 2, kPassFused = 3 };

struct Pass {
  int32_t kind = kPassPlain;
  uint64_t qubits = 0;          // qubit set of the pass
  uint64_t alg_bytes = 0;       // algorithmic HBM bytes (read + write)
  std::vector<int> gates;       // gates applied, in application order
  // tile
  int32_t L = 0;
  int32_t q[16] = {0};
  struct Seg {
    int32_t reg_bits[6] = {0};
    std::vector<int> gates;
  };
  std::vector<Seg> segs;
  bool steer = false;           // order segments for ownership (see above)
  // fused
  int32_t fk = 0;
  int32_t fq[8] = {0};
};

struct PlanOptions {
  int strategy = 0;     // qsv_strategy
  int tile_log2 = 12;
  int k_max = 5;
  int low_qubits = 4;
  int reg_log2 = 4;
  // Spend planning time on fewer tile ops (each two-qubit diagonal gate
  // given to the side where it joins the most gates, segments built and
  // ordered for it).  Worth it where the plan's run time dwarfs the
  // planning: from 16 qubits, and for batches.
  bool steer = true;
};

struct Plan {
  std::vector<Pass> passes;
  uint64_t alg_bytes = 0;
  int tile_passes = 0, plain_passes = 0, fused_passes = 0, segments = 0;
};

// Fill defaults for zero fields and validate ranges; returns "" or an error.
std::string resolve_options(int n, int bytes_per_amp, const int* in5,
                            PlanOptions* out);

// Convert and validate the i-th gate of a flat gate list.
std::string make_gate(int n, int k, int c, const int32_t* qubits,
                      const double* matrix, HostGate* out);

// Build the pass list for gates on n qubits.
void make_plan(const std::vector<HostGate>& gates, int n, int bytes_per_amp,
               const PlanOptions& opt, Plan* plan);

// Counts of what emit_tile_pass produced (accumulated over calls).
struct TileEmitStats {
  uint64_t ops = 0;          // tile ops (phase-block data records excluded)
  uint64_t blocks = 0;       // kOpPhaseBlock ops
  uint64_t block_gates = 0;  // diagonal gates applied inside phase blocks
  // Real flops per state amplitude that the ops define: a 2x2 complex
  // matrix row (14: two complex products and a sum) per amplitude a dense
  // op changes, a complex product (6) per amplitude a diagonal op, a phase
  // op or a phase block multiplies.  Times 2^n it is the arithmetic of the
  // tile passes.
  double flops_per_amp = 0;
};

// Append the device records of one tile pass (its TilePass, segments and
// ops; segment and op indices are global into the output vectors; the
// pass's phase-block records follow its ops).

std::string emit_tile_pass(const Pass& p, const std::vector<HostGate>& G,
                           int reg_log2, std::vector<TilePass>* passes,
                           std::vector<TileSeg>* segs,
                           std::vector<TileOp>* ops,
                           TileEmitStats* stats = nullptr);

// Fill a finished tile op's dispatch code and argument (kernel header)
// from its kind, mux and controls; returns an error text or "".
std::string set_op_code(TileOp* op);

// Algorithmic bytes of applying gate g as a plain per-gate kernel.
uint64_t plain_gate_bytes(const HostGate& g, int n, int bytes_per_amp);

}  // namespace qsv
