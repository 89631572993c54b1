// Internal interface of the batch engine, shared with the request server.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "device_common.h"
#include "planner.h"
#include "program.h"
#include "qsv.h"

namespace qsv {

qsv_status set_error(qsv_status st, const std::string& msg);

// Host image of a batch program: variants, their tile passes, segments and
// ops, the ragged output layout and the scratch slot size.
struct HostProgram {
  std::vector<BatchCircuit> circs;
  std::vector<int32_t> order;
  std::vector<TilePass> passes;
  std::vector<TileSeg> segs;
  std::vector<TileOp> ops;
  std::vector<uint64_t> out_offsets;  // circs.size() + 1 entries
  uint64_t slot_amps = 0;
  uint64_t tiles = 0, amp_updates = 0, single_tile = 0;
};

// Plan one variant (validated gates G on w qubits, started in |0...0>) and
// append it to hp; *cost (may be null) receives its estimated work.
std::string append_variant(int w, const std::vector<HostGate>& G, int b,
                           int L, int RB, HostProgram* hp, double* cost);

// True when every gate can run inside batched tiles.
inline bool batchable(const std::vector<HostGate>& G) {
  for (const HostGate& g : G)
    if (!(g.diagonal ? (g.masked_phase || g.k <= 2) : g.k == 1)) return false;
  return true;
}

// Resident work-groups per CU of the batch kernel (0 if the query fails).
int batch_blocks_per_cu(int prec, int out_fp64, int rb, int L);

hipError_t launch_batch(int prec, int out_fp64, int rb, const BatchCircuit* circs,
                        const int32_t* order, int32_t count,
                        const TilePass* passes, const TileSeg* segs,
                        const TileOp* ops, void* out, void* scratch,
                        uint64_t slot_amps, int L, int grid,
                        hipStream_t stream);

}  // namespace qsv
