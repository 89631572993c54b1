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
  uint64_t tiles = 0, amp_updates = 0, single_tile = 0;
  // filled by finalize_program: phase runs, and the state buffer layout
  std::vector<BatchWork> work;
  std::vector<uint64_t> phase_work_begin;  // phases + 1 entries
  std::vector<uint64_t> phase_tiles;       // tiles per phase
  std::vector<uint64_t> phase_cost;        // summed tile cost per phase
  uint64_t state_amps = 0;
};

// Lay out the states of multi-pass variants and list each phase's tile
// runs (variants in hp->order, or in index order when it is empty).
void finalize_program(HostProgram* hp);

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

// Launch every phase of a finalized batch program on `stream`: phase p
// runs on min(grid, phase_tiles[p]) work-groups.  `states` holds
// hp.state_amps amplitudes; `work` is hp.work on the device.
hipError_t launch_batch(int prec, int out_fp64, int rb,
                        const BatchCircuit* circs, const TilePass* passes,
                        const TileSeg* segs, const TileOp* ops,
                        const BatchWork* work, const HostProgram& hp,
                        void* out, void* states, int L, int grid,
                        hipStream_t stream);

}  // namespace qsv
