// Outputs folded into a circuit's last tile pass: the reductions over tiles.
//
// The last tile pass leaves, per tile x and key k, the FP64 sums of p over
// the groups of the tile's amplitudes that share the key's tile bits
// (OutSpec in program.h).  These kernels combine them into the marginal of
// specified qubits (the Builder's distribution of specified qubits,
// Section IV.A) and into the 1024-amplitude block sums that inverse-CDF
// sampling needs (shots, Section III.A), each output summed over its tiles
// in increasing tile index with Neumaier compensation: a fixed order, so a
// given state always gives the same bits, without one more read of the
// state per output.
#include "reduce_core.h"

namespace qsv {

// Bin j of the marginal: its bits on tile qubits form the group index g, its
// bits on outer qubits fix those bits of the tile index; the remaining tile
// index bits (free_mask) are enumerated in increasing order.  One wave per
// bin; lane l takes enumeration indices l, l + 64, ...; the 64 lane sums
// meet in a fixed shuffle tree.
__global__ void __launch_bounds__(256)
    marg_tiles_kernel(const double* __restrict__ part, MargTileArgs args,
                      double* __restrict__ out) {
  const uint64_t j = uint64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= (uint64_t(1) << args.m)) return;  // whole waves exit together
  uint64_t g = 0, pat = 0;
  for (int l = 0; l < args.m; ++l) {
    if (!(j >> l & 1)) continue;
    if (args.gpos[l] >= 0) g |= uint64_t(1) << args.gpos[l];
    else pat |= uint64_t(1) << args.tpos[l];
  }
  double s = 0, c = 0;
  for (uint64_t e = lane; e < args.n_enum; e += 64) {
    // tix = pat | pdep(e, free_mask)
    uint64_t tix = pat, rest = e;
    for (int b = 0; b < args.free_bits; ++b) {
      if (rest & 1) tix |= uint64_t(1) << args.free_pos[b];
      rest >>= 1;
    }
    nadd(s, c, part[(tix << args.kb) + g]);
  }
  for (int d = 32; d > 0; d >>= 1) {
    const double s2 = __shfl_down(s, d, 64);
    const double c2 = __shfl_down(c, d, 64);
    if (lane < d) {
      nadd(s, c, s2);
      c += c2;
    }
  }
  if (lane == 0) out[j] = s + c;
}

// Block b (global index bits 10 and up) of the sampler: its bits on tile
// qubits form the group index, its bits on outer qubits fix those bits of
// the tile index, and the outer qubits below 10 are enumerated in
// increasing order.  One thread per block.
__global__ void __launch_bounds__(256)
    blocks_tiles_kernel(const double* __restrict__ part, BlockTileArgs args,
                        double* __restrict__ P) {
  const uint64_t b = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= args.nblocks) return;
  uint64_t g = 0, pat = 0;
  for (int i = 0; i < args.nhi; ++i) {
    if (!(b >> i & 1)) continue;
    if (args.hi_g[i] >= 0) g |= uint64_t(1) << args.hi_g[i];
    else pat |= uint64_t(1) << args.hi_t[i];
  }
  double s = 0, c = 0;
  const uint64_t n_enum = uint64_t(1) << args.free_bits;
  for (uint64_t e = 0; e < n_enum; ++e) {
    uint64_t tix = pat;
    for (int k = 0; k < args.free_bits; ++k)
      if (e >> k & 1) tix |= uint64_t(1) << args.free_pos[k];
    nadd(s, c, part[(tix << args.kb) + g]);
  }
  P[b] = s + c;
}

hipError_t launch_marg_tiles(const double* part, const MargTileArgs& args,
                             double* out_dev, hipStream_t stream) {
  const uint64_t bins = uint64_t(1) << args.m;
  marg_tiles_kernel<<<unsigned((bins + 3) / 4), 256, 0, stream>>>(part, args,
                                                                  out_dev);
  return hipGetLastError();
}

hipError_t launch_blocks_tiles(const double* part, const BlockTileArgs& args,
                               double* P, hipStream_t stream) {
  blocks_tiles_kernel<<<unsigned((args.nblocks + 255) / 256), 256, 0,
                        stream>>>(part, args, P);
  return hipGetLastError();
}

}  // namespace qsv
