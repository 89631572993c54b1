// Device program records shared by the host planner and the HIP kernels.
//
// A planned circuit is uploaded once per qsv_apply_fused call as one device
// buffer holding these plain records; kernels read them with uniform loads.
#pragma once
#include <stdint.h>

namespace qsv {

constexpr int kMaxQubits = 34;
constexpr int kMaxK = 5;
constexpr int kMaxTileBits = 14;

// Tile op kinds.
enum : int32_t {
  kOpDense1 = 0,  // 2x2 matrix on one register bit, optional controls
  kOpDiag = 1,    // diagonal table on 1-2 qubits (local or outside the tile)
  kOpPhase = 2,   // multiply by m[0..1] where every bit of a mask is 1
  kOpPhaseBlock = 3  // a run of diagonal gates as one phase polynomial
};

// Dispatch classes of a tile op, precomputed by the planner (TileOp::code
// = class << 3 | register index of the target).  The kernel reads an op's
// header and both matrices in one batch of scalar loads and branches once.
//  kCodeUniform:   2x2 matrix mf (m) on register bit `reg`, or mf2 (m2)
//                  where bit `arg` of the tile's base index is 1 (an outer
//                  mux qubit; arg = 63, a bit no index has, when there is
//                  no mux).  The matrix is the same for the whole tile.
//  kCodeRegMux:    mf where register bit `arg` of the pair's index is 0,
//                  mf2 where it is 1 (fixed per register pair).
//  kCodeThreadMux: mf or mf2 by tile-local bit `arg`, which a thread bit
//                  holds (fixed per thread).
//  kCodeCtrl:      as kCodeUniform, applied only where every tile-local
//                  bit of lctrl is 1.
//  kCodeCtrlMux:   mf or mf2 by tile-local bit `arg`, applied only where
//                  every bit of lctrl is 1.
//  kCodePhase:     multiply by mf[0..1] (m[0..1]) where every tile-local
//                  bit of lctrl is 1.
//  kCodeDiag:      diagonal table on arg (1 or 2) targets, see dbit0/1.
//  kCodePhaseBlock: a PhaseBlock record `blob` bytes after the op.
enum : int32_t {
  kCodeUniform = 0,
  kCodeRegMux = 1,
  kCodeThreadMux = 2,
  kCodeCtrl = 3,
  kCodeCtrlMux = 4,
  kCodePhase = 5,
  kCodeDiag = 6,
  kCodePhaseBlock = 7
};

// One gate inside a tile segment.  The first 32 bytes and the FP32 (mf,
// mf2) or FP64 (m, m2) matrices are what the kernels read; the fields
// after them describe the op for the host (planner, host emulation).
//  kOpDense1: reg = index (0..RB-1) of the register bit holding the target;
//             m = 2x2 complex matrix, row-major interleaved (see mux below).
//  kOpDiag:   dk targets (1 or 2); dbit[j] >= 0 is the tile-local bit of
//             target j, dbit[j] < 0 means qubit (-1 - dbit[j]) outside the
//             tile (its value is fixed per tile); m holds the 2^dk diagonal
//             entries (re, im), entry index r = sum_j bit_j * 2^j.
//  kOpPhase:  a diagonal gate whose entries are all 1 except the last
//             (CZ, CP, S, T, P, multi-controlled phases): the amplitude is
//             multiplied by the phase m[0..1] when all its target and
//             control bits are 1; lctrl/gctrl then hold targets as well.
//  kOpPhaseBlock: a run of diagonal unitary gates applied as one factor
//             e^{i phi(x)}, phi a sum of terms; see PhaseBlock.  `blob` is
//             the byte offset from this op to its PhaseBlock record.
//  lctrl: controls inside the tile as a mask of tile-local bits.
//  gctrl: controls outside the tile as a mask of global qubits.
struct alignas(16) TileOp {
  // kernel header (32 bytes)
  int32_t code;   // class << 3 | reg (see kCode*)
  int32_t arg;    // mux bit or outer mux qubit; target count for kCodeDiag
  uint32_t lctrl;
  int32_t blob;   // kOpPhaseBlock only
  uint64_t gctrl;
  int32_t dbit0;
  int32_t dbit1;
  // matrices
  float mf[8];    // m rounded to FP32 (complex64 states)
  float mf2[8];
  double m[8];
  double m2[8];
  // host description
  int32_t kind;
  int32_t reg;
  // kOpDense1 only: the matrix may depend on one more qubit ("mux"):
  // kMuxNone, a tile-local bit (>= 0) or an outer qubit q as -1 - q.  The
  // op applies m where that bit is 0 and m2 where it is 1.
  int32_t mux;
  // kOpDense1 with a tile-local mux bit: the index of the register bit that
  // holds it in the op's segment, or -1 when a thread bit holds it (then the
  // matrix is fixed per thread).  -1 for every other op.
  int32_t mux_reg;
  int32_t dk;
  int32_t pad_[3];
};
static_assert(sizeof(TileOp) == 256, "tile ops are 256-byte records");

constexpr int32_t kMuxNone = -1000;

// Phase blocks.  A product of diagonal unitary gates is e^{i phi(x)} with
// phi(x) = sum over terms of angle * [every bit of the term's mask is 1 in
// x] (mod 2 pi): the multilinear expansion of each gate's phase function.
// Within a segment every term's mask splits into register bits, thread bits
// (tile-local, mask `tmask`) and outer qubits (global mask `gmask`); the
// planner keeps only terms with at most one register bit, plus terms made
// of register bits alone, which go into a 2^RB-entry table.  Angles are
// fixed-point fractions of a turn, so that sums wrap exactly modulo 2 pi.
constexpr int kMaxRegBits = 5;

struct alignas(16) PhaseTerm {
  uint64_t gmask;    // outer qubits that must be 1
  uint32_t tmask;    // thread bits (tile-local) that must be 1
  uint32_t turns32;  // turns rounded to 32 bits (complex64)
  uint64_t turns;    // angle / (2 pi) * 2^64, modulo 2^64
  uint64_t pad;
};

// Accumulator 0 holds the terms without a register bit; accumulator 1 + r
// the terms whose one register bit is register bit r of the segment.  The
// terms follow the record in accumulator order, each accumulator's terms
// with tmask == 0 (uniform over a tile) first.
struct alignas(16) PhaseBlock {
  int32_t n_uni[kMaxRegBits + 1];  // terms with tmask == 0
  int32_t n_thr[kMaxRegBits + 1];  // terms with tmask != 0
  int32_t has_table;               // table below differs from all ones
  int32_t n_terms;
  int32_t pad[2];
  // factor of register index j from terms on register bits only
  float tf[2 << kMaxRegBits];
  double td[2 << kMaxRegBits];
};

// A run of ops executed with one register layout: the tile-local bits in
// reg_bits[0..RB-1] (ascending) index each thread's registers; the other
// tile-local bits, in ascending order, index the threads.
struct alignas(16) TileSeg {
  int32_t reg_bits[6];
  int32_t op_begin;
  int32_t op_end;
};

// TilePass flags.
//  kPassLane32: the lane part of the I/O layout's byte offsets (the lowest
//               six thread bits spread over their tile qubits) fits 32
//               bits, so each access is a wave-uniform 64-bit address plus
//               one 32-bit per-lane offset.
//  kPassSpread: work-group g takes tile bitreverse(g) instead of tile g, so
//               that work-groups running at the same time touch far-apart
//               parts of the state.  Used for tiles made of many short runs
//               spaced by a large power of two, whose concurrent accesses
//               otherwise crowd a few DRAM channels.
constexpr int32_t kPassLane32 = 1;
constexpr int32_t kPassSpread = 2;
//  kPassOutputs: the pass also reduces its final amplitudes (an OutSpec
//               `out_spec` bytes after the TilePass record).
constexpr int32_t kPassOutputs = 4;

// Outputs folded into a circuit's last tile pass.  After its amplitudes are
// stored, each tile writes p = |a|^2 (optional) and, for up to two keys, the
// FP64 sums of p over the groups of its amplitudes that share the tile bits
// of the key: group g of tile x gathers the tile indices t with
// pext(t, key_mask) = g, and its sum goes to part[x * 2^key_bits + g].
// Within a tile the sum runs in a fixed order (16 consecutive group members
// per thread, then a pairwise tree over threads), so the partial sums, and
// the fixed-order reductions over tiles that follow, are reproducible.
// The kernel stages p in LDS in group-major order, tile index t at
// position (pext(t, key_mask) << (L - key_bits)) | pext(t, ~key_mask); a
// position is the sum of one term per set bit of t, given here per thread
// bit (tile bits 0..W-1 of the I/O layout) and per register index (tile
// bits W..L-1).  The host requires key_bits <= L - RB, so that each
// thread's 2^RB consecutive positions belong to one group.
struct alignas(16) OutSpec {
  uint64_t probs;       // device address of the 2^n probabilities, 0: none
  int32_t probs_fp64;   // 1: double, 0: float
  int32_t n_keys;       // 0..2
  uint64_t part[2];     // device addresses of each key's partial sums
  int32_t key_bits[2];  // popcount of each key's tile-local mask
  int32_t pad_[2];
  uint32_t thr_pos[2][10];
  uint32_t reg_pos[2][32];
};

// One tile pass: 2^L amplitudes per tile, tile-local bit b is global qubit
// q[b] (ascending).  Tiles are the cosets of the other n - L qubits.
struct alignas(16) TilePass {
  int32_t L;
  int32_t nseg;
  int32_t seg_begin;
  int32_t flags;  // kPassLane32 | kPassSpread | kPassOutputs
  int32_t q[16];
  int32_t out_spec;  // kPassOutputs: byte offset from this record
  int32_t pad_[3];
};

// One gate of a fused block, in the block's local qubit numbering
// (block qubit j = j-th smallest qubit of the block).
struct alignas(16) FusedGate {
  int32_t k;          // targets (1..5)
  int32_t c;          // controls
  int32_t t[5];
  int32_t ctl[5];
  int64_t m_offset;   // offset (in doubles) of the 2^k x 2^k matrix
};

// One fused block: apply the product of its gates, a 2^k x 2^k unitary on
// block qubits q[0..k-1].
struct alignas(16) FusedBlock {
  int32_t k;
  int32_t n_gates;
  int32_t gate_begin;
  int32_t pad;
  int64_t u64_offset;  // FP64 product, 2^k x 2^k complex (in doubles)
  int64_t u32_offset;  // the same rounded once to FP32 (in floats)
  int32_t q[8];
  uint64_t cmask;      // control qubits (all must be 1); 0 for products
};

// One variant of a batch: its width, its tile passes (all its gates run in
// tile passes) and where its 2^w probabilities go in the ragged output.
struct alignas(16) BatchCircuit {
  int32_t w;
  int32_t n_passes;
  int32_t pass_begin;
  int32_t pad;
  uint64_t out_offset;
  uint64_t state_offset;  // its state in the batch's state buffer (variants
                          // of more than one pass)
};

// Phase p of a batch runs pass p of every variant that has one; its tiles
// are listed as runs, one per variant: entry k covers the phase's tiles
// tile_begin(k) .. tile_begin(k+1) - 1, which are the tiles of that pass.
// Work-groups take equal shares of the phase's summed tile cost.
struct alignas(16) BatchWork {
  int32_t circ;
  uint32_t tile_cost;    // estimated cost of one of its tiles
  uint64_t tile_begin;
  uint64_t cost_begin;   // summed cost of the phase's tiles before it
  uint64_t pad;
};

}  // namespace qsv
