// Records shared by the cut-reconstruction host code and its kernels.
#pragma once
#include <stdint.h>

namespace qsv {

constexpr int kCutMaxSub = 16;
constexpr int kCutMaxCuts = 8;
constexpr int kCutMaxWidth = 24;
constexpr int kCutMaxEnds = 6;
constexpr int kCutMaxQubits = 30;
constexpr int kCutMaxVary = 4;  // wave kernel: subcircuits varying in a wave

// One subcircuit, as the kernels see it.
//  out_pos[i]  : local qubit of the subcircuit's i-th output (ascending);
//                bit i of an output index y is that qubit's value
//  out_uncut[i]: the uncut qubit measured there
//  end_kind[e] : 0 = downstream end (initialised), 1 = upstream end
//                (measured), for its e-th cut end in variant-digit order
//  end_pos[e]  : local qubit of the end
//  end_mult[e] : multiplier of the end's digit in the variant index
// The term vectors T[t][y] (t over 4^n_ends term choices, two bits per end,
// end 0 lowest; y over 2^eff outputs) start at element t_offset of T, and
// the subcircuit's variant offsets at element v_offset of the offset table.
struct alignas(16) CutSubDev {
  int32_t width;
  int32_t eff;
  int32_t n_ends;
  int32_t pad;
  int32_t out_pos[kCutMaxWidth];
  int32_t out_uncut[kCutMaxWidth];
  int32_t end_kind[kCutMaxEnds];
  int32_t end_pos[kCutMaxEnds];
  int32_t end_mult[kCutMaxEnds];
  // the outputs as runs of consecutive uncut qubits: output bits
  // run_dst[r] .. run_dst[r] + run_len[r] - 1 are uncut qubits
  // run_src[r] .. run_src[r] + run_len[r] - 1
  int32_t n_runs;
  int32_t pad2;
  int32_t run_src[kCutMaxWidth];
  int32_t run_dst[kCutMaxWidth];
  int32_t run_len[kCutMaxWidth];
  uint64_t t_offset;
  uint64_t v_offset;
  uint64_t entry_begin;  // first global term-vector entry of this subcircuit
  uint64_t n_entries;    // 4^n_ends * 2^eff
};

struct CutArgs {
  int32_t n_sub;
  int32_t n_cuts;
  int32_t n_qubits;
  int32_t probs_fp64;
  uint64_t n_terms;       // 4^n_cuts
  uint64_t total_entries; // sum of n_entries
  const CutSubDev* subs;
  const uint64_t* voff;   // element offsets of the variant vectors
  const uint64_t* tt;     // [n_terms][n_sub]: start of the chosen term
                          // vector of each subcircuit (simple kernel)
  // Wave kernel.  Subcircuits are split into "varying" ones (an output
  // among uncut qubits 0..5, which change across a wave's 64 lanes) and
  // "uniform" ones; c indexes the term digits of the cuts that touch a
  // varying subcircuit (n_c values), u those of the other cuts (n_u).
  const uint64_t* ttv;    // [n_c][n_vary]: term-vector start, varying subs
  const uint64_t* ttu;    // [n_c][n_u][n_uni]: the same, uniform subs
  int32_t vary_sub[kCutMaxSub];
  int32_t uni_sub[kCutMaxSub];
  int32_t n_vary;
  int32_t n_uni;
  uint64_t n_c;
  uint64_t n_u;
  double* T;
  const void* probs;
};

}  // namespace qsv
