// Device helpers shared by the HIP kernels (complex arithmetic, bit
// insertion) and the launcher declarations used by the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "planner.h"
#include "program.h"

namespace qsv {

// The device program (passes, segments, ops, phase-block records) is read
// through the constant address space.  The kernels never write it, and
// uniform reads through such pointers are scalar loads even in loops that
// also hold asm statements with memory clobbers (the LDS barriers and the
// streaming kernel's DMA), where the compiler could no longer prove the
// records unchanged and would read them with vector loads.
template <typename R>
using cptr = const __attribute__((address_space(4))) R*;
template <typename R>
__device__ __forceinline__ cptr<R> as_const(const R* p) {
  return (cptr<R>)(p);
}
// 16 bytes of such a record as a plain vector (no constructors, so it loads
// through a constant-address-space pointer on both compilation passes)
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct CxT;
template <>
struct CxT<float> {
  using type = float2;
};
template <>
struct CxT<double> {
  using type = double2;
};

// Fused multiply-add of the component type.
__device__ __forceinline__ float fmac(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fmac(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// Complex products with their fused multiply-adds written out, so that
// every kernel rounds them the same way (left to the compiler, contraction
// can differ between kernels that inline the same code).
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = fmac(a.x, b.x, -(a.y * b.y));
  r.y = fmac(a.x, b.y, a.y * b.x);
  return r;
}

// a*x + b*y for complex a, b, x, y
template <typename C>
__device__ __forceinline__ C cmul2(C a, C x, C b, C y) {
  C r;
  r.x = fmac(b.y, -y.y, fmac(b.x, y.x, fmac(a.x, x.x, -(a.y * x.y))));
  r.y = fmac(b.y, y.x, fmac(b.x, y.y, fmac(a.x, x.y, a.y * x.x)));
  return r;
}

// Component-wise select.  A conditional operator on the HIP vector structs
// selects between their addresses, which keeps register arrays in memory.
template <typename C>
__device__ __forceinline__ C csel(bool c, C a, C b) {
  C r;
  r.x = c ? a.x : b.x;
  r.y = c ? a.y : b.y;
  return r;
}

// Insert a zero bit at position p (bits >= p move up by one).
__device__ __forceinline__ uint64_t insert_zero64(uint64_t x, int p) {
  const uint64_t lo = x & ((uint64_t(1) << p) - 1);
  return ((x >> p) << (p + 1)) | lo;
}
__device__ __forceinline__ uint32_t insert_zero32(uint32_t x, int p) {
  const uint32_t lo = x & ((uint32_t(1) << p) - 1);
  return ((x >> p) << (p + 1)) | lo;
}

inline unsigned grid_blocks(uint64_t items, unsigned threads,
                            unsigned cap = 1u << 20) {
  uint64_t b = (items + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

// ------------------------------------------------------------ launchers
// All launchers enqueue on `stream` and return hipGetLastError().
// prec: 1 = complex64 (float2), 2 = complex128 (double2).

hipError_t launch_fill_basis(int prec, void* amp, int n, uint64_t index,
                             hipStream_t stream);
// Plain dense gate; dev_matrix (2^k x 2^k, FP64) is required for k >= 3.
hipError_t launch_dense(int prec, void* amp, int n, const HostGate& g,
                        const double* dev_matrix, hipStream_t stream);
// Plain diagonal gate (any k, controls).
hipError_t launch_diag(int prec, void* amp, int n, const HostGate& g,
                       hipStream_t stream);
// One tile pass: pass/segs/ops point into the device program buffer,
// host_pass is the host copy of *pass; rb is the register bits.
hipError_t launch_tile(int prec, int rb, void* amp, int n,
                       const TilePass& host_pass, const TilePass* pass,
                       const TileSeg* segs, const TileOp* ops,
                       hipStream_t stream);
// Build all fused unitaries (FP64, then rounded to FP32).
hipError_t launch_fused_build(const FusedBlock* blocks, int n_blocks,
                              const FusedGate* gates, double* mats64,
                              float* mats32, hipStream_t stream);
// Apply one fused block of width k on qubits q (host copy) with the device
// matrix u (FP64 for c128, FP32 for c64), where every qubit of cmask is 1
// (k >= 4 when cmask is not 0).
hipError_t launch_fused_apply(int prec, void* amp, int n, int k,
                              const int32_t* q, const void* u,
                              uint64_t cmask, hipStream_t stream);

// Reductions.  Scratch sizes are given by the *_scratch helpers (bytes).
size_t norm_scratch_bytes(int n);
// Fixed scratch of the allocation-free entry points: its size, and its
// device address on `device`, which must be the current device (looked up
// once per device).
constexpr int kMaxDevices = 64;
size_t fixed_scratch_bytes();
hipError_t fixed_scratch(int device, void** out);
hipError_t launch_probs(int prec, const void* amp, int n, void* out,
                        int out_fp64, double* scratch, double* norm_dev,
                        hipStream_t stream);
hipError_t launch_scale(int prec, void* amp, int n, const double* norm_dev,
                        hipStream_t stream);
size_t marginal_scratch_bytes(int n, int m);
hipError_t launch_marginal(int prec, const void* amp, int n,
                           const int32_t* qubits, int m, double* scratch,
                           double* out_dev, hipStream_t stream);
size_t sample_scratch_bytes(int n, uint64_t shots);
// top-k and Pauli expectations (k_outputs.hip)
hipError_t launch_topk_hist(int prec, const void* amp, uint64_t count,
                            uint64_t mask, uint64_t prefix, int shift,
                            int bins, unsigned long long* hist,
                            hipStream_t stream);
hipError_t launch_topk_collect(int prec, const void* amp, uint64_t count,
                               uint64_t mask, uint64_t prefix, int ge,
                               unsigned long long* counter, uint64_t cap,
                               uint64_t* out_key, uint64_t* out_idx,
                               hipStream_t stream);
hipError_t launch_topk_ties(int prec, const void* amp, uint64_t count,
                            uint64_t key, unsigned blocks, uint64_t chunk,
                            unsigned long long* counts,
                            const unsigned long long* offsets, uint64_t need,
                            uint64_t* out_idx, hipStream_t stream);
// qubit relabelling (k_permute.hip): tile source bits s_bits (ascending,
// s of them), their destinations d_bits (ascending), destination tile bit j
// taken from source tile bit src_of[j], and the outer source bits with their
// destinations
struct PermArgs {
  int32_t s;
  int32_t n_outer;
  int32_t m;  // lowest qubits kept contiguous (the LDS slot fold width)
  int32_t ne; // steps of blockDim.x amplitudes per tile
  // per step e (r = e * blockDim.x + tid): the uniform parts of the source
  // spread, the destination spread and the destination-to-source map
  uint64_t se[16];
  uint64_t de[16];
  uint32_t ge[16];
  int32_t s_bits[10];
  int32_t d_bits[10];
  int32_t src_of[10];
  int32_t outer_src[34];
  int32_t outer_dst[34];
};
hipError_t launch_permute(int prec, const void* src, void* dst, int n,
                          const PermArgs& p, hipStream_t stream);
size_t pauli_scratch_bytes(int n);
hipError_t launch_pauli(int prec, const void* amp, int n, uint64_t xm,
                        uint64_t zm, double* scratch, double* out_dev,
                        hipStream_t stream);
hipError_t launch_sample(int prec, const void* amp, int n, uint64_t shots,
                         uint64_t seed, void* scratch, uint64_t* out_dev,
                         hipStream_t stream);
// The same draws when the scratch already holds the 2^(n-10) block sums
// (n > 10): the scan and the per-shot search only.
hipError_t launch_sample_from_blocks(int prec, const void* amp, int n,
                                     uint64_t shots, uint64_t seed,
                                     void* scratch, uint64_t* out_dev,
                                     hipStream_t stream);

// Reductions over the per-tile partial sums of a last tile pass with
// outputs (k_stream.hip).  Marginal bin j (output bit l = qubit qubits[l]):
// gpos[l] >= 0 is its bit in the group index (a tile qubit), else tpos[l]
// its bit in the tile index; the tile index bits of the other outer qubits
// (free_pos, ascending) are enumerated, n_enum = 2^free_bits values.
struct MargTileArgs {
  int32_t m;
  int32_t kb;
  int32_t free_bits;
  int32_t pad;
  uint64_t n_enum;
  int32_t gpos[20];
  int32_t tpos[20];
  int32_t free_pos[34];
};
hipError_t launch_marg_tiles(const double* part, const MargTileArgs& args,
                             double* out_dev, hipStream_t stream);
// Sampler block b (global bits 10..n-1, nhi = n - 10 of them): bit i of b is
// qubit 10 + i, in the group index at hi_g[i] >= 0 (a tile qubit) or the
// tile index at hi_t[i]; the outer qubits below 10 (free_pos, tile index
// bits, ascending) are enumerated.
struct BlockTileArgs {
  uint64_t nblocks;
  int32_t kb;
  int32_t nhi;
  int32_t free_bits;
  int32_t pad;
  int32_t hi_g[34];
  int32_t hi_t[34];
  int32_t free_pos[10];
};
hipError_t launch_blocks_tiles(const double* part, const BlockTileArgs& args,
                               double* P, hipStream_t stream);
// The same draws from a stored probability vector (float or double).
hipError_t launch_sample_probs(int fp64, const void* probs, int n,
                               uint64_t shots, uint64_t seed, void* scratch,
                               uint64_t* out_dev, hipStream_t stream);

}  // namespace qsv
