// LDS-staged tile kernel: one HBM read and one HBM write of the state apply
// a whole run of gates.
//
// A pass chooses L tile qubits q[0] < ... < q[L-1] (always including the
// lowest qubits, so each tile is a set of contiguous 2^m-amplitude runs in
// HBM).  Work-group b owns the coset of the other n - L qubits given by b and
// holds its 2^L amplitudes in registers: 2^RB per thread.  A segment fixes
// which RB tile-local bits select a thread's register (the "register bits");
// every dense gate of the segment targets a register bit, so a 2x2 update
// never leaves the thread.  Between segments the tile is re-distributed
// through LDS.  Diagonal gates and controls need no register bit: their
// effect depends only on the amplitude's index (tile-local bits, plus the
// tile's fixed outer bits), which each thread knows.
//
// This is the single-GPU form of the paper's chunking with cache blocking
// (Section III.B): a tile is a 2^L-amplitude chunk, and a pass runs every
// gate that the planner could move onto the chunk's qubits.
#include <algorithm>
#include <mutex>

#include "reduce_core.h"
#include "tile_core.h"

namespace qsv {

// Tile kernels whose re-layouts go in halves (one component per amplitude
// through LDS): complex64 with 16 registers per thread, and complex128.
template <typename T, int RB>
constexpr bool kHalves = (sizeof(T) == 4 && RB == 4) || sizeof(T) == 8;

// Tile index -> global index of the tile's first amplitude: the index's
// bits spread over the non-tile qubits.
__device__ __forceinline__ uint64_t tile_base(const TilePass* pass,
                                              uint32_t tile) {
  const cptr<TilePass> cp = as_const(pass);
  uint64_t base = tile;
  const int L = cp->L;
  for (int b = 0; b < L; ++b) base = insert_zero64(base, cp->q[b]);
  return base;
}

// Outputs of the last tile pass (kPassOutputs): p = |a|^2 of the tile's
// final amplitudes (in the I/O layout, register j of thread tid is tile
// index tid | j << W), stored if requested, then for each key the FP64 sum
// over each group of the tile, in a fixed order: p staged in LDS in
// group-major order, each thread sums its 2^RB consecutive entries (all in
// one group), a pairwise tree combines the threads of each group.
// e_base: element index of register 0 of this lane; e_reg[j]: element
// offset of register j.
template <typename T, int RB>
__device__ __forceinline__ void tile_outputs(
    const typename CxT<T>::type* a, typename CxT<T>::type* lds,
    const TilePass* pass, uint32_t tix, uint64_t e_base, const uint64_t* e_reg,
    uint32_t tid) {
  constexpr int R = 1 << RB;
  const cptr<TilePass> cp = as_const(pass);
  const OutSpec* osg = reinterpret_cast<const OutSpec*>(
      reinterpret_cast<const char*>(pass) + cp->out_spec);
  const cptr<OutSpec> os = as_const(osg);
  const int L = cp->L;
  const int W = L - RB;
  double p[R];
#pragma unroll
  for (int j = 0; j < R; ++j) p[j] = prob_of(a[j]);
  const uint64_t probs = os->probs;
  if (probs) {
    if (os->probs_fp64) {
      double* pd = reinterpret_cast<double*>(probs);
#pragma unroll
      for (int j = 0; j < R; ++j) pd[e_base + e_reg[j]] = p[j];
    } else {
      float* pf = reinterpret_cast<float*>(probs);
#pragma unroll
      for (int j = 0; j < R; ++j) pf[e_base + e_reg[j]] = float(p[j]);
    }
  }
  double* sh = reinterpret_cast<double*>(lds);
  const int n_keys = os->n_keys;
  for (int k = 0; k < n_keys; ++k) {
    const int kb = os->key_bits[k];
    uint32_t tpos = 0;
    for (int b = 0; b < W; ++b)
      if (tid >> b & 1) tpos += os->thr_pos[k][b];
    lds_barrier();  // every earlier use of the LDS is over
#pragma unroll
    for (int j = 0; j < R; ++j) sh[tpos + os->reg_pos[k][j]] = p[j];
    lds_barrier();
    double sum = 0;
#pragma unroll
    for (int e = 0; e < R; ++e) sum += sh[tid * R + e];
    lds_barrier();
    sh[tid] = sum;
    const int tg = L - kb - RB;  // log2 of the threads per group
    for (int st = 0; st < tg; ++st) {
      lds_barrier();
      if ((tid & ((2u << st) - 1)) == 0) sh[tid] += sh[tid + (1u << st)];
    }
    lds_barrier();
    if ((tid & ((1u << tg) - 1)) == 0) {
      double* part = reinterpret_cast<double*>(os->part[k]);
      part[(uint64_t(tix) << kb) + (tid >> tg)] = sh[tid];
    }
  }
}

// One tile per work-group (at most 512 threads, L - RB <= 9).  HBM
// transfers use the I/O layout: registers select the top RB tile bits and
// consecutive threads take consecutive low tile bits, so a wave's accesses
// are contiguous runs of the lowest (always tile) qubits.  A thread's
// element index is base | lane part | wave part | register part, four
// disjoint bit sets: the lane part (thread bits 0..5 spread over their tile
// qubits) differs per lane, the others are uniform over a wave.  Each access
// is therefore one wave-uniform 64-bit address plus a per-lane offset,
// 32-bit where LANE32 says it fits (else 64-bit).
template <typename T, int RB, bool LANE32>
__device__ __forceinline__ void tile_body(typename CxT<T>::type* __restrict__ amp,
                                          const TilePass* __restrict__ pass,
                                          const TileSeg* __restrict__ segs,
                                          const TileOp* __restrict__ ops) {
  using C = typename CxT<T>::type;
  using Off = std::conditional_t<LANE32, uint32_t, uint64_t>;
  constexpr int R = 1 << RB;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  uint32_t tix = blockIdx.x;
  if (pass->flags & kPassSpread) {
    const uint32_t tb = 31u - __builtin_clz(gridDim.x);  // log2(#tiles)
    tix = tb ? (__builtin_bitreverse32(tix) >> (32u - tb)) : 0u;
  }
  const uint64_t base = tile_base(pass, tix);
  const int W = pass->L - RB;
  const int lane_bits = W < 6 ? W : 6;
  const uint32_t lane = tid & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  Off lane_el = 0;
  for (int b = 0; b < lane_bits; ++b)
    if (lane >> b & 1) lane_el |= Off(1) << pass->q[b];
  const Off lane_off = lane_el * Off(sizeof(C));
  uint64_t wave_el = base;
  for (int b = 6; b < W; ++b)
    if (wave >> (b - 6) & 1) wave_el |= uint64_t(1) << pass->q[b];
  // byte step of each register bit (uniform)
  uint64_t rstep[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) rstep[i] = uint64_t(sizeof(C)) << pass->q[W + i];
  C a[R];
  {
    const char* wp = reinterpret_cast<const char*>(amp) + wave_el * sizeof(C);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      uint64_t ro = 0;
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if (j >> i & 1) ro += rstep[i];
      a[j] = *reinterpret_cast<const C*>(wp + ro + lane_off);
    }
  }
  // complex64 with 16 registers and complex128 re-lay out in halves (half
  // the LDS)
  tile_apply<T, RB, kHalves<T, RB>>(a, lds, pass, segs, ops, base, tid, true);
  // The store addresses are formed again from the few values they derive
  // from (opaque to the compiler), so that the sixteen register addresses
  // are not held in scalar registers across the op loop.
  asm volatile("" : "+s"(wave_el));
#pragma unroll
  for (int i = 0; i < RB; ++i) asm volatile("" : "+s"(rstep[i]));
  {
    char* wp = reinterpret_cast<char*>(amp) + wave_el * sizeof(C);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      uint64_t ro = 0;
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if (j >> i & 1) ro += rstep[i];
      *reinterpret_cast<C*>(wp + ro + lane_off) = a[j];
    }
  }
  if (as_const(pass)->flags & kPassOutputs) {
    uint64_t e_reg[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      uint64_t ro = 0;
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if (j >> i & 1) ro += rstep[i];
      e_reg[j] = ro / sizeof(C);
    }
    tile_outputs<T, RB>(a, lds, pass, tix, wave_el + uint64_t(lane_el), e_reg,
                        tid);
  }
}

// complex64 with 16 registers per thread: capped at 102 VGPRs so that at
// least five waves share each SIMD (the build reaches 80 VGPRs, six waves;
// the half re-layouts take 16 KiB of LDS per tile, ten tiles per CU).
template <bool LANE32>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(5)))
    tile_kernel_c64_rb4(float2* __restrict__ amp,
                        const TilePass* __restrict__ pass,
                        const TileSeg* __restrict__ segs,
                        const TileOp* __restrict__ ops) {
  tile_body<float, 4, LANE32>(amp, pass, segs, ops);
}

template <typename T, int RB, bool LANE32>
__global__ void __launch_bounds__(512)
    tile_kernel(typename CxT<T>::type* __restrict__ amp,
                const TilePass* __restrict__ pass,
                const TileSeg* __restrict__ segs,
                const TileOp* __restrict__ ops) {
  tile_body<T, RB, LANE32>(amp, pass, segs, ops);
}

// Kernel variants: 0 = 64-bit lane offsets, 1 = 32-bit lane offsets.
template <typename T, int RB, int V>
static const void* tile_fn() {
  if constexpr (sizeof(T) == 4 && RB == 4)
    return reinterpret_cast<const void*>(&tile_kernel_c64_rb4<V == 1>);
  else
    return reinterpret_cast<const void*>(&tile_kernel<T, RB, V == 1>);
}

template <typename T, int RB, int V>
static hipError_t tile_launch(void* amp, int n, int L, bool outputs,
                              const TilePass* pass, const TileSeg* segs,
                              const TileOp* ops, hipStream_t stream) {
  using C = typename CxT<T>::type;
  // re-layouts in halves need one component per amplitude; the folded
  // outputs stage FP64 values (8 bytes)
  const size_t lds = !kHalves<T, RB> ? size_t(sizeof(C)) << L
                     : outputs      ? std::max(size_t(8), sizeof(T)) << L
                                    : size_t(sizeof(T)) << L;
  // set once per kernel function; callers on several threads (the server's
  // scheduler and its clients) reach this together, hence call_once
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute(tile_fn<T, RB, V>(),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024);
  });
  if (attr_err != hipSuccess) return attr_err;
  const unsigned threads = 1u << (L - RB);
  const uint64_t tiles = uint64_t(1) << (n - L);
  if constexpr (sizeof(T) == 4 && RB == 4) {
    tile_kernel_c64_rb4<V == 1><<<unsigned(tiles), threads, lds, stream>>>(
        static_cast<C*>(amp), pass, segs, ops);
  } else {
    tile_kernel<T, RB, V == 1><<<unsigned(tiles), threads, lds, stream>>>(
        static_cast<C*>(amp), pass, segs, ops);
  }
  return hipGetLastError();
}

hipError_t launch_tile(int prec, int rb, void* amp, int n,
                       const TilePass& host_pass, const TilePass* pass,
                       const TileSeg* segs, const TileOp* ops,
                       hipStream_t stream) {
  const int L = host_pass.L;
  const bool boff32 = (host_pass.flags & kPassLane32) != 0;
  if (L - rb < 0 || L - rb > 9 || L > kMaxTileBits || n - L > 31)
    return hipErrorInvalidValue;
  const bool outputs = (host_pass.flags & kPassOutputs) != 0;
#define QSV_T(T, RBV, V) \
  return tile_launch<T, RBV, V>(amp, n, L, outputs, pass, segs, ops, stream)
  if (prec == 1) {
    if (rb == 3) {
      if (boff32) QSV_T(float, 3, 1);
      QSV_T(float, 3, 0);
    }
    if (rb == 4) {
      if (boff32) QSV_T(float, 4, 1);
      QSV_T(float, 4, 0);
    }
    if (rb != 5) return hipErrorInvalidValue;
    if (boff32) QSV_T(float, 5, 1);
    QSV_T(float, 5, 0);
  }
  // complex128 tiles use 8 or 16 registers per thread (the planner rejects
  // reg_log2 = 5 for them: 32 double2 registers would spill)
  if (rb == 3) {
    if (boff32) QSV_T(double, 3, 1);
    QSV_T(double, 3, 0);
  }
  if (rb != 4) return hipErrorInvalidValue;
  if (boff32) QSV_T(double, 4, 1);
  QSV_T(double, 4, 0);
#undef QSV_T
}

}  // namespace qsv
