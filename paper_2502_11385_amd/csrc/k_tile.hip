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
#include "tile_core.h"

namespace qsv {

// Tile index -> global index of the tile's first amplitude: the index's
// bits spread over the non-tile qubits.
__device__ __forceinline__ uint64_t tile_base(const TilePass* pass,
                                              uint32_t tile) {
  uint64_t base = tile;
  const int L = pass->L;
  for (int b = 0; b < L; ++b) base = insert_zero64(base, pass->q[b]);
  return base;
}

// One tile per work-group.  At most 512 threads per tile (L - RB <= 9).
// BOFF32 as for the persistent kernel; otherwise 64-bit addressing.
template <typename T, int RB, bool BOFF32>
__device__ __forceinline__ void tile_body(typename CxT<T>::type* __restrict__ amp,
                                          const TilePass* __restrict__ pass,
                                          const TileSeg* __restrict__ segs,
                                          const TileOp* __restrict__ ops) {
  using C = typename CxT<T>::type;
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
  // HBM transfers use the I/O layout: registers select the top RB tile bits
  // and consecutive threads take consecutive low tile bits, so a wave's
  // accesses are contiguous runs of the lowest (always tile) qubits.
  C a[R];
  if constexpr (BOFF32) {
    const uint32_t boff = io_thread_boff<C, RB>(pass, tid);
    uint64_t roff[R];
    io_reg_offsets<C, RB>(pass, roff);
    const char* tile = reinterpret_cast<const char*>(amp + base);
#pragma unroll
    for (int j = 0; j < R; ++j)
      a[j] = load_at(amp, raw_rsrc<C>(tile + roff[j]), boff);
    tile_apply<T, RB>(a, lds, pass, segs, ops, base, tid, true);
#pragma unroll
    for (int j = 0; j < R; ++j) store_at(raw_rsrc<C>(tile + roff[j]), boff, a[j]);
  } else {
    uint64_t gthr, greg[RB];
    io_offsets<RB>(pass, base, tid, &gthr, greg);
#pragma unroll
    for (int j = 0; j < R; ++j) a[j] = amp[io_addr<RB>(gthr, greg, j)];
    tile_apply<T, RB>(a, lds, pass, segs, ops, base, tid, true);
#pragma unroll
    for (int j = 0; j < R; ++j) amp[io_addr<RB>(gthr, greg, j)] = a[j];
  }
}

// complex64 with 16 registers per thread: capped at 128 VGPRs so that four
// waves share each SIMD.
template <bool BOFF32>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
    tile_kernel_c64_rb4(float2* __restrict__ amp,
                        const TilePass* __restrict__ pass,
                        const TileSeg* __restrict__ segs,
                        const TileOp* __restrict__ ops) {
  tile_body<float, 4, BOFF32>(amp, pass, segs, ops);
}

template <typename T, int RB, bool BOFF32>
__global__ void __launch_bounds__(512)
    tile_kernel(typename CxT<T>::type* __restrict__ amp,
                const TilePass* __restrict__ pass,
                const TileSeg* __restrict__ segs,
                const TileOp* __restrict__ ops) {
  tile_body<T, RB, BOFF32>(amp, pass, segs, ops);
}

// Kernel variants: 0 = 64-bit addressing, 1 = 32-bit offsets.
template <typename T, int RB, int V>
static const void* tile_fn() {
  if constexpr (sizeof(T) == 4 && RB == 4)
    return reinterpret_cast<const void*>(&tile_kernel_c64_rb4<V == 1>);
  else
    return reinterpret_cast<const void*>(&tile_kernel<T, RB, V == 1>);
}

template <typename T, int RB, int V>
static hipError_t tile_launch(void* amp, int n, int L, const TilePass* pass,
                              const TileSeg* segs, const TileOp* ops,
                              hipStream_t stream) {
  using C = typename CxT<T>::type;
  const size_t lds = size_t(sizeof(C)) << L;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(tile_fn<T, RB, V>(),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
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

hipError_t launch_tile(int prec, int rb, void* amp, int n, int L,
                       int32_t flags, const TilePass* pass, const TileSeg* segs,
                       const TileOp* ops, hipStream_t stream) {
  const bool boff32 = (flags & kPassBoff32) != 0;
  if (L - rb < 0 || L - rb > 9 || L > kMaxTileBits || n - L > 31)
    return hipErrorInvalidValue;
#define QSV_T(T, RBV, V) return tile_launch<T, RBV, V>(amp, n, L, pass, segs, ops, stream)
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
