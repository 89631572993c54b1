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

// One tile pass per work-group.  At most 512 threads per tile (L - RB <= 9).
// BOFF32: the I/O layout's thread byte offsets fit 32 bits (decided on the
// host per pass), so loads and stores use a uniform per-register pointer
// plus a 32-bit per-thread offset and need no 64-bit vector address math.
template <typename T, int RB, bool BOFF32>
__device__ __forceinline__ void tile_body(typename CxT<T>::type* __restrict__ amp,
                                          const TilePass* __restrict__ pass,
                                          const TileSeg* __restrict__ segs,
                                          const TileOp* __restrict__ ops) {
  using C = typename CxT<T>::type;
  constexpr int R = 1 << RB;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const int L = pass->L;
  const uint32_t tid = threadIdx.x;
  // Tile base: the block index spread over the non-tile qubits.
  uint64_t base = blockIdx.x;
  for (int b = 0; b < L; ++b) base = insert_zero64(base, pass->q[b]);
  // HBM transfers use the I/O layout: registers select the top RB tile bits
  // and consecutive threads take consecutive low tile bits, so a wave's
  // accesses are contiguous runs of the lowest (always tile) qubits.
  C a[R];
  if constexpr (BOFF32) {
    C* tile = amp + base;
    const uint32_t boff = io_thread_boff<C, RB>(pass, tid);
#pragma unroll
    for (int j = 0; j < R; ++j)
      a[j] = load_at(tile, io_reg_rsrc<C, RB>(tile, pass, j), boff);
    tile_apply<T, RB>(a, lds, pass, segs, ops, base, tid, true);
#pragma unroll
    for (int j = 0; j < R; ++j)
      store_at(io_reg_rsrc<C, RB>(tile, pass, j), boff, a[j]);
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
// waves share each SIMD (occupancy hides HBM and VALU latencies).
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

template <typename T, int RB, bool BOFF32>
static const void* tile_fn() {
  if constexpr (sizeof(T) == 4 && RB == 4)
    return reinterpret_cast<const void*>(&tile_kernel_c64_rb4<BOFF32>);
  else
    return reinterpret_cast<const void*>(&tile_kernel<T, RB, BOFF32>);
}

template <typename T, int RB, bool BOFF32>
static hipError_t tile_launch(void* amp, int n, int L, const TilePass* pass,
                              const TileSeg* segs, const TileOp* ops,
                              hipStream_t stream) {
  using C = typename CxT<T>::type;
  const size_t lds = size_t(sizeof(C)) << L;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(tile_fn<T, RB, BOFF32>(),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const unsigned threads = 1u << (L - RB);
  const uint64_t tiles = uint64_t(1) << (n - L);
  if constexpr (sizeof(T) == 4 && RB == 4)
    tile_kernel_c64_rb4<BOFF32><<<unsigned(tiles), threads, lds, stream>>>(
        static_cast<C*>(amp), pass, segs, ops);
  else
    tile_kernel<T, RB, BOFF32><<<unsigned(tiles), threads, lds, stream>>>(
        static_cast<C*>(amp), pass, segs, ops);
  return hipGetLastError();
}

hipError_t launch_tile(int prec, int rb, void* amp, int n, int L,
                       bool boff32, const TilePass* pass, const TileSeg* segs,
                       const TileOp* ops, hipStream_t stream) {
  if (L - rb < 0 || L - rb > 9 || n - L > 31) return hipErrorInvalidValue;
#define QSV_T(T, RBV)                                                        \
  return boff32 ? tile_launch<T, RBV, true>(amp, n, L, pass, segs, ops, stream) \
                : tile_launch<T, RBV, false>(amp, n, L, pass, segs, ops, stream)
  if (prec == 1) {
    if (rb == 4) QSV_T(float, 4);
    QSV_T(float, 5);
  }
  // complex128 tiles always use 16 registers per thread (the planner
  // rejects reg_log2 = 5 for them: 32 double2 registers would spill)
  if (rb != 4) return hipErrorInvalidValue;
  QSV_T(double, 4);
#undef QSV_T
}

}  // namespace qsv
