// Batched ragged subcircuit variants.
//
// Circuit cutting evaluates every variant of every subcircuit independently
// (Section III.A; the evaluator runs them as a process pool, Section IV.A).
// Here the batch runs in phases: phase p applies pass p of every variant
// that has one, with the tiles of all those variants spread evenly over the
// work-groups, and kernel boundaries separate the phases.  A variant whose
// 2^w amplitudes fit one tile starts from |0...0> in registers, applies all
// of its gates in one tile pass in phase 0 and writes its probability
// vector: its state never touches HBM.  A wider variant keeps its state in
// the batch's state buffer between phases; its first pass starts from
// |0...0> generated in registers and its last writes the probabilities
// instead of the amplitudes.  No variant's tiles wait for another variant,
// so a wide variant no longer bounds the batch's time, and each tile is
// computed the same way whatever else is in the batch.
#include <mutex>
#include "batch_internal.h"
#include "tile_core.h"

namespace qsv {

template <typename T, typename OUT, int RB>
__device__ __forceinline__ void batch_phase_body(
    const BatchCircuit* __restrict__ circs, const TilePass* __restrict__ passes,
    const TileSeg* __restrict__ segs, const TileOp* __restrict__ ops,
    const BatchWork* __restrict__ work, uint32_t n_work, uint64_t n_tiles,
    uint64_t n_cost, int phase, OUT* __restrict__ out,
    typename CxT<T>::type* __restrict__ states) {
  using C = typename CxT<T>::type;
  constexpr int R = 1 << RB;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  // this work-group's share of the phase: the tiles whose cumulative cost
  // start lies in [clo, chi)
  const uint64_t clo = n_cost * blockIdx.x / gridDim.x;
  const uint64_t chi = n_cost * (blockIdx.x + 1) / gridDim.x;
  // tile index of the first tile starting at or after cost c
  auto first_tile_at = [&](uint64_t c) -> uint64_t {
    if (c >= n_cost) return n_tiles;
    uint32_t a0 = 0, a1 = n_work;  // last entry with cost_begin <= c
    while (a1 - a0 > 1) {
      const uint32_t mid = (a0 + a1) / 2;
      if (work[mid].cost_begin <= c) a0 = mid; else a1 = mid;
    }
    const uint64_t into = c - work[a0].cost_begin;
    const uint64_t tc = work[a0].tile_cost;
    return work[a0].tile_begin + (into + tc - 1) / tc;
  };
  const uint64_t lo = first_tile_at(clo), hi = first_tile_at(chi);
  if (lo >= hi) return;  // uniform over the work-group
  // the run holding tile lo: last entry with tile_begin <= lo
  uint32_t e0 = 0, e1 = n_work;
  while (e1 - e0 > 1) {
    const uint32_t mid = (e0 + e1) / 2;
    if (work[mid].tile_begin <= lo) e0 = mid; else e1 = mid;
  }
  uint32_t e = e0;
  for (uint64_t g = lo; g < hi;) {
    const uint64_t run_end =
        e + 1 < n_work ? work[e + 1].tile_begin : n_tiles;
    const BatchCircuit c = circs[work[e].circ];
    const TilePass* pass = passes + c.pass_begin + phase;
    const int L = pass->L;
    const bool active = tid < (1u << (L - RB));
    const bool first = phase == 0, last = phase + 1 == c.n_passes;
    C* state = states + c.state_offset;
    // I/O layout: element index = tile base | register part | thread
    // part; a variant has at most 2^24 amplitudes, so every offset inside
    // its state or its output fits 32 bits
    const uint32_t thr = active ? io_thread_index<RB>(pass, tid) : 0u;
    // the load test is uniform over the wave (inactive lanes of a partly
    // active wave read the tile's first element, in bounds, and their
    // registers are never written back), so the loads issue back to back
    const bool wave_on = __ballot(active) != 0;
    uint64_t roff[R];
    io_reg_offsets<C, RB>(pass, roff);  // bytes of C
    const uint64_t end = run_end < hi ? run_end : hi;
    for (; g < end; ++g) {
      const uint64_t t = g - work[e].tile_begin;
      uint64_t base = t;
      for (int b = 0; b < L; ++b) base = insert_zero64(base, pass->q[b]);
      const char* sb = reinterpret_cast<const char*>(state + base);
      C a[R];
      if (!first && wave_on) {
#pragma unroll
        for (int j = 0; j < R; ++j)
          a[j] = load_at(state, raw_rsrc<C>(sb + roff[j]),
                         thr * uint32_t(sizeof(C)));
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const bool one = first && active && base == 0 && roff[j] == 0 &&
                           thr == 0;
          a[j].x = one ? T(1) : T(0);
          a[j].y = T(0);
        }
      }
      // complex64 with 16 registers re-lays out in halves (half the LDS)
      tile_apply<T, RB, sizeof(T) == 4 && RB == 4>(a, lds, pass, segs, ops,
                                                  base, tid, active);
      if (active) {
        if (last) {
          const char* ob =
              reinterpret_cast<const char*>(out + c.out_offset + base);
#pragma unroll
          for (int j = 0; j < R; ++j) {
            const double x = double(a[j].x), y = double(a[j].y);
            const uint64_t ro = roff[j] / sizeof(C) * sizeof(OUT);
            store_at(raw_rsrc<OUT>(ob + ro), thr * uint32_t(sizeof(OUT)),
                     OUT(x * x + y * y));
          }
        } else {
#pragma unroll
          for (int j = 0; j < R; ++j)
            store_at(raw_rsrc<C>(sb + roff[j]), thr * uint32_t(sizeof(C)),
                     a[j]);
        }
      }
    }
    ++e;
  }
}

template <typename T, typename OUT, int RB>
__global__ void __launch_bounds__(256)
    batch_phase_kernel(const BatchCircuit* __restrict__ circs,
                       const TilePass* __restrict__ passes,
                       const TileSeg* __restrict__ segs,
                       const TileOp* __restrict__ ops,
                       const BatchWork* __restrict__ work, uint32_t n_work,
                       uint64_t n_tiles, uint64_t n_cost, int phase,
                       OUT* __restrict__ out,
                       typename CxT<T>::type* __restrict__ states) {
  batch_phase_body<T, OUT, RB>(circs, passes, segs, ops, work, n_work,
                               n_tiles, n_cost, phase, out, states);
}

// complex64 with 16 registers per thread: capped at 128 VGPRs so that four
// waves share each SIMD.
template <typename OUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    batch_phase_kernel_c64_rb4(const BatchCircuit* __restrict__ circs,
                               const TilePass* __restrict__ passes,
                               const TileSeg* __restrict__ segs,
                               const TileOp* __restrict__ ops,
                               const BatchWork* __restrict__ work,
                               uint32_t n_work, uint64_t n_tiles,
                               uint64_t n_cost, int phase,
                               OUT* __restrict__ out,
                               float2* __restrict__ states) {
  batch_phase_body<float, OUT, 4>(circs, passes, segs, ops, work, n_work,
                                  n_tiles, n_cost, phase, out, states);
}

template <typename T, typename OUT, int RB>
static const void* batch_fn() {
  if constexpr (sizeof(T) == 4 && RB == 4)
    return reinterpret_cast<const void*>(&batch_phase_kernel_c64_rb4<OUT>);
  else
    return reinterpret_cast<const void*>(&batch_phase_kernel<T, OUT, RB>);
}

// LDS of one work-group: the tile, at 4 bytes per amplitude where the
// re-layouts go in halves (complex64, 16 registers per thread).
template <typename T, int RB>
static size_t batch_lds_bytes(int L) {
  using C = typename CxT<T>::type;
  return (sizeof(T) == 4 && RB == 4) ? size_t(4) << L : size_t(sizeof(C)) << L;
}

template <typename T, typename OUT, int RB>
static hipError_t batch_launch_t(const BatchCircuit* circs,
                                 const TilePass* passes, const TileSeg* segs,
                                 const TileOp* ops, const BatchWork* work,
                                 const HostProgram& hp, void* out,
                                 void* states, int L, int grid,
                                 hipStream_t stream) {
  using C = typename CxT<T>::type;
  // set once per kernel function; the server's scheduler thread and its
  // clients can reach this together, hence call_once
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    attr_err = hipFuncSetAttribute(batch_fn<T, OUT, RB>(),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024);
  });
  if (attr_err != hipSuccess) return attr_err;
  const size_t lds = batch_lds_bytes<T, RB>(L);
  const size_t phases = hp.phase_tiles.size();
  for (size_t p = 0; p < phases; ++p) {
    const uint64_t tiles = hp.phase_tiles[p];
    if (!tiles) continue;
    const uint64_t wb = hp.phase_work_begin[p];
    const uint32_t nw = uint32_t(hp.phase_work_begin[p + 1] - wb);
    const unsigned g = unsigned(tiles < uint64_t(grid) ? tiles : uint64_t(grid));
    if constexpr (sizeof(T) == 4 && RB == 4)
      batch_phase_kernel_c64_rb4<OUT><<<g, 256, lds, stream>>>(
          circs, passes, segs, ops, work + wb, nw, tiles, hp.phase_cost[p],
          int(p), static_cast<OUT*>(out), static_cast<C*>(states));
    else
      batch_phase_kernel<T, OUT, RB><<<g, 256, lds, stream>>>(
          circs, passes, segs, ops, work + wb, nw, tiles, hp.phase_cost[p],
          int(p), static_cast<OUT*>(out), static_cast<C*>(states));
  }
  return hipGetLastError();
}

// Resident work-groups per CU of the batch kernel for (prec, out, rb, L).
// (Its LDS: batch_lds_bytes.)
template <typename T, typename OUT, int RB>
static int batch_occupancy_t(int L) {
  using C = typename CxT<T>::type;
  (void)hipFuncSetAttribute(batch_fn<T, OUT, RB>(),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, batch_fn<T, OUT, RB>(), 256, batch_lds_bytes<T, RB>(L)) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

int batch_blocks_per_cu(int prec, int out_fp64, int rb, int L) {
  if (prec == 1) {
    if (rb == 4)
      return out_fp64 ? batch_occupancy_t<float, double, 4>(L)
                      : batch_occupancy_t<float, float, 4>(L);
    return out_fp64 ? batch_occupancy_t<float, double, 5>(L)
                    : batch_occupancy_t<float, float, 5>(L);
  }
  return out_fp64 ? batch_occupancy_t<double, double, 4>(L)
                  : batch_occupancy_t<double, float, 4>(L);
}

hipError_t launch_batch(int prec, int out_fp64, int rb,
                        const BatchCircuit* circs, const TilePass* passes,
                        const TileSeg* segs, const TileOp* ops,
                        const BatchWork* work, const HostProgram& hp,
                        void* out, void* states, int L, int grid,
                        hipStream_t stream) {
  if (L - rb < 0 || L - rb > 8 || grid < 1) return hipErrorInvalidValue;
#define QSV_B(T, O, RBV)                                                  \
  return batch_launch_t<T, O, RBV>(circs, passes, segs, ops, work, hp, out, \
                                   states, L, grid, stream)
  if (prec == 1) {
    if (out_fp64) {
      if (rb == 4) QSV_B(float, double, 4);
      QSV_B(float, double, 5);
    }
    if (rb == 4) QSV_B(float, float, 4);
    QSV_B(float, float, 5);
  }
  if (out_fp64) QSV_B(double, double, 4);
  QSV_B(double, float, 4);
#undef QSV_B
}

}  // namespace qsv
