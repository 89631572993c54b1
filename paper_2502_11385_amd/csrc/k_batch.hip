// Batched ragged subcircuit variants in one persistent launch.
//
// Circuit cutting evaluates every variant of every subcircuit independently
// (Section III.A; the evaluator runs them as a process pool, Section IV.A).
// Here one launch runs the whole batch: work-group b takes variants
// order[b], order[b + G], ... (order = longest first), so the assignment is
// static and each variant's result does not depend on what else is in the
// batch.  A variant whose 2^w amplitudes fit one tile starts from |0...0>
// in registers, applies all of its gates in one tile pass and writes its
// probability vector: its state never touches HBM.  Wider variants run their
// tile passes over a private scratch slot of the work-group, starting from
// |0...0> generated in registers, with the probabilities written by the last
// pass instead of the amplitudes.
#include "tile_core.h"

namespace qsv {

template <typename T, typename OUT, int RB>
__global__ void __launch_bounds__(256)
    batch_kernel(const BatchCircuit* __restrict__ circs,
                 const int32_t* __restrict__ order, int32_t count,
                 const TilePass* __restrict__ passes,
                 const TileSeg* __restrict__ segs,
                 const TileOp* __restrict__ ops, OUT* __restrict__ out,
                 typename CxT<T>::type* __restrict__ scratch,
                 uint64_t slot_amps) {
  using C = typename CxT<T>::type;
  constexpr int R = 1 << RB;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  C* slot = scratch + uint64_t(blockIdx.x) * slot_amps;

  for (int k = blockIdx.x; k < count; k += gridDim.x) {
    const BatchCircuit c = circs[order[k]];
    for (int pi = 0; pi < c.n_passes; ++pi) {
      const TilePass* pass = passes + c.pass_begin + pi;
      const int L = pass->L;
      const bool active = tid < (1u << (L - RB));
      const bool first = pi == 0, last = pi + 1 == c.n_passes;
      const uint64_t ntiles = uint64_t(1) << (c.w - L);
      // I/O layout: element index = tile base | register part | thread
      // part; a variant has at most 2^24 amplitudes, so every offset inside
      // the slot or the variant's output fits 32 bits
      const uint32_t thr = active ? io_thread_index<RB>(pass, tid) : 0u;
      uint64_t roff[R];
      io_reg_offsets<C, RB>(pass, roff);  // bytes of C
      for (uint64_t t = 0; t < ntiles; ++t) {
        uint64_t base = t;
        for (int b = 0; b < L; ++b) base = insert_zero64(base, pass->q[b]);
        const char* sb = reinterpret_cast<const char*>(slot + base);
        C a[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (!first && active) {
            a[j] = load_at(slot, raw_rsrc<C>(sb + roff[j]),
                           thr * uint32_t(sizeof(C)));
          } else {
            const bool one = first && active && base == 0 && roff[j] == 0 &&
                             thr == 0;
            a[j].x = one ? T(1) : T(0);
            a[j].y = T(0);
          }
        }
        tile_apply<T, RB>(a, lds, pass, segs, ops, base, tid, active);
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
      // All tiles of this pass are stored before the next pass reads them
      // (one work-group owns the slot; the barrier orders its accesses).
      __syncthreads();
    }
  }
}

template <typename T, typename OUT, int RB>
static hipError_t batch_launch_t(const BatchCircuit* circs,
                                 const int32_t* order, int32_t count,
                                 const TilePass* passes, const TileSeg* segs,
                                 const TileOp* ops, void* out, void* scratch,
                                 uint64_t slot_amps, int L, int grid,
                                 hipStream_t stream) {
  using C = typename CxT<T>::type;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&batch_kernel<T, OUT, RB>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const size_t lds = size_t(sizeof(C)) << L;
  batch_kernel<T, OUT, RB><<<grid, 256, lds, stream>>>(
      circs, order, count, passes, segs, ops, static_cast<OUT*>(out),
      static_cast<C*>(scratch), slot_amps);
  return hipGetLastError();
}

// Resident work-groups per CU of the batch kernel for (prec, out, rb, L).
template <typename T, typename OUT, int RB>
static int batch_occupancy_t(int L) {
  using C = typename CxT<T>::type;
  (void)hipFuncSetAttribute(
      reinterpret_cast<const void*>(&batch_kernel<T, OUT, RB>),
      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, reinterpret_cast<const void*>(&batch_kernel<T, OUT, RB>), 256,
          size_t(sizeof(C)) << L) != hipSuccess) {
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

hipError_t launch_batch(int prec, int out_fp64, int rb, const BatchCircuit* circs,
                        const int32_t* order, int32_t count,
                        const TilePass* passes, const TileSeg* segs,
                        const TileOp* ops, void* out, void* scratch,
                        uint64_t slot_amps, int L, int grid,
                        hipStream_t stream) {
  if (L - rb < 0 || L - rb > 8) return hipErrorInvalidValue;
#define QSV_B(T, O, RBV)                                                     \
  return batch_launch_t<T, O, RBV>(circs, order, count, passes, segs, ops,   \
                                   out, scratch, slot_amps, L, grid, stream)
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
