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
#include "device_common.h"

namespace qsv {

// Bijective XOR swizzle of tile-local indices to spread LDS banks.
template <typename T>
__device__ __forceinline__ uint32_t lds_swz(uint32_t r) {
  if constexpr (sizeof(T) == 4)
    return r ^ (((r >> 4) ^ (r >> 8)) & 15u);
  else
    return r ^ (((r >> 3) ^ (r >> 6) ^ (r >> 9)) & 7u);
}

template <int I, int R, bool CTRL, typename C, typename T>
__device__ __forceinline__ void dense1_regs(C* a, T m0r, T m0i, T m1r, T m1i,
                                            T m2r, T m2i, T m3r, T m3i,
                                            uint32_t rt, const uint32_t* lr,
                                            uint32_t lctrl) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (j & (1 << I)) continue;
    const int j1 = j | (1 << I);
    const C x0 = a[j], x1 = a[j1];
    C y0, y1;
    y0.x = m0r * x0.x - m0i * x0.y + m1r * x1.x - m1i * x1.y;
    y0.y = m0r * x0.y + m0i * x0.x + m1r * x1.y + m1i * x1.x;
    y1.x = m2r * x0.x - m2i * x0.y + m3r * x1.x - m3i * x1.y;
    y1.y = m2r * x0.y + m2i * x0.x + m3r * x1.y + m3i * x1.x;
    if constexpr (CTRL) {
      const bool on = ((rt | lr[j]) & lctrl) == lctrl;
      a[j] = csel(on, y0, x0);
      a[j1] = csel(on, y1, x1);
    } else {
      a[j] = y0;
      a[j1] = y1;
    }
  }
}

template <int R, bool CTRL, typename C, typename T>
__device__ __forceinline__ void dense1_dispatch(int reg, C* a, const T* m,
                                                uint32_t rt, const uint32_t* lr,
                                                uint32_t lctrl) {
#define QSV_D1(I)                                                          \
  case I:                                                                  \
    if constexpr ((1 << I) < R)                                            \
      dense1_regs<I, R, CTRL>(a, m[0], m[1], m[2], m[3], m[4], m[5], m[6], \
                              m[7], rt, lr, lctrl);                        \
    break;
  switch (reg) {
    QSV_D1(0)
    QSV_D1(1)
    QSV_D1(2)
    QSV_D1(3)
    QSV_D1(4)
    QSV_D1(5)
  }
#undef QSV_D1
}

// Register layout: reg_bits[i] (ascending) is the tile-local bit selecting
// register i; the remaining bits, ascending, come from the thread index.
template <int RB>
struct Layout {
  int rb[RB];
};

template <int RB>
__device__ __forceinline__ bool same_layout(const Layout<RB>& a,
                                            const Layout<RB>& b) {
  bool same = true;
#pragma unroll
  for (int i = 0; i < RB; ++i) same = same && a.rb[i] == b.rb[i];
  return same;
}

template <int RB>
__device__ __forceinline__ uint32_t thread_local_base(const Layout<RB>& lay,
                                                      uint32_t tid) {
  uint32_t rt = tid;
#pragma unroll
  for (int i = 0; i < RB; ++i) rt = insert_zero32(rt, lay.rb[i]);
  return rt;
}

template <int RB>
__device__ __forceinline__ uint32_t reg_offset(const Layout<RB>& lay, int j) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < RB; ++i)
    if (j >> i & 1) o |= 1u << lay.rb[i];
  return o;
}

// Move the tile from layout `from` to layout `to` through LDS.
template <typename T, int RB, typename C>
__device__ __forceinline__ void relayout(C* a, C* lds, const Layout<RB>& from,
                                         const Layout<RB>& to, uint32_t tid) {
  constexpr int R = 1 << RB;
  const uint32_t rf = thread_local_base(from, tid);
#pragma unroll
  for (int j = 0; j < R; ++j) lds[lds_swz<T>(rf | reg_offset(from, j))] = a[j];
  __syncthreads();
  const uint32_t rt = thread_local_base(to, tid);
#pragma unroll
  for (int j = 0; j < R; ++j) a[j] = lds[lds_swz<T>(rt | reg_offset(to, j))];
  __syncthreads();
}

// At most 512 threads per tile (L - RB <= 9), which leaves up to 256 VGPRs
// per lane for the register-resident tile.
template <typename T, int RB>
__global__ void __launch_bounds__(512)
    tile_kernel(typename CxT<T>::type* __restrict__ amp,
                const TilePass* __restrict__ pass,
                const TileSeg* __restrict__ segs,
                const TileOp* __restrict__ ops) {
  using C = typename CxT<T>::type;
  constexpr int R = 1 << RB;
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);

  const int L = pass->L;
  const int W = L - RB;  // thread bits
  const uint32_t tid = threadIdx.x;
  // Tile base: the block index spread over the non-tile qubits.
  uint64_t base = blockIdx.x;
  for (int b = 0; b < L; ++b) base = insert_zero64(base, pass->q[b]);

  // HBM transfers use the I/O layout: registers select the top RB tile bits
  // and consecutive threads take consecutive low tile bits, so a wave's
  // accesses are contiguous runs of the lowest (always tile) qubits.
  Layout<RB> io;
#pragma unroll
  for (int i = 0; i < RB; ++i) io.rb[i] = W + i;
  uint64_t gthr = base;
  for (int b = 0; b < W; ++b)
    if (tid >> b & 1) gthr |= uint64_t(1) << pass->q[b];
  uint64_t greg[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) greg[i] = uint64_t(1) << pass->q[W + i];

  C a[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    uint64_t o = gthr;
#pragma unroll
    for (int i = 0; i < RB; ++i)
      if (j >> i & 1) o |= greg[i];
    a[j] = amp[o];
  }

  Layout<RB> cur = io;
  const int nseg = pass->nseg;
  const TileSeg* sp = segs + pass->seg_begin;
  for (int s = 0; s < nseg; ++s) {
    Layout<RB> lay;
#pragma unroll
    for (int i = 0; i < RB; ++i) lay.rb[i] = sp[s].reg_bits[i];
    if (!same_layout(cur, lay)) relayout<T, RB>(a, lds, cur, lay, tid);
    cur = lay;
    const uint32_t rt = thread_local_base(lay, tid);
    uint32_t lr[R];
#pragma unroll
    for (int j = 0; j < R; ++j) lr[j] = reg_offset(lay, j);

    for (int o = sp[s].op_begin; o < sp[s].op_end; ++o) {
      const TileOp* op = ops + o;
      const uint64_t gctrl = op->gctrl;
      if ((base & gctrl) != gctrl) continue;  // an outer control bit is 0
      const int kind = op->kind;
      const uint32_t lctrl = op->lctrl;
      if (kind == kOpDense1) {
        T m[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if constexpr (sizeof(T) == 4)
            m[e] = op->mf[e];
          else
            m[e] = op->m[e];
        }
        if (lctrl)
          dense1_dispatch<R, true>(op->reg, a, m, rt, lr, lctrl);
        else
          dense1_dispatch<R, false>(op->reg, a, m, rt, lr, lctrl);
      } else if (kind == kOpPhase) {
        C ph;
        ph.x = T(op->m[0]);
        ph.y = T(op->m[1]);
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const bool on = ((rt | lr[j]) & lctrl) == lctrl;
          const C y = cmul(a[j], ph);
          a[j] = csel(on, y, a[j]);
        }
      } else {  // kOpDiag
        const int dk = op->dk;
        const int d0 = op->dbit0, d1 = op->dbit1;
        const uint32_t g0 =
            d0 < 0 ? uint32_t((base >> ((-1 - d0) & 63)) & 1) : 0u;
        const uint32_t g1 =
            (dk > 1 && d1 < 0) ? uint32_t((base >> ((-1 - d1) & 63)) & 1) : 0u;
        C t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          t[e].x = T(op->m[2 * e]);
          t[e].y = T(op->m[2 * e + 1]);
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t r = rt | lr[j];
          const uint32_t b0 = d0 >= 0 ? (r >> (d0 & 31)) & 1u : g0;
          const uint32_t b1 =
              dk > 1 ? (d1 >= 0 ? (r >> (d1 & 31)) & 1u : g1) : 0u;
          const C f01 = csel(b0 != 0, t[1], t[0]);
          const C f23 = csel(b0 != 0, t[3], t[2]);
          const C f = csel(b1 != 0, f23, f01);
          const bool on = (r & lctrl) == lctrl;
          const C y = cmul(a[j], f);
          a[j] = csel(on, y, a[j]);
        }
      }
    }
  }
  if (!same_layout(cur, io)) relayout<T, RB>(a, lds, cur, io, tid);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    uint64_t o = gthr;
#pragma unroll
    for (int i = 0; i < RB; ++i)
      if (j >> i & 1) o |= greg[i];
    amp[o] = a[j];
  }
}

template <typename T, int RB>
static hipError_t tile_launch(void* amp, int n, int L, const TilePass* pass,
                              const TileSeg* segs, const TileOp* ops,
                              hipStream_t stream) {
  using C = typename CxT<T>::type;
  const size_t lds = size_t(sizeof(C)) << L;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&tile_kernel<T, RB>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const unsigned threads = 1u << (L - RB);
  const uint64_t tiles = uint64_t(1) << (n - L);
  tile_kernel<T, RB><<<unsigned(tiles), threads, lds, stream>>>(
      static_cast<C*>(amp), pass, segs, ops);
  return hipGetLastError();
}

hipError_t launch_tile(int prec, int rb, void* amp, int n, int L,
                       const TilePass* pass, const TileSeg* segs,
                       const TileOp* ops, hipStream_t stream) {
  if (L - rb < 0 || L - rb > 9 || n - L > 31) return hipErrorInvalidValue;
  if (prec == 1)
    return rb == 4 ? tile_launch<float, 4>(amp, n, L, pass, segs, ops, stream)
                   : tile_launch<float, 5>(amp, n, L, pass, segs, ops, stream);
  return rb == 4 ? tile_launch<double, 4>(amp, n, L, pass, segs, ops, stream)
                 : tile_launch<double, 5>(amp, n, L, pass, segs, ops, stream);
}

}  // namespace qsv
