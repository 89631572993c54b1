// Register-tile core shared by the tile-pass kernel and the batch kernel.
//
// A tile of 2^L amplitudes lives in registers, 2^RB per thread.  A register
// layout names the RB tile-local bits that select a thread's register; the
// other tile bits come from the thread index.  Every dense gate of a
// segment targets a register bit, so its 2x2 update stays in the thread;
// between segments the tile is re-laid out through LDS.
#pragma once
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
      // rt and lr[j] have disjoint bits: test the thread part once
      const bool on = ((rt & lctrl) | (lr[j] & lctrl)) == lctrl;
      a[j] = csel(on, y0, x0);
      a[j1] = csel(on, y1, x1);
    } else {
      a[j] = y0;
      a[j1] = y1;
    }
  }
}

// The same update with the matrix chosen per pair by tile-local bit mbit:
// m0 where the bit is 0, m1 where it is 1 (mbit differs from the target).
template <int I, int R, bool CTRL, typename C, typename T>
__device__ __forceinline__ void dense1_mux_regs(C* a, const T* m0,
                                                const T* m1, uint32_t rt,
                                                const uint32_t* lr,
                                                uint32_t lctrl, int mbit) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (j & (1 << I)) continue;
    const int j1 = j | (1 << I);
    const bool sel = (((rt >> mbit) | (lr[j] >> mbit)) & 1u) != 0;
    T m[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) m[e] = sel ? m1[e] : m0[e];
    const C x0 = a[j], x1 = a[j1];
    C y0, y1;
    y0.x = m[0] * x0.x - m[1] * x0.y + m[2] * x1.x - m[3] * x1.y;
    y0.y = m[0] * x0.y + m[1] * x0.x + m[2] * x1.y + m[3] * x1.x;
    y1.x = m[4] * x0.x - m[5] * x0.y + m[6] * x1.x - m[7] * x1.y;
    y1.y = m[4] * x0.y + m[5] * x0.x + m[6] * x1.y + m[7] * x1.x;
    if constexpr (CTRL) {
      const bool on = ((rt & lctrl) | (lr[j] & lctrl)) == lctrl;
      a[j] = csel(on, y0, x0);
      a[j1] = csel(on, y1, x1);
    } else {
      a[j] = y0;
      a[j1] = y1;
    }
  }
}

template <int R, bool CTRL, typename C, typename T>
__device__ __forceinline__ void dense1_mux_dispatch(int reg, C* a, const T* m0,
                                                    const T* m1, uint32_t rt,
                                                    const uint32_t* lr,
                                                    uint32_t lctrl, int mbit) {
#define QSV_D1M(I)                                                        \
  case I:                                                                 \
    if constexpr ((1 << I) < R) {                                         \
      dense1_mux_regs<I, R, CTRL>(a, m0, m1, rt, lr, lctrl, mbit);        \
      break;                                                              \
    } else {                                                              \
      __builtin_unreachable();                                            \
    }
  switch (reg) {
    QSV_D1M(0)
    QSV_D1M(1)
    QSV_D1M(2)
    QSV_D1M(3)
    QSV_D1M(4)
    QSV_D1M(5)
    default:
      __builtin_unreachable();  // the planner emits reg < RB only
  }
#undef QSV_D1M
}

template <int R, bool CTRL, typename C, typename T>
__device__ __forceinline__ void dense1_dispatch(int reg, C* a, const T* m,
                                                uint32_t rt, const uint32_t* lr,
                                                uint32_t lctrl) {
#define QSV_D1(I)                                                          \
  case I:                                                                  \
    if constexpr ((1 << I) < R) {                                          \
      dense1_regs<I, R, CTRL>(a, m[0], m[1], m[2], m[3], m[4], m[5], m[6], \
                              m[7], rt, lr, lctrl);                        \
      break;                                                               \
    } else {                                                               \
      __builtin_unreachable();                                             \
    }
  switch (reg) {
    QSV_D1(0)
    QSV_D1(1)
    QSV_D1(2)
    QSV_D1(3)
    QSV_D1(4)
    QSV_D1(5)
    default:
      __builtin_unreachable();  // the planner emits reg < RB only
  }
#undef QSV_D1
}

// The mux update when the mux bit is register bit K of the segment: which
// matrix a pair takes is known at compile time, both matrices are uniform.
template <int I, int K, int R, typename C, typename T>
__device__ __forceinline__ void dense1_muxreg_regs(C* a, const T* m0,
                                                   const T* m1) {
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (j & (1 << I)) continue;
    const int j1 = j | (1 << I);
    const T* m = (j >> K & 1) ? m1 : m0;
    const C x0 = a[j], x1 = a[j1];
    C y0, y1;
    y0.x = m[0] * x0.x - m[1] * x0.y + m[2] * x1.x - m[3] * x1.y;
    y0.y = m[0] * x0.y + m[1] * x0.x + m[2] * x1.y + m[3] * x1.x;
    y1.x = m[4] * x0.x - m[5] * x0.y + m[6] * x1.x - m[7] * x1.y;
    y1.y = m[4] * x0.y + m[5] * x0.x + m[6] * x1.y + m[7] * x1.x;
    a[j] = y0;
    a[j1] = y1;
  }
}

template <int R, typename C, typename T>
__device__ __forceinline__ void dense1_muxreg_dispatch(int reg, int k, C* a,
                                                       const T* m0,
                                                       const T* m1) {
#define QSV_D1K(I, K)                                                     \
  case I * 8 + K:                                                         \
    if constexpr ((1 << I) < R && (1 << K) < R && I != K) {               \
      dense1_muxreg_regs<I, K, R>(a, m0, m1);                             \
      break;                                                              \
    } else {                                                              \
      __builtin_unreachable();                                            \
    }
#define QSV_D1K_ROW(I) \
  QSV_D1K(I, 0) QSV_D1K(I, 1) QSV_D1K(I, 2) QSV_D1K(I, 3) QSV_D1K(I, 4)
  switch (reg * 8 + k) {
    QSV_D1K_ROW(0)
    QSV_D1K_ROW(1)
    QSV_D1K_ROW(2)
    QSV_D1K_ROW(3)
    QSV_D1K_ROW(4)
    default:
      __builtin_unreachable();  // reg, k < RB <= 5 and reg != k
  }
#undef QSV_D1K_ROW
#undef QSV_D1K
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

// LDS byte offsets of a layout's registers, swz(reg_offset(j)) * sizeof(C),
// as uniform values.  The swizzle is linear over XOR, so the offsets are
// XOR combinations of one value per register bit.
template <typename T, int RB>
__device__ __forceinline__ void lds_reg_offsets(const Layout<RB>& lay,
                                                uint32_t* so) {
  using C = typename CxT<T>::type;
  uint32_t basis[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
    basis[i] = __builtin_amdgcn_readfirstlane(
        lds_swz<T>(1u << lay.rb[i]) * uint32_t(sizeof(C)));
  so[0] = 0;
#pragma unroll
  for (int j = 1; j < (1 << RB); ++j)
    so[j] = so[j & (j - 1)] ^ basis[__builtin_ctz(j)];
}

// Move the tile from layout `from` to layout `to` through LDS.
// Threads with active == false (beyond the tile) only join the barriers.
template <typename T, int RB, typename C>
__device__ __forceinline__ void relayout(C* a, C* lds, const Layout<RB>& from,
                                         const Layout<RB>& to, uint32_t tid,
                                         bool active) {
  constexpr int R = 1 << RB;
  // The thread and register parts of a tile index have disjoint bits and
  // the swizzle is linear over XOR: swz(rt | o_j) = swz(rt) ^ swz(o_j), one
  // per-thread term and one uniform term per register.
  char* lb = reinterpret_cast<char*>(lds);
  uint32_t so[R];
  if (active) {
    lds_reg_offsets<T, RB>(from, so);
    const uint32_t rf =
        lds_swz<T>(thread_local_base(from, tid)) * uint32_t(sizeof(C));
#pragma unroll
    for (int j = 0; j < R; ++j) *reinterpret_cast<C*>(lb + (rf ^ so[j])) = a[j];
  }
  __syncthreads();
  if (active) {
    lds_reg_offsets<T, RB>(to, so);
    const uint32_t rt =
        lds_swz<T>(thread_local_base(to, tid)) * uint32_t(sizeof(C));
#pragma unroll
    for (int j = 0; j < R; ++j) a[j] = *reinterpret_cast<const C*>(lb + (rt ^ so[j]));
  }
  __syncthreads();
}

// e^{2 pi i t / 2^32} for a fixed-point fraction of a turn.  The top 24
// bits go through sincospi exactly (an int32 with its low 8 bits clear is
// exact in FP32); the low 8 bits, below 4e-7 rad, enter to first order.
__device__ __forceinline__ float2 turn_phase32(uint32_t t) {
  const float y = float(int32_t(t & ~0xFFu)) * 0x1p-31f;
  float sn, cs;
  sincospif(y, &sn, &cs);
  const float d = float(t & 0xFFu) * (3.14159265358979f * 0x1p-31f);
  return make_float2(__builtin_fmaf(-sn, d, cs), __builtin_fmaf(cs, d, sn));
}

// e^{2 pi i t / 2^64} in FP64 (the int64 -> double rounding is 2^-53 of a
// half turn at most).
__device__ __forceinline__ double2 turn_phase64(uint64_t t) {
  const double y = double(int64_t(t)) * 0x1p-63;
  double sn, cs;
  sincospi(y, &sn, &cs);
  return make_double2(cs, sn);
}

// Multiply the register tile by a PhaseBlock's factor.  Per thread, each
// accumulator sums the angles of its terms whose thread and outer bits are
// all 1 (terms without thread bits are uniform over the tile); then one
// phase per accumulator multiplies the registers that carry its register
// bit, and the register table (terms on register bits only) the rest.
template <typename T, int RB>
__device__ __forceinline__ void phase_block(typename CxT<T>::type* a,
                                            const PhaseBlock* pb, uint32_t rt,
                                            uint64_t base) {
  using C = typename CxT<T>::type;
  using U = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
  constexpr int R = 1 << RB;
  const PhaseTerm* t = reinterpret_cast<const PhaseTerm*>(pb + 1);
  U acc[RB + 1];
  // A term's first 16 bytes (outer mask, thread mask, 32-bit turns) are
  // read as one vector, so that each term costs one scalar load round trip.
  auto head = [](const PhaseTerm* p, uint64_t* gm, uint32_t* tm, U* w) {
    const uint4 h = *reinterpret_cast<const uint4*>(p);
    *gm = uint64_t(h.x) | (uint64_t(h.y) << 32);
    *tm = h.z;
    if constexpr (sizeof(T) == 4) *w = U(h.w);
    else *w = U(p->turns);
  };
#pragma unroll
  for (int k = 0; k <= RB; ++k) {
    U au = 0;
    const int nu = pb->n_uni[k];
#pragma unroll 4
    for (int i = 0; i < nu; ++i, ++t) {
      uint64_t gm;
      uint32_t tm;
      U w;
      head(t, &gm, &tm, &w);
      au += (base & gm) == gm ? w : U(0);
    }
    U av = 0;
    const int nv = pb->n_thr[k];
#pragma unroll 4
    for (int i = 0; i < nv; ++i, ++t) {
      uint64_t gm;
      uint32_t tm;
      U w;
      head(t, &gm, &tm, &w);
      const bool on = ((base & gm) == gm) & ((rt & tm) == tm);
      av += on ? w : U(0);
    }
    acc[k] = au + av;
  }
  if (pb->n_uni[0] + pb->n_thr[0] > 0) {
    C f0;
    if constexpr (sizeof(T) == 4) f0 = turn_phase32(acc[0]);
    else f0 = turn_phase64(acc[0]);
    if (pb->has_table) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        C u;
        if constexpr (sizeof(T) == 4) u = make_float2(pb->tf[2 * j], pb->tf[2 * j + 1]);
        else u = make_double2(pb->td[2 * j], pb->td[2 * j + 1]);
        a[j] = cmul(a[j], cmul(f0, u));
      }
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) a[j] = cmul(a[j], f0);
    }
  } else if (pb->has_table) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      C u;
      if constexpr (sizeof(T) == 4) u = make_float2(pb->tf[2 * j], pb->tf[2 * j + 1]);
      else u = make_double2(pb->td[2 * j], pb->td[2 * j + 1]);
      a[j] = cmul(a[j], u);
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (pb->n_uni[1 + r] + pb->n_thr[1 + r] == 0) continue;
    C kr;
    if constexpr (sizeof(T) == 4) kr = turn_phase32(acc[1 + r]);
    else kr = turn_phase64(acc[1 + r]);
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (j >> r & 1) a[j] = cmul(a[j], kr);
  }
}

// Apply every segment of one tile pass to the register tile `a`, which is
// in the I/O layout on entry and is left in the I/O layout on exit.  `base`
// is the tile's global index with all tile bits zero (outer controls and
// diagonal bits outside the tile are read from it).
template <typename T, int RB>
__device__ __forceinline__ void tile_apply(typename CxT<T>::type* a,
                                           typename CxT<T>::type* lds,
                                           const TilePass* pass,
                                           const TileSeg* segs,
                                           const TileOp* ops, uint64_t base,
                                           uint32_t tid, bool active) {
  using C = typename CxT<T>::type;
  constexpr int R = 1 << RB;
  const int W = pass->L - RB;
  Layout<RB> io;
#pragma unroll
  for (int i = 0; i < RB; ++i) io.rb[i] = W + i;
  Layout<RB> cur = io;
  const int nseg = pass->nseg;
  const TileSeg* sp = segs + pass->seg_begin;
  // complex64 amplitudes are carried as 64-bit values, so the copies where
  // the ops' arms and the segments join move register pairs
  using W64 = std::conditional_t<sizeof(T) == 4, uint64_t, C>;
  W64 w[R];
#pragma unroll
  for (int j = 0; j < R; ++j) w[j] = __builtin_bit_cast(W64, a[j]);
  for (int s = 0; s < nseg; ++s) {
    Layout<RB> lay;
#pragma unroll
    for (int i = 0; i < RB; ++i) lay.rb[i] = sp[s].reg_bits[i];
    if (!same_layout(cur, lay)) {
#pragma unroll
      for (int j = 0; j < R; ++j) a[j] = __builtin_bit_cast(C, w[j]);
      relayout<T, RB>(a, lds, cur, lay, tid, active);
#pragma unroll
      for (int j = 0; j < R; ++j) w[j] = __builtin_bit_cast(W64, a[j]);
    }
    cur = lay;
    const uint32_t rt = thread_local_base(lay, tid);
    uint32_t lr[R];
#pragma unroll
    for (int j = 0; j < R; ++j) lr[j] = reg_offset(lay, j);

    for (int o = sp[s].op_begin; o < sp[s].op_end; ++o) {
#pragma unroll
      for (int j = 0; j < R; ++j) a[j] = __builtin_bit_cast(C, w[j]);
      const TileOp* op = ops + o;
      // Read the header and both matrices before any branch, so that the
      // scalar loads issue together and the op waits for them once (a
      // variant that prefetched the next op's fields during this op was
      // slower: the copies and the register pressure cost more than the
      // latency it hid).
      const int kind = op->kind;
      const int oreg = op->reg;
      const int mux = op->mux;
      const int mreg = op->mux_reg;
      const uint32_t lctrl = op->lctrl;
      const uint64_t gctrl = op->gctrl;
      T m0[8], m1[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if constexpr (sizeof(T) == 4) {
          m0[e] = op->mf[e];
          m1[e] = op->mf2[e];
        } else {
          m0[e] = op->m[e];
          m1[e] = op->m2[e];
        }
      }
      if ((base & gctrl) != gctrl) continue;  // an outer control bit is 0
      if (kind == kOpDense1) {
        // an outer mux qubit is fixed per tile: pick the matrix once
        const bool second =
            mux != kMuxNone && mux < 0 && ((base >> ((-1 - mux) & 63)) & 1);
        T m[8], m2[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          m[e] = second ? m1[e] : m0[e];
          m2[e] = m1[e];
        }
        if (mux >= 0 && lctrl == 0 && mreg >= 0) {
          // mux bit in a register: the pairs' matrices are fixed
          dense1_muxreg_dispatch<R>(oreg, mreg, a, m, m2);
        } else if (mux >= 0 && lctrl == 0) {
          // mux bit in the thread index: one matrix per thread
          const bool sel = ((rt >> mux) & 1u) != 0;
#pragma unroll
          for (int e = 0; e < 8; ++e) m[e] = sel ? m2[e] : m[e];
          dense1_dispatch<R, false>(oreg, a, m, rt, lr, lctrl);
        } else if (mux >= 0) {
          dense1_mux_dispatch<R, true>(oreg, a, m, m2, rt, lr, lctrl, mux);
        } else if (lctrl) {
          dense1_dispatch<R, true>(oreg, a, m, rt, lr, lctrl);
        } else {
          dense1_dispatch<R, false>(oreg, a, m, rt, lr, lctrl);
        }
      } else if (kind == kOpPhaseBlock) {
        phase_block<T, RB>(
            a,
            reinterpret_cast<const PhaseBlock*>(
                reinterpret_cast<const char*>(op) + op->blob),
            rt, base);
      } else if (kind == kOpPhase) {
        C ph;
        ph.x = m0[0];
        ph.y = m0[1];
        // the index's thread and register parts have disjoint bits
        const uint32_t tm = rt & lctrl;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const bool on = (tm | (lr[j] & lctrl)) == lctrl;
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
          t[e].x = m0[2 * e];
          t[e].y = m0[2 * e + 1];
        }
        // thread parts of the two index bits, once per op
        const uint32_t t0 = d0 >= 0 ? (rt >> (d0 & 31)) & 1u : g0;
        const uint32_t t1 =
            dk > 1 ? (d1 >= 0 ? (rt >> (d1 & 31)) & 1u : g1) : 0u;
        const uint32_t tm = rt & lctrl;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t b0 = d0 >= 0 ? t0 | ((lr[j] >> (d0 & 31)) & 1u) : g0;
          const uint32_t b1 =
              dk > 1 ? (d1 >= 0 ? t1 | ((lr[j] >> (d1 & 31)) & 1u) : g1) : 0u;
          const C f01 = csel(b0 != 0, t[1], t[0]);
          const C f23 = csel(b0 != 0, t[3], t[2]);
          const C f = csel(b1 != 0, f23, f01);
          const bool on = (tm | (lr[j] & lctrl)) == lctrl;
          const C y = cmul(a[j], f);
          a[j] = csel(on, y, a[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j) w[j] = __builtin_bit_cast(W64, a[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) a[j] = __builtin_bit_cast(C, w[j]);
  if (!same_layout(cur, io)) relayout<T, RB>(a, lds, cur, io, tid, active);
}

// Global offsets of a thread's registers in the I/O layout: register j of
// thread tid sits at gthr | (sum over set bits i of j of greg[i]).
template <int RB>
__device__ __forceinline__ void io_offsets(const TilePass* pass, uint64_t base,
                                           uint32_t tid, uint64_t* gthr,
                                           uint64_t* greg) {
  const int W = pass->L - RB;
  uint64_t g = base;
  for (int b = 0; b < W; ++b)
    if (tid >> b & 1) g |= uint64_t(1) << pass->q[b];
  *gthr = g;
#pragma unroll
  for (int i = 0; i < RB; ++i) greg[i] = uint64_t(1) << pass->q[W + i];
}

// I/O addressing with a uniform per-register pointer and a per-thread
// 32-bit byte offset (valid when the thread part of the tile index times
// the amplitude size fits in 32 bits): register j of thread tid is at
// byte  (tile + sum over set bits i of j of 2^q[W+i]) + thread_off.
template <typename C, int RB>
__device__ __forceinline__ uint32_t io_thread_boff(const TilePass* pass,
                                                   uint32_t tid) {
  const int W = pass->L - RB;
  uint32_t o = 0;
  for (int b = 0; b < W; ++b)
    if (tid >> b & 1) o |= 1u << pass->q[b];
  return o * uint32_t(sizeof(C));
}

// Byte offset of register j of the I/O layout within a tile (uniform).
template <typename C, int RB>
__device__ __forceinline__ void io_reg_offsets(const TilePass* pass,
                                               uint64_t* roff) {
  const int W = pass->L - RB;
  roff[0] = 0;
#pragma unroll
  for (int j = 1; j < (1 << RB); ++j) {
    const int i = __builtin_ctz(j);
    roff[j] = roff[j & (j - 1)] + (uint64_t(sizeof(C)) << pass->q[W + i]);
  }
}

template <typename C>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p) {
  // stride 0 (raw), the full 32-bit byte range, gfx9 word-3 layout with a
  // 32-bit data format; offsets used here stay below 2^31
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), short(0),
                                           int(0xffffffffu), 0x00020000);
}

// Element index of a thread's part of the I/O layout (its tile-local
// thread bits spread over the tile qubits).
template <int RB>
__device__ __forceinline__ uint32_t io_thread_index(const TilePass* pass,
                                                    uint32_t tid) {
  const int W = pass->L - RB;
  uint32_t o = 0;
  for (int b = 0; b < W; ++b)
    if (tid >> b & 1) o |= 1u << pass->q[b];
  return o;
}

// Raw buffer loads and stores at a 32-bit byte offset from a uniform buffer
// resource (no per-access 64-bit vector address arithmetic).
__device__ __forceinline__ float2 load_at(const float2*,
                                          __amdgpu_buffer_rsrc_t r,
                                          uint32_t boff) {
  return __builtin_bit_cast(float2,
                            __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}
__device__ __forceinline__ double2 load_at(const double2*,
                                           __amdgpu_buffer_rsrc_t r,
                                           uint32_t boff) {
  return __builtin_bit_cast(double2,
                            __builtin_amdgcn_raw_buffer_load_b128(r, boff, 0, 0));
}
__device__ __forceinline__ void store_at(__amdgpu_buffer_rsrc_t r,
                                         uint32_t boff, float2 v) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, boff, 0, 0);
}
__device__ __forceinline__ void store_at(__amdgpu_buffer_rsrc_t r,
                                         uint32_t boff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r,
                                        boff, 0, 0);
}
__device__ __forceinline__ void store_at(__amdgpu_buffer_rsrc_t r,
                                         uint32_t boff, double v) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, boff, 0,
                                        0);
}
__device__ __forceinline__ void store_at(__amdgpu_buffer_rsrc_t r,
                                         uint32_t boff, double2 v) {
  using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, boff, 0,
                                         0);
}

template <int RB>
__device__ __forceinline__ uint64_t io_addr(uint64_t gthr, const uint64_t* greg,
                                            int j) {
  uint64_t o = gthr;
#pragma unroll
  for (int i = 0; i < RB; ++i)
    if (j >> i & 1) o |= greg[i];
  return o;
}


}  // namespace qsv
