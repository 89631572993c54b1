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

// Pair update (x0, x1) <- M (x0, x1) for a 2x2 complex M = m[0..7]
// (row-major, interleaved), in place: x0 = (a, b), x1 = (c, d).  Each
// output first sums the three terms that do not read its own input (in
// t0..t3, the four chains interleaved), then adds its own term into its own
// register.  Written as one asm block per pair so that the amplitudes stay
// in their registers through every switch arm of an op: compiled code
// computed the new values into fresh registers and copied all sixteen
// amplitudes back at the arms' join (32 moves per op, a fifth of its
// instructions).  SM: the matrix is uniform, in scalar registers (each
// instruction reads one of them); else it is in vector registers.
#define QSV_PAIR_F32(MC)                                                      \
  asm volatile(                                                               \
      "v_mul_f32 %[t0], -%[m1], %[b]\n\t"                                     \
      "v_mul_f32 %[t1], %[m1], %[a]\n\t"                                      \
      "v_mul_f32 %[t2], %[m4], %[a]\n\t"                                      \
      "v_mul_f32 %[t3], %[m4], %[b]\n\t"                                      \
      "v_fmac_f32 %[t0], %[m2], %[c]\n\t"                                     \
      "v_fmac_f32 %[t1], %[m2], %[d]\n\t"                                     \
      "v_fma_f32 %[t2], -%[m5], %[b], %[t2]\n\t"                              \
      "v_fmac_f32 %[t3], %[m5], %[a]\n\t"                                     \
      "v_fma_f32 %[t0], -%[m3], %[d], %[t0]\n\t"                              \
      "v_fmac_f32 %[t1], %[m3], %[c]\n\t"                                     \
      "v_fma_f32 %[t2], -%[m7], %[d], %[t2]\n\t"                              \
      "v_fmac_f32 %[t3], %[m7], %[c]\n\t"                                     \
      "v_fma_f32 %[a], %[m0], %[a], %[t0]\n\t"                                \
      "v_fma_f32 %[b], %[m0], %[b], %[t1]\n\t"                                \
      "v_fma_f32 %[c], %[m6], %[c], %[t2]\n\t"                                \
      "v_fma_f32 %[d], %[m6], %[d], %[t3]"                                     \
      : [a] "+v"(x0.x), [b] "+v"(x0.y), [c] "+v"(x1.x), [d] "+v"(x1.y),     \
        [t0] "=&v"(t0), [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3)        \
      : [m0] MC(m0r), [m1] MC(m0i), [m2] MC(m1r), [m3] MC(m1i),             \
        [m4] MC(m2r), [m5] MC(m2i), [m6] MC(m3r), [m7] MC(m3i))
#define QSV_PAIR_F64(MC)                                                      \
  asm volatile(                                                               \
      "v_mul_f64 %[t0], -%[m1], %[b]\n\t"                                     \
      "v_mul_f64 %[t1], %[m1], %[a]\n\t"                                      \
      "v_mul_f64 %[t2], %[m4], %[a]\n\t"                                      \
      "v_mul_f64 %[t3], %[m4], %[b]\n\t"                                      \
      "v_fma_f64 %[t0], %[m2], %[c], %[t0]\n\t"                               \
      "v_fma_f64 %[t1], %[m2], %[d], %[t1]\n\t"                               \
      "v_fma_f64 %[t2], -%[m5], %[b], %[t2]\n\t"                              \
      "v_fma_f64 %[t3], %[m5], %[a], %[t3]\n\t"                               \
      "v_fma_f64 %[t0], -%[m3], %[d], %[t0]\n\t"                              \
      "v_fma_f64 %[t1], %[m3], %[c], %[t1]\n\t"                               \
      "v_fma_f64 %[t2], -%[m7], %[d], %[t2]\n\t"                              \
      "v_fma_f64 %[t3], %[m7], %[c], %[t3]\n\t"                               \
      "v_fma_f64 %[a], %[m0], %[a], %[t0]\n\t"                                \
      "v_fma_f64 %[b], %[m0], %[b], %[t1]\n\t"                                \
      "v_fma_f64 %[c], %[m6], %[c], %[t2]\n\t"                                \
      "v_fma_f64 %[d], %[m6], %[d], %[t3]"                                     \
      : [a] "+v"(x0.x), [b] "+v"(x0.y), [c] "+v"(x1.x), [d] "+v"(x1.y),     \
        [t0] "=&v"(t0), [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3)        \
      : [m0] MC(m0r), [m1] MC(m0i), [m2] MC(m1r), [m3] MC(m1i),             \
        [m4] MC(m2r), [m5] MC(m2i), [m6] MC(m3r), [m7] MC(m3i))
#define QSV_SREG(x) "s"(x)
#define QSV_VREG(x) "v"(x)

template <bool SM, typename C, typename T>
__device__ __forceinline__ void pair2x2(C& x0, C& x1, T m0r, T m0i, T m1r,
                                        T m1i, T m2r, T m2i, T m3r, T m3i) {
  T t0, t1, t2, t3;
  if constexpr (sizeof(T) == 4) {
    if constexpr (SM) QSV_PAIR_F32(QSV_SREG);
    else QSV_PAIR_F32(QSV_VREG);
  } else {
    if constexpr (SM) QSV_PAIR_F64(QSV_SREG);
    else QSV_PAIR_F64(QSV_VREG);
  }
}

// A 2x2 FP32 matrix for the complex64 pair update, with the negated
// imaginary part of each entry beside it.  Multiplies and two-operand FMAs
// (VOP2 encoding) whose operands are all vector registers issue at twice
// the rate of the same instructions reading a scalar register or carrying
// a negation on this chip, so the cross terms take their factors from
// vector registers: an op copies its uniform matrix there once (six moves,
// four of them 64-bit) and each pair's twelve cross terms run at the
// double rate.  The diagonal
// entries' real parts (m[0], m[6]) feed only the four three-operand FMAs,
// which run at the single rate either way; for a uniform matrix (SM) they
// stay in scalar registers, which keeps the tile kernel at six waves per
// SIMD.
struct VMat32 {
  float m[8];  // as pair2x2's m0r..m3i
  float n[4];  // -m[1], -m[3], -m[5], -m[7]
};

// Two uniform FP32 values into a vector-register pair with one 64-bit move
// (a move from scalar registers costs the same issue time for 64 bits as
// for 32).
__device__ __forceinline__ void vmov2(float lo, float hi, float* vlo,
                                      float* vhi) {
  const uint64_t s = uint64_t(__builtin_bit_cast(uint32_t, lo)) |
                     (uint64_t(__builtin_bit_cast(uint32_t, hi)) << 32);
  uint64_t d;
  asm volatile("v_mov_b64 %0, %1" : "=v"(d) : "s"(s));
  *vlo = __builtin_bit_cast(float, uint32_t(d));
  *vhi = __builtin_bit_cast(float, uint32_t(d >> 32));
}

template <bool SM>
__device__ __forceinline__ VMat32 vmat32(const float* m) {
  VMat32 v;
  if constexpr (SM) {
    // uniform: m[2..5] and the four negations in 64-bit pairs, m[1] and
    // m[7] alone; m[0] and m[6] stay scalar (six moves, not ten)
    v.m[0] = m[0];
    v.m[6] = m[6];
    vmov2(m[2], m[3], &v.m[2], &v.m[3]);
    vmov2(m[4], m[5], &v.m[4], &v.m[5]);
    vmov2(-m[1], -m[3], &v.n[0], &v.n[1]);
    vmov2(-m[5], -m[7], &v.n[2], &v.n[3]);
    v.m[1] = m[1];
    v.m[7] = m[7];
    asm volatile("" : "+v"(v.m[1]), "+v"(v.m[7]));
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      v.m[e] = m[e];
      asm volatile("" : "+v"(v.m[e]));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v.n[k] = -m[2 * k + 1];
      asm volatile("" : "+v"(v.n[k]));
    }
  }
  return v;
}

// The pair update of pair2x2 with the cross-term factors in vector
// registers: the same products and fused sums in the same order (a negated
// factor gives the exactly negated product), so the results are bitwise
// those of pair2x2; the twelve cross terms are VOP2 instructions, the four
// own terms stay three-operand FMAs that write the amplitude registers in
// place.
#define QSV_PAIR_F32V(DC)                                                     \
  asm volatile(                                                               \
      "v_mul_f32_e32 %[t0], %[n0], %[b]\n\t"                                  \
      "v_mul_f32_e32 %[t1], %[m1], %[a]\n\t"                                  \
      "v_mul_f32_e32 %[t2], %[m4], %[a]\n\t"                                  \
      "v_mul_f32_e32 %[t3], %[m4], %[b]\n\t"                                  \
      "v_fmac_f32_e32 %[t0], %[m2], %[c]\n\t"                                 \
      "v_fmac_f32_e32 %[t1], %[m2], %[d]\n\t"                                 \
      "v_fmac_f32_e32 %[t2], %[n2], %[b]\n\t"                                 \
      "v_fmac_f32_e32 %[t3], %[m5], %[a]\n\t"                                 \
      "v_fmac_f32_e32 %[t0], %[n1], %[d]\n\t"                                 \
      "v_fmac_f32_e32 %[t1], %[m3], %[c]\n\t"                                 \
      "v_fmac_f32_e32 %[t2], %[n3], %[d]\n\t"                                 \
      "v_fmac_f32_e32 %[t3], %[m7], %[c]\n\t"                                 \
      "v_fma_f32 %[a], %[m0], %[a], %[t0]\n\t"                                \
      "v_fma_f32 %[b], %[m0], %[b], %[t1]\n\t"                                \
      "v_fma_f32 %[c], %[m6], %[c], %[t2]\n\t"                                \
      "v_fma_f32 %[d], %[m6], %[d], %[t3]"                                     \
      : [a] "+v"(x0.x), [b] "+v"(x0.y), [c] "+v"(x1.x), [d] "+v"(x1.y),     \
        [t0] "=&v"(t0), [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3)        \
      : [m0] DC(v.m[0]), [m1] "v"(v.m[1]), [m2] "v"(v.m[2]),                  \
        [m3] "v"(v.m[3]), [m4] "v"(v.m[4]), [m5] "v"(v.m[5]),                 \
        [m6] DC(v.m[6]), [m7] "v"(v.m[7]), [n0] "v"(v.n[0]),                  \
        [n1] "v"(v.n[1]), [n2] "v"(v.n[2]), [n3] "v"(v.n[3]))

template <bool SM, typename C>
__device__ __forceinline__ void pair2x2v(C& x0, C& x1, const VMat32& v) {
  float t0, t1, t2, t3;
  if constexpr (SM) QSV_PAIR_F32V(QSV_SREG);
  else QSV_PAIR_F32V(QSV_VREG);
}

template <int I, int R, bool CTRL, bool SM, typename C, typename T>
__device__ __forceinline__ void dense1_regs(C* a, const T* m, uint32_t rt,
                                            const uint32_t* lr,
                                            uint32_t lctrl) {
  if constexpr (sizeof(T) == 4) {
    const VMat32 v = vmat32<SM>(m);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j & (1 << I)) continue;
      const int j1 = j | (1 << I);
      if constexpr (CTRL) {
        C y0 = a[j], y1 = a[j1];
        pair2x2v<SM>(y0, y1, v);
        const bool on = ((rt & lctrl) | (lr[j] & lctrl)) == lctrl;
        a[j] = csel(on, y0, a[j]);
        a[j1] = csel(on, y1, a[j1]);
      } else {
        pair2x2v<SM>(a[j], a[j1], v);
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (j & (1 << I)) continue;
    const int j1 = j | (1 << I);
    if constexpr (CTRL) {
      C y0 = a[j], y1 = a[j1];
      pair2x2<SM>(y0, y1, m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7]);
      // rt and lr[j] have disjoint bits: test the thread part once
      const bool on = ((rt & lctrl) | (lr[j] & lctrl)) == lctrl;
      a[j] = csel(on, y0, a[j]);
      a[j1] = csel(on, y1, a[j1]);
    } else {
      pair2x2<SM>(a[j], a[j1], m[0], m[1], m[2], m[3], m[4], m[5], m[6],
                  m[7]);
    }
  }
}

// The same update with the matrix chosen per pair by tile-local bit mbit:
// m0 where the bit is 0, m1 where it is 1 (mbit differs from the target),
// applied only where every bit of lctrl is 1.  Each pair takes both uniform
// matrices in turn and keeps the one its bits select: twice the FMAs of a
// plain op, but the matrices stay in scalar registers (selecting one per
// pair in vector registers set the register peak of the whole kernel, for
// an op class that circuits rarely produce).
template <int I, int R, typename C, typename T>
__device__ __forceinline__ void dense1_mux_regs(C* a, const T* m0,
                                                const T* m1, uint32_t rt,
                                                const uint32_t* lr,
                                                uint32_t lctrl, int mbit) {
  if constexpr (sizeof(T) == 4) {
    // complex64: every pair under m0 (kept where selected), then under m1,
    // with one matrix at a time in vector registers
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const VMat32 v = vmat32<true>(h ? m1 : m0);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (j & (1 << I)) continue;
        const int j1 = j | (1 << I);
        const bool sel = (((rt >> mbit) | (lr[j] >> mbit)) & 1u) != 0;
        const bool on = ((rt & lctrl) | (lr[j] & lctrl)) == lctrl;
        C y0 = a[j], y1 = a[j1];
        pair2x2v<true>(y0, y1, v);
        const bool keep = on && (h ? sel : !sel);
        a[j] = csel(keep, y0, a[j]);
        a[j1] = csel(keep, y1, a[j1]);
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (j & (1 << I)) continue;
    const int j1 = j | (1 << I);
    const bool sel = (((rt >> mbit) | (lr[j] >> mbit)) & 1u) != 0;
    const bool on = ((rt & lctrl) | (lr[j] & lctrl)) == lctrl;
    C y0 = a[j], y1 = a[j1];
    pair2x2<true>(y0, y1, m0[0], m0[1], m0[2], m0[3], m0[4], m0[5], m0[6],
                  m0[7]);
    a[j] = csel(on && !sel, y0, a[j]);
    a[j1] = csel(on && !sel, y1, a[j1]);
    C z0 = a[j], z1 = a[j1];
    pair2x2<true>(z0, z1, m1[0], m1[1], m1[2], m1[3], m1[4], m1[5], m1[6],
                  m1[7]);
    a[j] = csel(on && sel, z0, a[j]);
    a[j1] = csel(on && sel, z1, a[j1]);
  }
}

template <int R, typename C, typename T>
__device__ __forceinline__ void dense1_mux_dispatch(int reg, C* a, const T* m0,
                                                    const T* m1, uint32_t rt,
                                                    const uint32_t* lr,
                                                    uint32_t lctrl, int mbit) {
#define QSV_D1M(I)                                                        \
  case I:                                                                 \
    if constexpr ((1 << I) < R) {                                         \
      dense1_mux_regs<I, R>(a, m0, m1, rt, lr, lctrl, mbit);              \
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
    default:
      __builtin_unreachable();  // the planner emits reg < RB only
  }
#undef QSV_D1M
}

template <int R, bool CTRL, bool SM, typename C, typename T>
__device__ __forceinline__ void dense1_dispatch(int reg, C* a, const T* m,
                                                uint32_t rt, const uint32_t* lr,
                                                uint32_t lctrl) {
#define QSV_D1(I)                                                          \
  case I:                                                                  \
    if constexpr ((1 << I) < R) {                                          \
      dense1_regs<I, R, CTRL, SM>(a, m, rt, lr, lctrl);                    \
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
  if constexpr (sizeof(T) == 4) {
    // complex64: the pairs of m0, then those of m1, one matrix at a time
    // in vector registers
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const VMat32 v = vmat32<true>(h ? m1 : m0);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (j & (1 << I)) continue;
        if ((j >> K & 1) != h) continue;
        pair2x2v<true>(a[j], a[j | (1 << I)], v);
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (j & (1 << I)) continue;
    const int j1 = j | (1 << I);
    const T* m = (j >> K & 1) ? m1 : m0;
    pair2x2<true>(a[j], a[j1], m[0], m[1], m[2], m[3], m[4], m[5], m[6],
                  m[7]);
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

// Work-group barrier for an exchange through LDS.  It waits for this wave's
// LDS (and scalar) accesses only, not for its outstanding global memory
// operations: a streaming tile pass keeps the next tile's prefetch and this
// tile's stores in flight across the exchanges.  The asm is also a compiler
// barrier, so no LDS access moves across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Byte address of a shared-memory pointer in the LDS address space.
template <typename C>
__device__ __forceinline__ uint32_t lds_address(const C* p) {
  return uint32_t(size_t((const __attribute__((address_space(3))) C*)p));
}

// Store and load one complex amplitude at LDS byte address `at` (as a
// two-element vector of its component type).
template <typename C>
__device__ __forceinline__ void lds_store(uint32_t at, const C& v) {
  using E = decltype(v.x);
  typedef E V __attribute__((ext_vector_type(2)));
  V w;
  w.x = v.x;
  w.y = v.y;
  *(__attribute__((address_space(3))) V*)(size_t(at)) = w;
}
template <typename C>
__device__ __forceinline__ void lds_load(uint32_t at, C& v) {
  using E = decltype(v.x);
  typedef E V __attribute__((ext_vector_type(2)));
  const V w = *(const __attribute__((address_space(3))) V*)(size_t(at));
  v.x = w.x;
  v.y = w.y;
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
  // per-thread term and one uniform term per register.  The kernels place
  // no other shared variable before the tile, so it starts at LDS address
  // 0 and each access is one XOR of the two terms; otherwise the base is
  // added (a uniform branch).
  const uint32_t lb = lds_address(lds);
  uint32_t so[R];
  if (active) {
    lds_reg_offsets<T, RB>(from, so);
    const uint32_t rf =
        lds_swz<T>(thread_local_base(from, tid)) * uint32_t(sizeof(C));
    if (lb == 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) lds_store(rf ^ so[j], a[j]);
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) lds_store(lb + (rf ^ so[j]), a[j]);
    }
  }
  lds_barrier();
  if (active) {
    lds_reg_offsets<T, RB>(to, so);
    const uint32_t rt =
        lds_swz<T>(thread_local_base(to, tid)) * uint32_t(sizeof(C));
    if (lb == 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) lds_load(rt ^ so[j], a[j]);
    } else {
#pragma unroll
      for (int j = 0; j < R; ++j) lds_load(lb + (rt ^ so[j]), a[j]);
    }
  }
  lds_barrier();
}

// Re-layout in two halves (the real parts, then the imaginary parts), each
// through a copy of the tile with one component per amplitude: half the
// LDS of relayout(), so that more work-groups fit on a CU, for two more
// barriers and twice the LDS instructions.  4-byte components (complex64)
// take a swizzle over the 32 banks like lds_swz's; 8-byte components
// (complex128) take lds_swz's own 8-byte swizzle.
__device__ __forceinline__ uint32_t lds_swz4(uint32_t r) {
  return r ^ (((r >> 5) ^ (r >> 10)) & 31u);
}

template <typename T>
__device__ __forceinline__ uint32_t half_swz(uint32_t r) {
  if constexpr (sizeof(T) == 4)
    return lds_swz4(r);
  else
    return lds_swz<float>(r);
}

template <typename T, int RB, typename C>
__device__ __forceinline__ void relayout_halves(C* a, C* lds,
                                                const Layout<RB>& from,
                                                const Layout<RB>& to,
                                                uint32_t tid, bool active) {
  constexpr int R = 1 << RB;
  constexpr uint32_t E = sizeof(T);
  uint32_t sf[R], st[R];
  {
    uint32_t bf[RB], bt[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      bf[i] = __builtin_amdgcn_readfirstlane(half_swz<T>(1u << from.rb[i]) * E);
      bt[i] = __builtin_amdgcn_readfirstlane(half_swz<T>(1u << to.rb[i]) * E);
    }
    sf[0] = st[0] = 0;
#pragma unroll
    for (int j = 1; j < R; ++j) {
      sf[j] = sf[j & (j - 1)] ^ bf[__builtin_ctz(j)];
      st[j] = st[j & (j - 1)] ^ bt[__builtin_ctz(j)];
    }
  }
  const uint32_t lb = lds_address(lds);
  const uint32_t rf = lb + half_swz<T>(thread_local_base(from, tid)) * E;
  const uint32_t rt = lb + half_swz<T>(thread_local_base(to, tid)) * E;
  typedef __attribute__((address_space(3))) T lds_t;
  // threads beyond the tile (active == false) only join the barriers
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (active) {
#pragma unroll
      for (int j = 0; j < R; ++j)
        *(lds_t*)(size_t(rf ^ sf[j])) = h ? a[j].y : a[j].x;
    }
    lds_barrier();
    if (active) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const T v = *(const lds_t*)(size_t(rt ^ st[j]));
        if (h) a[j].y = v; else a[j].x = v;
      }
    }
    lds_barrier();
  }
}

// e^{2 pi i t / 2^32} for a fixed-point fraction of a turn, from the
// angle's octant and a Taylor polynomial on [0, pi/4].  The top three bits
// of t give the octant o; the rest, f < 2^29, the angle inside it.  In odd
// octants the polynomial takes the complementary angle pi/4 - x (from
// 2^29 - f), so that its argument stays in [0, pi/4]; then cos and sin of
// the whole angle are those of the octant's reflection:
//   o:   0    1    2    3    4    5    6    7
//   cos  c    s   -s   -c   -c   -s    s    c
//   sin  s    c    c    s   -s   -c   -c   -s
// Truncating sin after x^9 / 9! and cos after x^10 / 10! leaves below 2e-9
// on [0, pi/4], under FP32 rounding.  Few registers: it runs while the
// whole tile is live.
__device__ __forceinline__ float2 turn_phase32(uint32_t t) {
  const uint32_t o = t >> 29;
  const uint32_t f = t & 0x1FFFFFFFu;
  const uint32_t g = (o & 1u) ? 0x20000000u - f : f;
  const float x = float(g) * (6.28318530717958648f * 0x1p-32f);
  const float x2 = x * x;
  float s = __builtin_fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  s = __builtin_fmaf(x2, s, 1.0f / 120.0f);
  s = __builtin_fmaf(x2, s, -1.0f / 6.0f);
  s = __builtin_fmaf(x2 * x, s, x);
  float c = __builtin_fmaf(x2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  c = __builtin_fmaf(x2, c, -1.0f / 720.0f);
  c = __builtin_fmaf(x2, c, 1.0f / 24.0f);
  c = __builtin_fmaf(x2, c, -0.5f);
  c = __builtin_fmaf(x2, c, 1.0f);
  const bool swap = ((o + 1u) >> 1) & 1u;  // octants 1, 2, 5, 6
  const float cv = swap ? s : c, sv = swap ? c : s;
  const bool neg_c = ((o + 2u) >> 2) & 1u;  // octants 2..5
  const bool neg_s = (o >> 2) & 1u;         // octants 4..7
  return make_float2(neg_c ? -cv : cv, neg_s ? -sv : sv);
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
                                            const PhaseBlock* pb_gen,
                                            uint32_t rt, uint64_t base) {
  using C = typename CxT<T>::type;
  using U = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
  constexpr int R = 1 << RB;
  const cptr<PhaseBlock> pb = as_const(pb_gen);
  cptr<PhaseTerm> t = as_const(reinterpret_cast<const PhaseTerm*>(pb_gen + 1));
  U acc[RB + 1];
  // A term's first 16 bytes (outer mask, thread mask, 32-bit turns) are
  // read as one vector, so that each term costs one scalar load round trip.
  auto head = [](cptr<PhaseTerm> p, uint64_t* gm, uint32_t* tm, U* w) {
    const u32x4 h = *(cptr<u32x4>)(p);
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

// The fields of one tile op that the kernels read: its 32-byte header and
// both matrices (FP32 for complex64 states, FP64 for complex128), as raw
// bit patterns, loaded in one batch of scalar loads.
template <typename T>
struct OpFields {
  using B = std::conditional_t<sizeof(T) == 4, uint32_t, uint64_t>;
  int32_t code, arg;
  uint32_t lctrl;
  int32_t blob;
  uint64_t gctrl;
  int32_t dbit0, dbit1;
  B m0[8], m1[8];
};

template <typename T>
__device__ __forceinline__ OpFields<T> load_op(const TileOp* op) {
  OpFields<T> f;
  const cptr<u32x4> h = as_const(reinterpret_cast<const u32x4*>(op));
  const u32x4 h0 = h[0], h1 = h[1];
  f.code = int32_t(h0.x);
  f.arg = int32_t(h0.y);
  f.lctrl = h0.z;
  f.blob = int32_t(h0.w);
  f.gctrl = uint64_t(h1.x) | (uint64_t(h1.y) << 32);
  f.dbit0 = int32_t(h1.z);
  f.dbit1 = int32_t(h1.w);
  if constexpr (sizeof(T) == 4) {
    const cptr<u32x4> mv = as_const(reinterpret_cast<const u32x4*>(op->mf));
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const u32x4 u = mv[i], v = mv[2 + i];
      f.m0[4 * i] = u.x; f.m0[4 * i + 1] = u.y;
      f.m0[4 * i + 2] = u.z; f.m0[4 * i + 3] = u.w;
      f.m1[4 * i] = v.x; f.m1[4 * i + 1] = v.y;
      f.m1[4 * i + 2] = v.z; f.m1[4 * i + 3] = v.w;
    }
  } else {
    const cptr<u32x4> mv = as_const(reinterpret_cast<const u32x4*>(op->m));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const u32x4 u = mv[i], v = mv[4 + i];
      f.m0[2 * i] = uint64_t(u.x) | (uint64_t(u.y) << 32);
      f.m0[2 * i + 1] = uint64_t(u.z) | (uint64_t(u.w) << 32);
      f.m1[2 * i] = uint64_t(v.x) | (uint64_t(v.y) << 32);
      f.m1[2 * i + 1] = uint64_t(v.z) | (uint64_t(v.w) << 32);
    }
  }
  return f;
}

// Every field of an op is live in scalar registers from here on: without
// this the compiler sinks each load to its first use, and the op waits for
// several dependent rounds of scalar loads instead of one.
template <typename T>
__device__ __forceinline__ void pin_op_fields(OpFields<T>& f) {
  asm volatile("" : "+s"(f.code), "+s"(f.arg), "+s"(f.lctrl), "+s"(f.blob),
                    "+s"(f.gctrl), "+s"(f.dbit0), "+s"(f.dbit1));
#pragma unroll
  for (int e = 0; e < 8; ++e) asm volatile("" : "+s"(f.m0[e]), "+s"(f.m1[e]));
}

// Apply every segment of one tile pass to the register tile `a`, which is
// in the I/O layout on entry and is left in the I/O layout on exit.  `base`
// is the tile's global index with all tile bits zero (outer controls and
// diagonal bits outside the tile are read from it).
template <typename T, int RB, bool HALVES = false>
__device__ __forceinline__ void tile_apply(typename CxT<T>::type* a,
                                           typename CxT<T>::type* lds,
                                           const TilePass* pass,
                                           const TileSeg* segs,
                                           const TileOp* ops, uint64_t base,
                                           uint32_t tid, bool active) {
  using C = typename CxT<T>::type;
  using Bits = typename OpFields<T>::B;
  constexpr int R = 1 << RB;
  const cptr<TilePass> cp = as_const(pass);
  const int W = cp->L - RB;
  Layout<RB> io;
#pragma unroll
  for (int i = 0; i < RB; ++i) io.rb[i] = W + i;
  Layout<RB> cur = io;
  const int nseg = cp->nseg;
  const cptr<TileSeg> sp = as_const(segs) + cp->seg_begin;
  for (int s = 0; s < nseg; ++s) {
    Layout<RB> lay;
#pragma unroll
    for (int i = 0; i < RB; ++i) lay.rb[i] = sp[s].reg_bits[i];
    if (!same_layout(cur, lay)) {
      if constexpr (HALVES)
        relayout_halves<T, RB>(a, lds, cur, lay, tid, active);
      else
        relayout<T, RB>(a, lds, cur, lay, tid, active);
    }
    cur = lay;
    const uint32_t rt = thread_local_base(lay, tid);
    const int o_end = sp[s].op_end;
    int o = sp[s].op_begin;
    while (o < o_end) {
      // Runs of control-free dense ops (the bulk of every circuit) go
      // through a tight loop that branches only on the class and the
      // target register, and whose every arm updates the amplitudes in
      // place; controlled, phase and diagonal ops take the general path.
      const TileOp* op = ops + o;
      // the header and both matrices, in one batch of scalar loads; the
      // planner resolved every choice it could into the dispatch code
      OpFields<T> f = load_op<T>(op);
      pin_op_fields(f);
      int cls = f.code >> 3;
      if (cls <= kCodeThreadMux) {
        for (;;) {
          if ((base & f.gctrl) == f.gctrl) {  // else an outer control is 0
            const int reg = f.code & 7;
            if (cls == kCodeUniform) {
              // one matrix for the whole tile, chosen by one bit of its
              // base index (an outer mux qubit, or bit 63, which no index
              // has); the choice is made on the bit patterns, so it stays
              // scalar and the FMAs read the matrix from scalar registers
              const bool second = ((base >> (f.arg & 63)) & 1) != 0;
              T m[8];
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                Bits b = second ? f.m1[e] : f.m0[e];
                asm volatile("" : "+s"(b));
                m[e] = __builtin_bit_cast(T, b);
              }
              dense1_dispatch<R, false, true>(reg, a, m, rt, nullptr, 0u);
            } else {
              T m0[8], m1[8];
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                m0[e] = __builtin_bit_cast(T, f.m0[e]);
                m1[e] = __builtin_bit_cast(T, f.m1[e]);
              }
              if (cls == kCodeRegMux) {
                // mux bit in a register: the pairs' matrices are fixed
                dense1_muxreg_dispatch<R>(reg, f.arg, a, m0, m1);
              } else {
                // mux bit in the thread index: one matrix per thread
                const bool sel = ((rt >> f.arg) & 1u) != 0;
                T m[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) m[e] = sel ? m1[e] : m0[e];
                dense1_dispatch<R, false, false>(reg, a, m, rt, nullptr, 0u);
              }
            }
          }
          if (++o >= o_end) break;
          f = load_op<T>(ops + o);
          pin_op_fields(f);
          cls = f.code >> 3;
          if (cls > kCodeThreadMux) break;
        }
        continue;  // o is the next op of another class, or the end
      }
      ++o;
      if ((base & f.gctrl) != f.gctrl) continue;  // an outer control is 0
      const int reg = f.code & 7;
      T m0[8], m1[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        m0[e] = __builtin_bit_cast(T, f.m0[e]);
        m1[e] = __builtin_bit_cast(T, f.m1[e]);
      }
      uint32_t lr[R];
#pragma unroll
      for (int j = 0; j < R; ++j) lr[j] = reg_offset(lay, j);
      if (cls == kCodeCtrl) {
        const bool second = ((base >> (f.arg & 63)) & 1) != 0;
        T m[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) m[e] = second ? m1[e] : m0[e];
        dense1_dispatch<R, true, false>(reg, a, m, rt, lr, f.lctrl);
      } else if (cls == kCodeCtrlMux) {
        dense1_mux_dispatch<R>(reg, a, m0, m1, rt, lr, f.lctrl, f.arg);
      } else if (cls == kCodePhaseBlock) {
        phase_block<T, RB>(
            a,
            reinterpret_cast<const PhaseBlock*>(
                reinterpret_cast<const char*>(op) + f.blob),
            rt, base);
      } else if (cls == kCodePhase) {
        C ph;
        ph.x = m0[0];
        ph.y = m0[1];
        // the index's thread and register parts have disjoint bits
        const uint32_t tm = rt & f.lctrl;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const bool on = (tm | (lr[j] & f.lctrl)) == f.lctrl;
          const C y = cmul(a[j], ph);
          a[j] = csel(on, y, a[j]);
        }
      } else {  // kCodeDiag
        const int dk = f.arg;
        const int d0 = f.dbit0, d1 = f.dbit1;
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
        const uint32_t tm = rt & f.lctrl;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t b0 = d0 >= 0 ? t0 | ((lr[j] >> (d0 & 31)) & 1u) : g0;
          const uint32_t b1 =
              dk > 1 ? (d1 >= 0 ? t1 | ((lr[j] >> (d1 & 31)) & 1u) : g1) : 0u;
          const C f01 = csel(b0 != 0, t[1], t[0]);
          const C f23 = csel(b0 != 0, t[3], t[2]);
          const C fv = csel(b1 != 0, f23, f01);
          const bool on = (tm | (lr[j] & f.lctrl)) == f.lctrl;
          const C y = cmul(a[j], fv);
          a[j] = csel(on, y, a[j]);
        }
      }
    }
  }
  if (!same_layout(cur, io)) {
    if constexpr (HALVES)
      relayout_halves<T, RB>(a, lds, cur, io, tid, active);
    else
      relayout<T, RB>(a, lds, cur, io, tid, active);
  }
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
