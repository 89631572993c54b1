// Fused k-qubit blocks.
//
// Build: the product of a block's gates, each embedded in 2^k dimensions, is
// formed in FP64 on the device (one work-group per block, the 2^k x 2^k
// matrix in LDS, every gate applied to all of its columns), then rounded once
// to FP32 for complex64 states.
//
// Apply: a'[group] = U a[group] over the 2^(n-k) groups is a complex GEMM
// [2^k x 2^k] x [2^k x 2^(n-k)].  For k >= 4 it runs on the matrix cores
// through the real embedding M = [[Re U, -Im U], [Im U, Re U]] (a
// 2^(k+1)-square real matrix): FP32 MFMA 32x32x2 for complex64, FP64 MFMA
// 16x16x4 for complex128.  Each wave owns a batch of groups (one group per
// MFMA column); a lane loads the amplitudes of its group whose index is
// congruent to its lane half (c64) or quarter (c128), which are exactly the
// B-operand values it supplies, and M stays in registers as A operands.
// k <= 3 blocks use the plain dense VALU kernel with the FP64 product.
#include "device_common.h"

namespace qsv {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ build

__global__ void __launch_bounds__(256)
    fused_build_kernel(const FusedBlock* __restrict__ blocks,
                       const FusedGate* __restrict__ gates,
                       double* __restrict__ mats64,
                       float* __restrict__ mats32) {
  __shared__ double2 U[32 * 32];
  const FusedBlock blk = blocks[blockIdx.x];
  const int k = blk.k;
  const int D = 1 << k;
  for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
    const int r = e / D, c = e % D;
    U[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int gi = 0; gi < blk.n_gates; ++gi) {
    const FusedGate g = gates[blk.gate_begin + gi];
    const double* m = mats64 + g.m_offset;
    const int gd = 1 << g.k;
    int cmask = 0, fixed = 0;
    for (int j = 0; j < g.c; ++j) cmask |= 1 << g.ctl[j];
    fixed = cmask;
    for (int j = 0; j < g.k; ++j) fixed |= 1 << g.t[j];
    const int nfree = k - g.k - g.c;
    const int items = D << nfree;  // (column, coset) pairs
    // Each item updates 2^gk entries of one column; gather first, then
    // write after a barrier so that no item reads another's output.
    double2 res[32];
    int rows[32];
    int nres = 0;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
      const int col = it >> nfree;
      int base = it & ((1 << nfree) - 1);
      for (int b = 0; b < k; ++b)
        if (fixed >> b & 1) {
          const int lo = base & ((1 << b) - 1);
          base = ((base >> b) << (b + 1)) | lo;
        }
      base |= cmask;
      for (int r = 0; r < gd; ++r) {
        int rr = base;
        for (int j = 0; j < g.k; ++j)
          if (r >> j & 1) rr |= 1 << g.t[j];
        double re = 0, im = 0;
        for (int s = 0; s < gd; ++s) {
          int ss = base;
          for (int j = 0; j < g.k; ++j)
            if (s >> j & 1) ss |= 1 << g.t[j];
          const double2 v = U[ss * D + col];
          const double mr = m[2 * (r * gd + s)], mi = m[2 * (r * gd + s) + 1];
          re += mr * v.x - mi * v.y;
          im += mr * v.y + mi * v.x;
        }
        if (nres < 32) {
          res[nres] = make_double2(re, im);
          rows[nres] = rr * D + col;
          ++nres;
        }
      }
    }
    __syncthreads();
    for (int e = 0; e < nres; ++e) U[rows[e]] = res[e];
    __syncthreads();
  }
  for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
    const double2 v = U[e];
    mats64[blk.u64_offset + 2 * e] = v.x;
    mats64[blk.u64_offset + 2 * e + 1] = v.y;
    mats32[blk.u32_offset + 2 * e] = float(v.x);
    mats32[blk.u32_offset + 2 * e + 1] = float(v.y);
  }
}

hipError_t launch_fused_build(const FusedBlock* blocks, int n_blocks,
                              const FusedGate* gates, double* mats64,
                              float* mats32, hipStream_t stream) {
  if (n_blocks <= 0) return hipSuccess;
  fused_build_kernel<<<n_blocks, 256, 0, stream>>>(blocks, gates, mats64,
                                                   mats32);
  return hipGetLastError();
}

// ------------------------------------------------------------------ apply

struct FusedArgs {
  uint64_t n_groups;
  int32_t k;
  int32_t pad;
  int32_t q[8];  // block qubits, ascending; local bit j <-> q[j]
};

__device__ __forceinline__ uint64_t deposit_bits(uint32_t s, const int32_t* q,
                                                 int k) {
  uint64_t o = 0;
  for (int j = 0; j < k; ++j)
    if (s >> j & 1) o |= uint64_t(1) << q[j];
  return o;
}

// Complex64, k = 4 or 5: FP32 MFMA 32x32x2.  Per wave: 32 groups (MFMA
// columns); lane l = 32 h + j holds group j and the amplitudes s = 2 e + h.
// K index of step st: part = st / E (0: real, 1: imaginary), e = st % E.
template <int K>
__global__ void __launch_bounds__(256)
    fused_mfma_c64_kernel(float2* __restrict__ amp, FusedArgs args,
                          const float* __restrict__ u) {
  constexpr int D = 1 << K;        // matrix dimension
  constexpr int E = D / 2;         // amplitudes per lane
  constexpr int NS = 2 * E;        // MFMA steps (K dim = 2 D, 2 per step)
  constexpr int NT = (2 * D) / 32; // row tiles of 32
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int i = lane & 31;  // A row within tile / B, D column (group)

  // A operands: M[row][col] with row R = 32 T + i, col (part, s = 2 e + h).
  float A[NT][NS];
#pragma unroll
  for (int T = 0; T < NT; ++T) {
    const int R = 32 * T + i;
    const bool re_row = R < D;
    const int r = re_row ? R : R - D;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int part = st / E;
      const int s = 2 * (st % E) + h;
      const float ur = u[2 * (r * D + s)], ui = u[2 * (r * D + s) + 1];
      A[T][st] = re_row ? (part == 0 ? ur : -ui) : (part == 0 ? ui : ur);
    }
  }
  uint64_t in_off[E];
#pragma unroll
  for (int e = 0; e < E; ++e) in_off[e] = deposit_bits(2 * e + h, args.q, K);
  // Output rows held by this lane: i(v) = 8 (v / 4) + 4 h + v % 4 in each
  // row tile.  Real row r and imaginary row r + D of output r sit in tiles
  // T and T + NT/2 (k = 5), or in registers v and v + 8 of the single tile
  // (k = 4, where i(v + 8) = i(v) + 16 = i(v) + D).
  constexpr int OUT_T = NT >= 2 ? NT / 2 : 1;
  constexpr int OUT_V = NT >= 2 ? 16 : 8;
  uint64_t out_off[OUT_T][OUT_V];
#pragma unroll
  for (int T = 0; T < OUT_T; ++T)
#pragma unroll
    for (int v = 0; v < OUT_V; ++v)
      out_off[T][v] =
          deposit_bits(32 * T + 8 * (v / 4) + 4 * h + (v % 4), args.q, K);

  const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  for (uint64_t g0 = wave * 32; g0 < args.n_groups; g0 += nwaves * 32) {
    const uint64_t gidx = g0 + i;
    const bool valid = gidx < args.n_groups;
    uint64_t base = valid ? gidx : 0;
    for (int j = 0; j < K; ++j) base = insert_zero64(base, args.q[j]);
    float2 x[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
      x[e] = valid ? amp[base + in_off[e]] : make_float2(0.f, 0.f);
    floatx16 acc[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[T][v] = 0.f;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const float b = (st < E) ? x[st % E].x : x[st % E].y;
#pragma unroll
      for (int T = 0; T < NT; ++T)
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[T][st], b, acc[T], 0,
                                                      0, 0);
    }
    if (valid) {
#pragma unroll
      for (int T = 0; T < OUT_T; ++T)
#pragma unroll
        for (int v = 0; v < OUT_V; ++v) {
          if constexpr (NT >= 2)
            amp[base + out_off[T][v]] =
                make_float2(acc[T][v], acc[T + OUT_T][v]);
          else
            amp[base + out_off[T][v]] = make_float2(acc[0][v], acc[0][v + 8]);
        }
    }
  }
}

// Complex128, k = 4 or 5: FP64 MFMA 16x16x4.  Per wave: 16 groups; lane
// l = 16 h + j holds group j and the amplitudes s = 4 e + h.  Operand
// layout: A[i = l % 16][k = l / 16], B[k = l / 16][j = l % 16]; the result
// D[i][j] sits in lane 16 (i % 4) + j, register i / 4.
template <int K>
__global__ void __launch_bounds__(256)
    fused_mfma_c128_kernel(double2* __restrict__ amp, FusedArgs args,
                           const double* __restrict__ u) {
  constexpr int D = 1 << K;
  constexpr int E = D / 4;
  constexpr int NS = 2 * E;
  constexpr int NT = (2 * D) / 16;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 4;
  const int i = lane & 15;

  double A[NT][NS];
#pragma unroll
  for (int T = 0; T < NT; ++T) {
    const int R = 16 * T + i;
    const bool re_row = R < D;
    const int r = re_row ? R : R - D;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int part = st / E;
      const int s = 4 * (st % E) + h;
      const double ur = u[2 * (r * D + s)], ui = u[2 * (r * D + s) + 1];
      A[T][st] = re_row ? (part == 0 ? ur : -ui) : (part == 0 ? ui : ur);
    }
  }
  uint64_t in_off[E];
#pragma unroll
  for (int e = 0; e < E; ++e) in_off[e] = deposit_bits(4 * e + h, args.q, K);
  // Result register v of lane (h, j) holds row h + 4 v of its tile.
  constexpr int OUT_T = NT / 2;
  uint64_t out_off[OUT_T][4];
#pragma unroll
  for (int T = 0; T < OUT_T; ++T)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      out_off[T][v] = deposit_bits(16 * T + h + 4 * v, args.q, K);

  const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  for (uint64_t g0 = wave * 16; g0 < args.n_groups; g0 += nwaves * 16) {
    const uint64_t gidx = g0 + i;
    const bool valid = gidx < args.n_groups;
    uint64_t base = valid ? gidx : 0;
    for (int j = 0; j < K; ++j) base = insert_zero64(base, args.q[j]);
    double2 x[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
      x[e] = valid ? amp[base + in_off[e]] : make_double2(0.0, 0.0);
    doublex4 acc[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[T][v] = 0.0;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const double b = (st < E) ? x[st % E].x : x[st % E].y;
#pragma unroll
      for (int T = 0; T < NT; ++T)
        acc[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[T][st], b, acc[T], 0,
                                                      0, 0);
    }
    if (valid) {
#pragma unroll
      for (int T = 0; T < OUT_T; ++T)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          amp[base + out_off[T][v]] =
              make_double2(acc[T][v], acc[T + OUT_T][v]);
    }
  }
}

hipError_t launch_dense_dev(int prec, void* amp, int n, int k,
                            const int32_t* q, const double* dev_matrix,
                            hipStream_t stream);

hipError_t launch_fused_apply(int prec, void* amp, int n, int k,
                              const int32_t* q, const void* u,
                              hipStream_t stream) {
  if (k <= 3)
    return launch_dense_dev(prec, amp, n, k, q,
                            static_cast<const double*>(u), stream);
  FusedArgs args = {};
  args.n_groups = uint64_t(1) << (n - k);
  args.k = k;
  for (int j = 0; j < k; ++j) args.q[j] = q[j];
  const uint64_t per_wave = prec == 1 ? 32 : 16;
  const uint64_t waves = (args.n_groups + per_wave - 1) / per_wave;
  const unsigned blocks = grid_blocks(waves * 64, 256, 1u << 16);
  if (prec == 1) {
    float2* a = static_cast<float2*>(amp);
    const float* m = static_cast<const float*>(u);
    if (k == 4)
      fused_mfma_c64_kernel<4><<<blocks, 256, 0, stream>>>(a, args, m);
    else
      fused_mfma_c64_kernel<5><<<blocks, 256, 0, stream>>>(a, args, m);
  } else {
    double2* a = static_cast<double2*>(amp);
    const double* m = static_cast<const double*>(u);
    if (k == 4)
      fused_mfma_c128_kernel<4><<<blocks, 256, 0, stream>>>(a, args, m);
    else
      fused_mfma_c128_kernel<5><<<blocks, 256, 0, stream>>>(a, args, m);
  }
  return hipGetLastError();
}

}  // namespace qsv
