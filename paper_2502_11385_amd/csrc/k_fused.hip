// Fused k-qubit blocks.
//
// Build: the product of a block's gates, each embedded in 2^k dimensions, is
// formed in FP64 on the device (one work-group per block, the 2^k x 2^k
// matrix in LDS, every gate applied to all of its columns, each entry of
// the new product computed from the previous one), then rounded once to
// FP32 for complex64 states.
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
#include <mutex>

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
  // U <- G U for each gate G in order: entry (row, col) of the new product
  // is the gate's row r (the row's target bits) times the old column over
  // the rows that differ from `row` in target bits only; rows whose
  // control bits are not all 1 are unchanged.  Two LDS copies alternate,
  // so every thread reads only the old product.
  __shared__ double2 Ubuf[2][32 * 32];
  const FusedBlock blk = blocks[blockIdx.x];
  const int k = blk.k;
  const int D = 1 << k;
  double2* Uo = Ubuf[0];
  double2* Un = Ubuf[1];
  for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
    const int r = e / D, c = e % D;
    Uo[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int gi = 0; gi < blk.n_gates; ++gi) {
    // by reference: the target and control lists are indexed at run time
    // and read from memory, not copied into a private array
    const FusedGate& g = gates[blk.gate_begin + gi];
    const double* m = mats64 + g.m_offset;
    const int gd = 1 << g.k;
    int cmask = 0, tmask = 0;
    for (int j = 0; j < g.c; ++j) cmask |= 1 << g.ctl[j];
    for (int j = 0; j < g.k; ++j) tmask |= 1 << g.t[j];
    for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
      const int row = e / D, col = e % D;
      if ((row & cmask) != cmask) {
        Un[e] = Uo[e];
        continue;
      }
      int r = 0;
      for (int j = 0; j < g.k; ++j) r |= ((row >> g.t[j]) & 1) << j;
      const int rest = row & ~tmask;
      double re = 0, im = 0;
      for (int sidx = 0; sidx < gd; ++sidx) {
        int rs = rest;
        for (int j = 0; j < g.k; ++j)
          if (sidx >> j & 1) rs |= 1 << g.t[j];
        const double2 v = Uo[rs * D + col];
        const double mr = m[2 * (r * gd + sidx)];
        const double mi = m[2 * (r * gd + sidx) + 1];
        re += mr * v.x - mi * v.y;
        im += mr * v.y + mi * v.x;
      }
      Un[e] = make_double2(re, im);
    }
    __syncthreads();
    double2* t = Uo;
    Uo = Un;
    Un = t;
  }
  for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
    const double2 v = Uo[e];
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
  uint64_t cmask;     // control qubits, set in every group base
  int32_t k;
  int32_t nfixed;     // block and control qubits
  int32_t q[8];       // block qubits, ascending; local bit j <-> q[j]
  int32_t fixed[34];  // block and control qubits, ascending
};

// Group base of group index g: zeros inserted at the block and control
// qubits, then the control qubits set.
__device__ __forceinline__ uint64_t group_base(uint64_t g,
                                               const FusedArgs& args) {
  for (int j = 0; j < args.nfixed; ++j) g = insert_zero64(g, args.fixed[j]);
  return g | args.cmask;
}

__device__ __forceinline__ uint64_t deposit_bits(uint32_t s, const int32_t* q,
                                                 int k) {
  uint64_t o = 0;
  for (int j = 0; j < k; ++j)
    if (s >> j & 1) o |= uint64_t(1) << q[j];
  return o;
}

// The real embedding's imaginary rows repeat its real rows: row D + r of
// M is (Im U[r], Re U[r]) and row r is (Re U[r], -Im U[r]).  So the
// imaginary half of the product is M's real rows times the permuted,
// negated operand (Im a, -Re a); where the real and imaginary rows fall in
// different row tiles, only the real rows' A operands are kept and each is
// fed with both operand orders.  The A operands live in LDS, read per
// step, so that the registers hold only amplitudes and accumulators.
//
// Offsets: an amplitude's index is its group base plus the deposit of its
// block-local index s onto the block qubits.  s splits into a part shared
// by the wave (uniform, scalar registers) and the lane's own bits, so a
// lane adds one per-lane term to its base and one uniform term per load.

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
  constexpr bool SYM = NT >= 2;    // imaginary rows in their own tiles
  constexpr int AT = SYM ? NT / 2 : NT;  // row tiles whose A a lane holds
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int i = lane & 31;  // A row within tile / B, D column (group)

  // A operands M[row][col], row R = 32 T + i, col (part, s = 2 e + h),
  // staged in LDS in the order the lanes read them (step, half, row), so
  // that they take no registers across the loop and a step's read is two
  // 128-byte runs.
  __shared__ float Ms[NS * 2 * AT * 32];
  for (int idx = threadIdx.x; idx < NS * 2 * AT * 32; idx += blockDim.x) {
    const int R = idx % (AT * 32);
    const int hh = (idx / (AT * 32)) % 2;
    const int st = idx / (AT * 64);
    const bool re_row = R < D;
    const int r = re_row ? R : R - D;
    const int part = st / E;
    const int s = 2 * (st % E) + hh;
    const float ur = u[2 * (r * D + s)], ui = u[2 * (r * D + s) + 1];
    Ms[idx] = re_row ? (part == 0 ? ur : -ui) : (part == 0 ? ui : ur);
  }
  __syncthreads();
  const float* Ml = Ms + h * (AT * 32) + i;  // + st * AT * 64 + 32 T
  // lane terms: s = 2 e + h puts h on block bit 0; output rows
  // i(v) = 8 (v / 4) + 4 h + v % 4 put h on block bit 2
  const uint64_t in_lane = uint64_t(h) << args.q[0];
  const uint64_t out_lane = uint64_t(h) << args.q[2];
  // Output rows held by this lane: i(v) in each row tile.  Real row r and
  // imaginary row r + D of output r sit in tiles T and T + NT/2 (k = 5), or
  // in registers v and v + 8 of the single tile (k = 4, where
  // i(v + 8) = i(v) + 16 = i(v) + D).
  constexpr int OUT_T = NT >= 2 ? NT / 2 : 1;
  constexpr int OUT_V = NT >= 2 ? 16 : 8;

  const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  // rows r and r + 1 (r even) of an output are adjacent amplitudes when the
  // block's lowest qubit is qubit 0: then a lane stores both as one 16-byte
  // write, so each store instruction writes whole runs
  const bool pair_store = args.q[0] == 0;
  for (uint64_t g0 = wave * 32; g0 < args.n_groups; g0 += nwaves * 32) {
    // reload the A operands every batch rather than keep them in registers
    asm volatile("" ::: "memory");
    // a lane past the last group reads the last group (in bounds, so the
    // loads need no mask) and stores nothing
    const uint64_t gidx = g0 + i;
    const bool valid = gidx < args.n_groups;
    const uint64_t base = group_base(valid ? gidx : args.n_groups - 1, args);
    float2 x[E];
    const uint64_t in_base = base + in_lane;
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = amp[in_base + deposit_bits(2 * e, args.q, K)];
    floatx16 acc[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[T][v] = 0.f;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const float b = (st < E) ? x[st % E].x : x[st % E].y;
#pragma unroll
      for (int T = 0; T < AT; ++T) {
        const float a = Ml[st * AT * 64 + 32 * T];
        acc[T] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[T], 0, 0, 0);
        if constexpr (SYM) {
          const float b2 = (st < E) ? x[st % E].y : -x[st % E].x;
          acc[AT + T] = __builtin_amdgcn_mfma_f32_32x32x2f32(
              a, b2, acc[AT + T], 0, 0, 0);
        }
      }
    }
    if (valid) {
      const uint64_t out_base = base + out_lane;
      auto re = [&](int T, int v) {
        return NT >= 2 ? acc[T][v] : acc[0][v];
      };
      auto im = [&](int T, int v) {
        return NT >= 2 ? acc[T + OUT_T][v] : acc[0][v + 8];
      };
      if (pair_store) {
#pragma unroll
        for (int T = 0; T < OUT_T; ++T)
#pragma unroll
          for (int v = 0; v < OUT_V; v += 2) {
            const uint64_t o = out_base + deposit_bits(
                32 * T + 8 * (v / 4) + (v % 4), args.q, K);
            *reinterpret_cast<float4*>(amp + o) =
                make_float4(re(T, v), im(T, v), re(T, v + 1), im(T, v + 1));
          }
      } else {
#pragma unroll
        for (int T = 0; T < OUT_T; ++T)
#pragma unroll
          for (int v = 0; v < OUT_V; ++v) {
            const uint64_t o = out_base + deposit_bits(
                32 * T + 8 * (v / 4) + (v % 4), args.q, K);
            amp[o] = make_float2(re(T, v), im(T, v));
          }
      }
    }
  }
}

// Complex128, k = 4 or 5: FP64 MFMA 16x16x4.  Per wave: 16 groups; lane
// l = 16 h + j holds group j and the amplitudes s = 4 e + h.  Operand
// layout: A[i = l % 16][k = l / 16], B[k = l / 16][j = l % 16]; the result
// D[i][j] sits in lane 16 (i % 4) + j, register i / 4.  The real rows fill
// the first NT / 2 row tiles, so a lane holds only their A operands.
template <int K>
__global__ void __launch_bounds__(256)
    fused_mfma_c128_kernel(double2* __restrict__ amp, FusedArgs args,
                           const double* __restrict__ u) {
  constexpr int D = 1 << K;
  constexpr int E = D / 4;
  constexpr int NS = 2 * E;
  constexpr int NT = (2 * D) / 16;
  constexpr int AT = NT / 2;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 4;
  const int i = lane & 15;

  // A operands of the real rows, staged in LDS in lane read order (step,
  // quarter, row).
  __shared__ double Ms[NS * 4 * AT * 16];
  for (int idx = threadIdx.x; idx < NS * 4 * AT * 16; idx += blockDim.x) {
    const int r = idx % (AT * 16);  // a real row
    const int hh = (idx / (AT * 16)) % 4;
    const int st = idx / (AT * 64);
    const int part = st / E;
    const int s = 4 * (st % E) + hh;
    const double ur = u[2 * (r * D + s)], ui = u[2 * (r * D + s) + 1];
    Ms[idx] = part == 0 ? ur : -ui;
  }
  __syncthreads();
  const double* Ml = Ms + h * (AT * 16) + i;  // + st * AT * 64 + 16 T
  // lane terms: s = 4 e + h puts h on block bits 0-1; output row h + 4 v
  // of a tile puts it there too
  const uint64_t lane_off = (uint64_t(h & 1) << args.q[0]) |
                            (uint64_t(h >> 1) << args.q[1]);
  constexpr int OUT_T = NT / 2;

  const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
  for (uint64_t g0 = wave * 16; g0 < args.n_groups; g0 += nwaves * 16) {
    // reload the A operands every batch rather than keep them in registers
    asm volatile("" ::: "memory");
    // a lane past the last group reads the last group and stores nothing
    const uint64_t gidx = g0 + i;
    const bool valid = gidx < args.n_groups;
    const uint64_t base = group_base(valid ? gidx : args.n_groups - 1, args);
    const uint64_t lbase = base + lane_off;
    double2 x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = amp[lbase + deposit_bits(4 * e, args.q, K)];
    doublex4 acc[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[T][v] = 0.0;
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const double b = (st < E) ? x[st % E].x : x[st % E].y;
      const double b2 = (st < E) ? x[st % E].y : -x[st % E].x;
#pragma unroll
      for (int T = 0; T < AT; ++T) {
        const double a = Ml[st * AT * 64 + 16 * T];
        acc[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[T], 0, 0, 0);
        acc[AT + T] = __builtin_amdgcn_mfma_f64_16x16x4f64(
            a, b2, acc[AT + T], 0, 0, 0);
      }
    }
    if (valid) {
#pragma unroll
      for (int T = 0; T < OUT_T; ++T)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          amp[lbase + deposit_bits(16 * T + 4 * v, args.q, K)] =
              make_double2(acc[T][v], acc[T + OUT_T][v]);
    }
  }
}

// Work-groups of 256 threads the fused kernel for (prec, k) keeps resident
// on the whole device (looked up once; 2^16 if the query fails).
static unsigned fused_resident_blocks(int prec, int k) {
  static std::once_flag once;
  static unsigned res[2][2] = {{1u << 16, 1u << 16}, {1u << 16, 1u << 16}};
  std::call_once(once, [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess || cus <= 0) {
      (void)hipGetLastError();
      return;
    }
    const void* fns[2][2] = {
        {reinterpret_cast<const void*>(&fused_mfma_c64_kernel<4>),
         reinterpret_cast<const void*>(&fused_mfma_c64_kernel<5>)},
        {reinterpret_cast<const void*>(&fused_mfma_c128_kernel<4>),
         reinterpret_cast<const void*>(&fused_mfma_c128_kernel<5>)}};
    for (int p = 0; p < 2; ++p)
      for (int j = 0; j < 2; ++j) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fns[p][j], 256,
                                                         0) != hipSuccess ||
            b <= 0) {
          (void)hipGetLastError();
          continue;
        }
        res[p][j] = unsigned(b) * unsigned(cus);
      }
  });
  return res[prec == 1 ? 0 : 1][k == 4 ? 0 : 1];
}

hipError_t launch_dense_dev(int prec, void* amp, int n, int k,
                            const int32_t* q, const double* dev_matrix,
                            hipStream_t stream);

hipError_t launch_fused_apply(int prec, void* amp, int n, int k,
                              const int32_t* q, const void* u,
                              uint64_t cmask, hipStream_t stream) {
  if (k <= 3) {
    if (cmask) return hipErrorInvalidValue;
    return launch_dense_dev(prec, amp, n, k, q,
                            static_cast<const double*>(u), stream);
  }
  FusedArgs args = {};
  const int c = __builtin_popcountll(cmask);
  args.n_groups = uint64_t(1) << (n - k - c);
  args.cmask = cmask;
  args.k = k;
  for (int j = 0; j < k; ++j) args.q[j] = q[j];
  uint64_t fixed = cmask;
  for (int j = 0; j < k; ++j) fixed |= uint64_t(1) << q[j];
  for (int b = 0; b < 64; ++b)
    if (fixed >> b & 1) args.fixed[args.nfixed++] = b;
  const uint64_t per_wave = prec == 1 ? 32 : 16;
  const uint64_t waves = (args.n_groups + per_wave - 1) / per_wave;
  // Resident work-groups only (each wave loops over group batches), so
  // that a wave loads its A operands once for many batches.
  const unsigned blocks =
      grid_blocks(waves * 64, 256, fused_resident_blocks(prec, k));
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
