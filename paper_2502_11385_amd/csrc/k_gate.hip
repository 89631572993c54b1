// Plain per-gate kernels: basis-state initialisation, dense k-target gates
// with controls (strided pair/quad/... updates), diagonal gates.
//
// A dense gate visits only the 2^(n-k-c) cosets whose control bits are 1:
// thread g expands g by inserting zero bits at the sorted target and control
// positions, sets the control bits, and updates the 2^k amplitudes at
// base + sum_j bit_j(r) 2^targets[j].  Consecutive threads take consecutive
// g, so for targets above the lowest few qubits both halves of every pair are
// contiguous HBM streams 2^t amplitudes apart.
#include "device_common.h"

namespace qsv {

// ---------------------------------------------------------------- init

template <typename T>
__global__ void __launch_bounds__(256)
    fill_basis_kernel(typename CxT<T>::type* __restrict__ a, uint64_t count,
                      uint64_t index) {
  using C = typename CxT<T>::type;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
       i < count; i += stride) {
    C v;
    v.x = (i == index) ? T(1) : T(0);
    v.y = T(0);
    a[i] = v;
  }
}

hipError_t launch_fill_basis(int prec, void* amp, int n, uint64_t index,
                             hipStream_t stream) {
  const uint64_t count = uint64_t(1) << n;
  const unsigned blocks = grid_blocks(count, 256, 1u << 18);
  if (prec == 1)
    fill_basis_kernel<float><<<blocks, 256, 0, stream>>>(
        static_cast<float2*>(amp), count, index);
  else
    fill_basis_kernel<double><<<blocks, 256, 0, stream>>>(
        static_cast<double2*>(amp), count, index);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dense

struct DenseArgs {
  uint64_t n_groups;
  uint64_t cmask;
  uint64_t lowmask;  // controls the lanes test themselves (LowMode)
  int32_t npos;
  int32_t pad;
  int32_t pos[40];   // sorted positions of targets and controls
  int32_t tq[8];     // targets, targets[0] = least significant matrix bit
  double m[32];      // matrix for k <= 2 (row-major, interleaved)
  const double* mptr;  // matrix for k >= 3
};

// Low fixed bits.  A pass that visits only the amplitudes whose fixed bits
// (controls, or the bits a diagonal pass needs set) are 1 walks runs of 2^p
// amplitudes, p the lowest such bit; where the runs are short every line is
// fetched anyway and each wave covers its lines in part.  For the lowest bits
// the lanes walk whole runs and test the bits themselves, and where one is 0
// they either store the amplitudes back unchanged (keep: whole lines are
// written) or leave them alone (skip).  Chosen by measurement on 30-qubit
// passes (ms, before and after):
//   keep, runs under 64 bytes: complex64 control on qubit 0, 1 or 2,
//     3.46 -> 2.81; complex64 CZ on qubit 0, 1 or 2, 1.57 -> 1.40;
//     complex128 CZ on qubit 0 or 1, 3.27 -> 2.90;
//   skip: complex64 control on qubit 3, 2.75-3.00 -> 2.47-2.90 over
//     targets 0 to 29; CZ on qubit 3 complex64, 1.21 -> 1.17; CZ on qubit 2
//     or 3 complex128, 3.00 -> 2.62 and 1.55 -> 1.42.
// Not taken: skip for a complex64 control on qubit 4 (target 29: 1.73 ->
// 1.51, but targets 0, 8, 15: 1.46-1.58 -> 1.54-1.63) or 5, 6 (likewise
// mixed), for a complex64 CZ on qubit 4 (0.77 -> 1.10), and testing higher
// bits beside keep ones (complex128 CZ on qubits 1, 2: 6.26 -> 6.53), so a
// gate with bits of both kinds has only its keep bits tested.  The
// complex128 dense kernel keeps the plain walk: neither form gained there
// (storing back made the compiler wait on each 16-byte store).
struct LowBits {
  uint64_t keep, skip;
};
constexpr LowBits kDenseLowC64 = {0x7, 0x8};
constexpr LowBits kDenseLowC128 = {0, 0};
constexpr LowBits kDiagLowC64 = {0x7, 0x8};
constexpr LowBits kDiagLowC128 = {0x3, 0xc};

// The fixed bits the lanes test: the keep bits among `fixed` if any, else
// its skip bits.
static uint64_t lane_tested(uint64_t fixed, LowBits lb) {
  return (fixed & lb.keep) ? fixed & lb.keep : fixed & lb.skip;
}

// How a dense pass treats the controls in args.lowmask: kLowNone has none;
// otherwise the lanes test them and, where one is 0, store the amplitudes
// back unchanged (kLowKeep: whole lines are written) or store nothing
// (kLowSkip).
enum LowMode { kLowNone, kLowKeep, kLowSkip };

// PTR: the matrix comes from device memory (FP64, rounded once to T while
// staged in LDS); otherwise from the kernel arguments (k <= 2).
template <typename T, int K, bool PTR, int LOW>
__global__ void __launch_bounds__(256)
    dense_kernel(typename CxT<T>::type* __restrict__ a, DenseArgs args) {
  using C = typename CxT<T>::type;
  constexpr int D = 1 << K;
  __shared__ C smat[PTR ? D * D : 1];
  if constexpr (PTR) {
    for (int e = threadIdx.x; e < D * D; e += blockDim.x) {
      C v;
      v.x = T(args.mptr[2 * e]);
      v.y = T(args.mptr[2 * e + 1]);
      smat[e] = v;
    }
    __syncthreads();
  }
  uint64_t off[D];
#pragma unroll
  for (int r = 0; r < D; ++r) {
    uint64_t o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (r >> j & 1) o |= uint64_t(1) << args.tq[j];
    off[r] = o;
  }
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
       g < args.n_groups; g += stride) {
    uint64_t base = g;
    for (int p = 0; p < args.npos; ++p) base = insert_zero64(base, args.pos[p]);
    base |= args.cmask;
    const bool on =
        LOW == kLowNone || (base & args.lowmask) == args.lowmask;
    C v[D];
#pragma unroll
    for (int r = 0; r < D; ++r) v[r] = a[base + off[r]];
    // All inputs are in registers, so each output can be stored at once.
#pragma unroll
    for (int r = 0; r < D; ++r) {
      T re = 0, im = 0;
#pragma unroll
      for (int s = 0; s < D; ++s) {
        T mr, mi;
        if constexpr (PTR) {
          mr = smat[r * D + s].x;
          mi = smat[r * D + s].y;
        } else {
          mr = T(args.m[2 * (r * D + s)]);
          mi = T(args.m[2 * (r * D + s) + 1]);
        }
        re += mr * v[s].x - mi * v[s].y;
        im += mr * v[s].y + mi * v[s].x;
      }
      C w;
      w.x = re;
      w.y = im;
      if constexpr (LOW == kLowKeep)
        a[base + off[r]] = on ? w : v[r];
      else if (on)
        a[base + off[r]] = w;
    }
  }
}

template <typename T, int LOW>
static void dense_dispatch_t(void* amp, int k, unsigned blocks,
                             const DenseArgs& args, hipStream_t stream) {
  using C = typename CxT<T>::type;
  C* a = static_cast<C*>(amp);
  const bool ptr = args.mptr != nullptr;
  switch (k) {
    case 1:
      if (ptr)
        dense_kernel<T, 1, true, LOW><<<blocks, 256, 0, stream>>>(a, args);
      else
        dense_kernel<T, 1, false, LOW><<<blocks, 256, 0, stream>>>(a, args);
      break;
    case 2:
      if (ptr)
        dense_kernel<T, 2, true, LOW><<<blocks, 256, 0, stream>>>(a, args);
      else
        dense_kernel<T, 2, false, LOW><<<blocks, 256, 0, stream>>>(a, args);
      break;
    case 3:
      dense_kernel<T, 3, true, LOW><<<blocks, 256, 0, stream>>>(a, args);
      break;
  }
}

template <typename T>
static void dense_dispatch(void* amp, int k, unsigned blocks,
                           const DenseArgs& args, hipStream_t stream) {
  constexpr LowBits lb = sizeof(T) == 4 ? kDenseLowC64 : kDenseLowC128;
  if constexpr (lb.keep | lb.skip) {
    if (args.lowmask & lb.keep) {
      dense_dispatch_t<T, kLowKeep>(amp, k, blocks, args, stream);
      return;
    }
    if (args.lowmask) {
      dense_dispatch_t<T, kLowSkip>(amp, k, blocks, args, stream);
      return;
    }
  }
  dense_dispatch_t<T, kLowNone>(amp, k, blocks, args, stream);
}

static void sorted_positions(uint64_t mask, int32_t* pos, int32_t* npos) {
  int j = 0;
  for (int q = 0; q < 64; ++q)
    if (mask >> q & 1) pos[j++] = q;
  *npos = j;
}

hipError_t launch_dense(int prec, void* amp, int n, const HostGate& g,
                        const double* dev_matrix, hipStream_t stream) {
  // 4-5 targets run on the matrix cores (launch_fused_apply)
  if (g.k > 3) return hipErrorInvalidValue;
  DenseArgs args = {};
  args.lowmask =
      lane_tested(g.cmask, prec == 1 ? kDenseLowC64 : kDenseLowC128);
  args.cmask = g.cmask & ~args.lowmask;
  sorted_positions(g.tmask | args.cmask, args.pos, &args.npos);
  args.n_groups = uint64_t(1) << (n - args.npos);
  for (int j = 0; j < g.k; ++j) args.tq[j] = g.t[j];
  if (g.k <= 2) {
    for (size_t e = 0; e < g.m.size(); ++e) args.m[e] = g.m[e];
  } else {
    if (!dev_matrix) return hipErrorInvalidValue;
    args.mptr = dev_matrix;
  }
  const unsigned blocks = grid_blocks(args.n_groups, 256);
  if (prec == 1)
    dense_dispatch<float>(amp, g.k, blocks, args, stream);
  else
    dense_dispatch<double>(amp, g.k, blocks, args, stream);
  return hipGetLastError();
}

// Dense k-qubit matrix from device memory on qubits q (no controls); used
// for fused blocks with k <= 3.
hipError_t launch_dense_dev(int prec, void* amp, int n, int k,
                            const int32_t* q, const double* dev_matrix,
                            hipStream_t stream) {
  if (!dev_matrix || k < 1 || k > 3) return hipErrorInvalidValue;
  DenseArgs args = {};
  args.n_groups = uint64_t(1) << (n - k);
  uint64_t mask = 0;
  for (int j = 0; j < k; ++j) {
    args.tq[j] = q[j];
    mask |= uint64_t(1) << q[j];
  }
  sorted_positions(mask, args.pos, &args.npos);
  args.mptr = dev_matrix;
  const unsigned blocks = grid_blocks(args.n_groups, 256);
  if (prec == 1)
    dense_dispatch<float>(amp, k, blocks, args, stream);
  else
    dense_dispatch<double>(amp, k, blocks, args, stream);
  return hipGetLastError();
}

// ---------------------------------------------------------------- diagonal

struct DiagArgs {
  uint64_t n_items;
  uint64_t fixed_mask;  // bits forced to 1 (controls; + targets if masked)
  uint64_t lowmask;     // fixed bits the lanes test themselves
  int32_t npos;
  int32_t k;
  int32_t pos[40];      // sorted positions of the fixed bits
  int32_t tq[8];
  double d[64];         // diagonal entries (re, im); masked: d[0..1] = phase
};

// Masked phase: multiply the amplitudes whose bits in fixed_mask and in
// lowmask are all 1 (SKIP: a lane whose lowmask bits are not leaves its
// amplitude alone; otherwise it stores it back unchanged).
template <typename T, bool SKIP>
__global__ void __launch_bounds__(256)
    diag_masked_kernel(typename CxT<T>::type* __restrict__ a, DiagArgs args) {
  using C = typename CxT<T>::type;
  C ph;
  ph.x = T(args.d[0]);
  ph.y = T(args.d[1]);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
       g < args.n_items; g += stride) {
    uint64_t i = g;
    for (int p = 0; p < args.npos; ++p) i = insert_zero64(i, args.pos[p]);
    i |= args.fixed_mask;
    const C v = a[i];
    const bool on = (i & args.lowmask) == args.lowmask;
    if constexpr (SKIP) {
      if (on) a[i] = cmul(v, ph);
    } else {
      a[i] = on ? cmul(v, ph) : v;
    }
  }
}

// General diagonal: multiply by d[r(i)], r the target bits, where the
// controls (fixed_mask and lowmask) are satisfied.
template <typename T, bool SKIP>
__global__ void __launch_bounds__(256)
    diag_table_kernel(typename CxT<T>::type* __restrict__ a, DiagArgs args) {
  using C = typename CxT<T>::type;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
       g < args.n_items; g += stride) {
    uint64_t i = g;
    for (int p = 0; p < args.npos; ++p) i = insert_zero64(i, args.pos[p]);
    i |= args.fixed_mask;
    int r = 0;
    for (int j = 0; j < args.k; ++j) r |= int((i >> args.tq[j]) & 1) << j;
    C f;
    f.x = T(args.d[2 * r]);
    f.y = T(args.d[2 * r + 1]);
    const C v = a[i];
    const bool on = (i & args.lowmask) == args.lowmask;
    if constexpr (SKIP) {
      if (on) a[i] = cmul(v, f);
    } else {
      a[i] = on ? cmul(v, f) : v;
    }
  }
}

hipError_t launch_diag(int prec, void* amp, int n, const HostGate& g,
                       hipStream_t stream) {
  DiagArgs args = {};
  args.k = g.k;
  for (int j = 0; j < g.k; ++j) args.tq[j] = g.t[j];
  const int d = 1 << g.k;
  if (g.masked_phase) {
    args.fixed_mask = g.tmask | g.cmask;
    args.d[0] = g.m[2 * ((d - 1) * d + (d - 1))];
    args.d[1] = g.m[2 * ((d - 1) * d + (d - 1)) + 1];
  } else {
    args.fixed_mask = g.cmask;
    for (int r = 0; r < d; ++r) {
      args.d[2 * r] = g.m[2 * (r * d + r)];
      args.d[2 * r + 1] = g.m[2 * (r * d + r) + 1];
    }
  }
  const LowBits lb = prec == 1 ? kDiagLowC64 : kDiagLowC128;
  args.lowmask = lane_tested(args.fixed_mask, lb);
  const bool skip = args.lowmask && !(args.lowmask & lb.keep);
  args.fixed_mask &= ~args.lowmask;
  sorted_positions(args.fixed_mask, args.pos, &args.npos);
  args.n_items = uint64_t(1) << (n - args.npos);
  const unsigned blocks = grid_blocks(args.n_items, 256);
#define QSV_DIAG(KERNEL, T)                                              \
  do {                                                                   \
    using C = typename CxT<T>::type;                                     \
    if (skip)                                                            \
      KERNEL<T, true><<<blocks, 256, 0, stream>>>(static_cast<C*>(amp),  \
                                                  args);                 \
    else                                                                 \
      KERNEL<T, false><<<blocks, 256, 0, stream>>>(static_cast<C*>(amp), \
                                                   args);                \
  } while (0)
  if (g.masked_phase) {
    if (prec == 1)
      QSV_DIAG(diag_masked_kernel, float);
    else
      QSV_DIAG(diag_masked_kernel, double);
  } else {
    if (prec == 1)
      QSV_DIAG(diag_table_kernel, float);
    else
      QSV_DIAG(diag_table_kernel, double);
  }
#undef QSV_DIAG
  return hipGetLastError();
}

}  // namespace qsv
