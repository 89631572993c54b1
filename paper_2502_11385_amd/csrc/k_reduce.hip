// Reductions of the state: probabilities and norm, renormalisation,
// marginals over specified qubits, and inverse-CDF sampling.
//
// Every floating-point sum runs in FP64 in a fixed order (per-thread
// sequential, then fixed LDS trees), so a given state always reduces to the
// same bits; the norm and marginal sums carry Neumaier compensation.  No
// floating-point atomics are used.
#include <mutex>

#include "reduce_core.h"

namespace qsv {

// ------------------------------------------------ fixed device scratch

// Scratch of the allocation-free entry points, resident on every device
// the library runs on until the process ends.  In host code `scratch`
// names a host-side stand-in: kernels get the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
// 4 MiB of (sum, compensation) pairs, one per 4096 amplitudes of a state of
// up to 30 qubits, and one 256-byte slot for the total.
constexpr size_t kFixedScratchBytes = (size_t(4) << 20) + 256;
static __device__ __align__(256) char scratch[kFixedScratchBytes];

static std::mutex g_fixed_mu;
static void* g_fixed_ptr[kMaxDevices] = {};

size_t fixed_scratch_bytes() { return kFixedScratchBytes; }

hipError_t fixed_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (!g_fixed_ptr[device]) {
    // the device is current (the caller selected it)
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_fixed_ptr[device] = p;
  }
  *out = g_fixed_ptr[device];
  return hipSuccess;
}

// ------------------------------------------------------- probabilities

constexpr int kProbChunkLog = 12;  // 4096 amplitudes per block, 16/thread

template <typename T, typename OUT>
__global__ void __launch_bounds__(256)
    probs_kernel(const typename CxT<T>::type* __restrict__ a, uint64_t count,
                 OUT* __restrict__ out, double* __restrict__ partial) {
  __shared__ double sh[512];
  const uint64_t start = uint64_t(blockIdx.x) << kProbChunkLog;
  double s = 0, c = 0;
#pragma unroll 4
  for (int it = 0; it < (1 << kProbChunkLog) / 256; ++it) {
    const uint64_t i = start + uint64_t(it) * 256 + threadIdx.x;
    if (i < count) {
      const double p = prob_of(a[i]);
      if (out) out[i] = OUT(p);
      nadd(s, c, p);
    }
  }
  block_reduce_pair(s, c, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s;
    partial[2 * blockIdx.x + 1] = c;
  }
}

// One block sums `count` (s, c) pairs in a fixed order into out[0].
__global__ void __launch_bounds__(256)
    sum_pairs_kernel(const double* __restrict__ pairs, uint64_t count,
                     double* __restrict__ out) {
  __shared__ double sh[512];
  double s = 0, c = 0;
  for (uint64_t k = threadIdx.x; k < count; k += 256) {
    nadd(s, c, pairs[2 * k]);
    c += pairs[2 * k + 1];
  }
  block_reduce_pair(s, c, sh);
  if (threadIdx.x == 0) out[0] = s + c;
}

size_t norm_scratch_bytes(int n) {
  uint64_t blocks = ((uint64_t(1) << n) + (1u << kProbChunkLog) - 1) >>
                    kProbChunkLog;
  return size_t(blocks) * 2 * sizeof(double);
}

template <typename T>
static void probs_dispatch(const void* amp, int n, void* out, int out_fp64,
                           double* scratch, hipStream_t stream) {
  using C = typename CxT<T>::type;
  const uint64_t count = uint64_t(1) << n;
  const unsigned blocks =
      unsigned((count + (1u << kProbChunkLog) - 1) >> kProbChunkLog);
  const C* a = static_cast<const C*>(amp);
  if (!out)
    probs_kernel<T, double><<<blocks, 256, 0, stream>>>(a, count, nullptr,
                                                        scratch);
  else if (out_fp64)
    probs_kernel<T, double><<<blocks, 256, 0, stream>>>(
        a, count, static_cast<double*>(out), scratch);
  else
    probs_kernel<T, float><<<blocks, 256, 0, stream>>>(
        a, count, static_cast<float*>(out), scratch);
}

hipError_t launch_probs(int prec, const void* amp, int n, void* out,
                        int out_fp64, double* scratch, double* norm_dev,
                        hipStream_t stream) {
  if (prec == 1)
    probs_dispatch<float>(amp, n, out, out_fp64, scratch, stream);
  else
    probs_dispatch<double>(amp, n, out, out_fp64, scratch, stream);
  const uint64_t blocks = ((uint64_t(1) << n) + (1u << kProbChunkLog) - 1) >>
                          kProbChunkLog;
  if (norm_dev)
    sum_pairs_kernel<<<1, 256, 0, stream>>>(scratch, blocks, norm_dev);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256)
    scale_kernel(typename CxT<T>::type* __restrict__ a, uint64_t count,
                 const double* __restrict__ norm) {
  const T f = T(1.0 / sqrt(norm[0]));
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
       i < count; i += stride) {
    auto v = a[i];
    v.x *= f;
    v.y *= f;
    a[i] = v;
  }
}

hipError_t launch_scale(int prec, void* amp, int n, const double* norm_dev,
                        hipStream_t stream) {
  const uint64_t count = uint64_t(1) << n;
  const unsigned blocks = grid_blocks(count, 256, 1u << 18);
  if (prec == 1)
    scale_kernel<float><<<blocks, 256, 0, stream>>>(
        static_cast<float2*>(amp), count, norm_dev);
  else
    scale_kernel<double><<<blocks, 256, 0, stream>>>(
        static_cast<double2*>(amp), count, norm_dev);
  return hipGetLastError();
}

// ------------------------------------------------------------ marginal

struct MargArgs {
  int32_t m;
  int32_t slice_bits;
  uint64_t ns;            // slices per bin
  int32_t qsorted[24];    // marginal qubits, ascending (for bit insertion)
  int32_t qorder[24];     // marginal qubits in output-bit order
};

// Block (j, slice): sums p_i over the slice's rest indices for bin j.
template <typename T>
__global__ void __launch_bounds__(256)
    marg_partial_kernel(const typename CxT<T>::type* __restrict__ a,
                        MargArgs args, double* __restrict__ partial) {
  __shared__ double sh[512];
  const uint64_t bid = blockIdx.x;
  const uint64_t j = bid / args.ns;
  const uint64_t sl = bid % args.ns;
  uint64_t jb = 0;
  for (int l = 0; l < args.m; ++l)
    if (j >> l & 1) jb |= uint64_t(1) << args.qorder[l];
  const uint64_t cnt = uint64_t(1) << args.slice_bits;
  const uint64_t r0 = sl << args.slice_bits;
  // Spreading the rest index over the non-marginal qubits distributes over
  // OR of disjoint bit sets: spread(r0 | k | t) = spread(r0) | spread(k) |
  // spread(t) for the slice base r0, the step k (multiple of 256) and the
  // thread offset t < 256, so only the uniform step term changes per step.
  auto spread = [&](uint64_t x) {
    for (int l = 0; l < args.m; ++l) x = insert_zero64(x, args.qsorted[l]);
    return x;
  };
  const uint64_t fixed = spread(r0) | spread(threadIdx.x) | jb;
  // spread(k) for k = 0, 256, 512, ... enumerates the subsets of the mask
  // mk in increasing order: next = ((x | ~mk) + 1) & mk.
  const uint64_t mk = cnt > 256 ? spread(cnt - 1) & ~spread(255) : 0;
  double s = 0, c = 0;
  if (threadIdx.x < cnt) {
    uint64_t x = 0;
    do {
      nadd(s, c, prob_of(a[fixed | x]));
      x = ((x | ~mk) + 1) & mk;
    } while (x != 0);
  }
  block_reduce_pair(s, c, sh);
  if (threadIdx.x == 0) {
    partial[2 * bid] = s;
    partial[2 * bid + 1] = c;
  }
}

__global__ void __launch_bounds__(256)
    marg_final_kernel(const double* __restrict__ partial, uint64_t ns,
                      uint64_t nbins, double* __restrict__ out) {
  const uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nbins) return;
  double s = 0, c = 0;
  for (uint64_t k = 0; k < ns; ++k) {
    nadd(s, c, partial[2 * (j * ns + k)]);
    c += partial[2 * (j * ns + k) + 1];
  }
  out[j] = s + c;
}

static int marg_slice_bits(int n, int m) {
  int r = n - m;
  return r < 14 ? r : 14;
}

size_t marginal_scratch_bytes(int n, int m) {
  const uint64_t blocks = uint64_t(1) << (n - marg_slice_bits(n, m));
  return size_t(blocks) * 2 * sizeof(double);
}

hipError_t launch_marginal(int prec, const void* amp, int n,
                           const int32_t* qubits, int m, double* scratch,
                           double* out_dev, hipStream_t stream) {
  MargArgs args = {};
  args.m = m;
  args.slice_bits = marg_slice_bits(n, m);
  args.ns = uint64_t(1) << (n - m - args.slice_bits);
  uint64_t mask = 0;
  for (int l = 0; l < m; ++l) {
    args.qorder[l] = qubits[l];
    mask |= uint64_t(1) << qubits[l];
  }
  for (int q = 0, l = 0; q < 64; ++q)
    if (mask >> q & 1) args.qsorted[l++] = q;
  const uint64_t nbins = uint64_t(1) << m;
  const uint64_t blocks = nbins * args.ns;
  if (prec == 1)
    marg_partial_kernel<float><<<unsigned(blocks), 256, 0, stream>>>(
        static_cast<const float2*>(amp), args, scratch);
  else
    marg_partial_kernel<double><<<unsigned(blocks), 256, 0, stream>>>(
        static_cast<const double2*>(amp), args, scratch);
  marg_final_kernel<<<unsigned((nbins + 255) / 256), 256, 0, stream>>>(
      scratch, args.ns, nbins, out_dev);
  return hipGetLastError();
}

// ------------------------------------------------------------ sampling
//
// C(i) = P[b-1] + (wave-exclusive prefix of the lane) + running sum within
// the lane, where block b holds 2^B amplitudes (B = min(n, 10)) handled by
// one wave (16 consecutive amplitudes per lane) and P is the inclusive scan
// of the block totals.  Both the block totals and the per-sample search use
// the same per-lane sums and wave scan.

constexpr int kSampleBlockLog = 10;

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double wave_incl_scan(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Probability of element i of the sampled vector: an amplitude's |a|^2, or a
// stored probability.
template <typename T>
struct FromAmps {
  using in_t = typename CxT<T>::type;
  static __device__ __forceinline__ double p(in_t v) { return prob_of(v); }
};
template <typename P>
struct FromProbs {
  using in_t = P;
  static __device__ __forceinline__ double p(P v) { return double(v); }
};

// Wave-local ordering of LDS writes before reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS slice of one wave: 1024 doubles plus one pad per 16 (bank spread).
constexpr int kWaveSlice = 1024 + 64;
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Probabilities of block `blk` (2^B amplitudes) as lane `lane` sees them:
// p[e] = p(amplitude lane * E + e), e < E, with E = 2^B / min(2^B, 64).  For
// full 1024-amplitude blocks the wave reads the block with coalesced loads
// (lane l takes amplitudes l, l + 64, ...) and redistributes it through its
// LDS slice, so every lane ends with its 16 consecutive probabilities.
template <class Acc>
__device__ __forceinline__ void block_probs(
    const typename Acc::in_t* __restrict__ a, uint64_t blk, int B, int lane,
    double* __restrict__ sl, double (&p)[16]) {
  const uint64_t base = blk << B;
  if (B == 10) {
#pragma unroll
    for (int e = 0; e < 16; ++e)
      sl[pad16(e * 64 + lane)] = Acc::p(a[base + uint64_t(e) * 64 + lane]);
    wave_sync();
#pragma unroll
    for (int e = 0; e < 16; ++e) p[e] = sl[pad16(lane * 16 + e)];
    wave_sync();  // the slice may be rewritten by the caller's next block
    return;
  }
  const int lanes = (1 << B) < 64 ? (1 << B) : 64;
  const int E = (1 << B) / lanes;
#pragma unroll
  for (int e = 0; e < 16; ++e)
    p[e] = (lane < lanes && e < E) ? Acc::p(a[base + uint64_t(lane) * E + e])
                                   : 0.0;
}

template <class Acc>
__global__ void __launch_bounds__(256)
    sample_blocksum_kernel(const typename Acc::in_t* __restrict__ a, int B,
                           uint64_t nblocks, double* __restrict__ S) {
  __shared__ double sh[4 * kWaveSlice];
  const uint64_t w = uint64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= nblocks) return;  // whole waves exit together
  double p[16];
  block_probs<Acc>(a, w, B, lane, sh + (threadIdx.x >> 6) * kWaveSlice, p);
  double loc = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) loc += p[e];
  const double incl = wave_incl_scan(loc);
  if (lane == 63) S[w] = incl;
}

// Inclusive scan of up to 4096 doubles per block (256 threads x 16).
__global__ void __launch_bounds__(256)
    scan_block_kernel(double* __restrict__ d, uint64_t count,
                      double* __restrict__ totals) {
  __shared__ double sh[256];
  const uint64_t start = uint64_t(blockIdx.x) * 4096 + threadIdx.x * 16;
  double v[16];
  double run = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint64_t i = start + e;
    run += (i < count) ? d[i] : 0.0;
    v[e] = run;
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  for (int w = 1; w < 256; w <<= 1) {
    const double add = threadIdx.x >= unsigned(w) ? sh[threadIdx.x - w] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  const double off = threadIdx.x ? sh[threadIdx.x - 1] : 0.0;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const uint64_t i = start + e;
    if (i < count) d[i] = off + v[e];
  }
  if (threadIdx.x == 255 && totals) totals[blockIdx.x] = sh[255];
}

__global__ void __launch_bounds__(256)
    scan_add_kernel(double* __restrict__ d, uint64_t count,
                    const double* __restrict__ scanned_totals) {
  if (blockIdx.x == 0) return;
  const double off = scanned_totals[blockIdx.x - 1];
  const uint64_t start = uint64_t(blockIdx.x) * 4096;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const uint64_t i = start + e;
    if (i < count) d[i] += off;
  }
}

static uint64_t scan_scratch_count(uint64_t count) {
  uint64_t tot = 0;
  while (count > 4096) {
    count = (count + 4095) / 4096;
    tot += count;
  }
  return tot;
}

static void scan_inclusive(double* d, uint64_t count, double* scratch,
                           hipStream_t stream) {
  const uint64_t blocks = (count + 4095) / 4096;
  if (blocks == 1) {
    scan_block_kernel<<<1, 256, 0, stream>>>(d, count, nullptr);
    return;
  }
  scan_block_kernel<<<unsigned(blocks), 256, 0, stream>>>(d, count, scratch);
  scan_inclusive(scratch, blocks, scratch + blocks, stream);
  scan_add_kernel<<<unsigned(blocks), 256, 0, stream>>>(d, count, scratch);
}

template <class Acc>
__global__ void __launch_bounds__(256)
    sample_kernel(const typename Acc::in_t* __restrict__ a, int B,
                  uint64_t nblocks, const double* __restrict__ P,
                  uint64_t shots, uint64_t seed, uint64_t* __restrict__ out) {
  __shared__ double sh[4 * kWaveSlice];
  const uint64_t j = uint64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= shots) return;  // whole waves exit together
  const double u = double(splitmix64_at(seed, j) >> 11) * 0x1p-53;
  const double t = u * P[nblocks - 1];
  uint64_t lo = 0, hi = nblocks - 1;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (P[mid] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  const uint64_t b = lo;
  const double base = b ? P[b - 1] : 0.0;
  const int lanes = (1 << B) < 64 ? (1 << B) : 64;
  const int E = (1 << B) / lanes;
  double p[16];
  block_probs<Acc>(a, b, B, lane, sh + (threadIdx.x >> 6) * kWaveSlice, p);
  double loc = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) loc += p[e];
  const double incl = wave_incl_scan(loc);
  double excl = __shfl_up(incl, 1, 64);
  if (lane == 0) excl = 0.0;
  double run = base + excl;
  int found = -1;
  int last_pos = -1;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    if (e < E) {
      run += p[e];
      if (found < 0 && run > t) found = e;
      if (p[e] > 0.0) last_pos = e;
    }
  }
  const uint64_t hit = __ballot(found >= 0);
  uint64_t idx;
  if (hit) {
    const int f = __ffsll((unsigned long long)hit) - 1;
    const int e = __shfl(found, f, 64);
    idx = (b << B) + uint64_t(f) * E + e;
  } else {
    // Rounding left t beyond this block's running sums: take the block's
    // last amplitude with nonzero probability.
    const uint64_t nz = __ballot(last_pos >= 0);
    const int f = nz ? 63 - __clzll((long long)nz) : 0;
    const int e = nz ? __shfl(last_pos, f, 64) : 0;
    idx = (b << B) + uint64_t(f) * E + e;
  }
  if (lane == 0) out[j] = idx;
}

static int sample_block_log(int n) {
  return n < kSampleBlockLog ? n : kSampleBlockLog;
}

size_t sample_scratch_bytes(int n, uint64_t shots) {
  const uint64_t nb = uint64_t(1) << (n - sample_block_log(n));
  return size_t(nb + scan_scratch_count(nb)) * sizeof(double) +
         size_t(shots) * sizeof(uint64_t);
}

template <class Acc>
static void sample_dispatch(const void* src, int n, uint64_t shots,
                            uint64_t seed, void* scratch, uint64_t* out_dev,
                            hipStream_t stream) {
  using In = typename Acc::in_t;
  const In* a = static_cast<const In*>(src);
  const int B = sample_block_log(n);
  const uint64_t nb = uint64_t(1) << (n - B);
  double* P = static_cast<double*>(scratch);
  double* sc = P + nb;
  sample_blocksum_kernel<Acc><<<unsigned((nb + 3) / 4), 256, 0, stream>>>(
      a, B, nb, P);
  scan_inclusive(P, nb, sc, stream);
  if (shots)
    sample_kernel<Acc><<<unsigned((shots + 3) / 4), 256, 0, stream>>>(
        a, B, nb, P, shots, seed, out_dev);
}

hipError_t launch_sample(int prec, const void* amp, int n, uint64_t shots,
                         uint64_t seed, void* scratch, uint64_t* out_dev,
                         hipStream_t stream) {
  if (prec == 1)
    sample_dispatch<FromAmps<float>>(amp, n, shots, seed, scratch, out_dev,
                                     stream);
  else
    sample_dispatch<FromAmps<double>>(amp, n, shots, seed, scratch, out_dev,
                                      stream);
  return hipGetLastError();
}

template <class Acc>
static void sample_from_blocks(const void* src, int n, uint64_t shots,
                               uint64_t seed, void* scratch, uint64_t* out_dev,
                               hipStream_t stream) {
  using In = typename Acc::in_t;
  const In* a = static_cast<const In*>(src);
  const uint64_t nb = uint64_t(1) << (n - kSampleBlockLog);
  double* P = static_cast<double*>(scratch);
  scan_inclusive(P, nb, P + nb, stream);
  if (shots)
    sample_kernel<Acc><<<unsigned((shots + 3) / 4), 256, 0, stream>>>(
        a, kSampleBlockLog, nb, P, shots, seed, out_dev);
}

hipError_t launch_sample_from_blocks(int prec, const void* amp, int n,
                                     uint64_t shots, uint64_t seed,
                                     void* scratch, uint64_t* out_dev,
                                     hipStream_t stream) {
  if (n <= kSampleBlockLog) return hipErrorInvalidValue;
  if (prec == 1)
    sample_from_blocks<FromAmps<float>>(amp, n, shots, seed, scratch, out_dev,
                                        stream);
  else
    sample_from_blocks<FromAmps<double>>(amp, n, shots, seed, scratch,
                                         out_dev, stream);
  return hipGetLastError();
}

hipError_t launch_sample_probs(int fp64, const void* probs, int n,
                               uint64_t shots, uint64_t seed, void* scratch,
                               uint64_t* out_dev, hipStream_t stream) {
  if (fp64)
    sample_dispatch<FromProbs<double>>(probs, n, shots, seed, scratch, out_dev,
                                       stream);
  else
    sample_dispatch<FromProbs<float>>(probs, n, shots, seed, scratch, out_dev,
                                      stream);
  return hipGetLastError();
}

}  // namespace qsv
