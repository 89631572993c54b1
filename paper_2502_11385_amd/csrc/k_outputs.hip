// Further outputs of a state: the k most probable outcomes, and expectation
// values of Pauli strings.
//
// Top-k decides on the key p = re*re + im*im computed in FP64 with every
// product and the sum rounded separately (no fused multiply-add), so the
// decision is the same as any plain FP64 evaluation of that expression.
// p >= 0, so the key's bit pattern orders like its value: a radix select on
// 12-bit digits (one histogram pass over the state per digit, integer
// counts) fixes the threshold key; the elements above it are gathered, and
// the remaining places go to the elements equal to it in index order.
#include "reduce_core.h"

namespace qsv {

constexpr int kTopkBins = 4096;  // 12-bit digits

template <typename C>
__device__ __forceinline__ uint64_t topk_key(C v) {
  // no contraction into a fused multiply-add: each operation rounds
#pragma clang fp contract(off)
  const double x = double(v.x), y = double(v.y);
  const double xx = x * x, yy = y * y;
  const double p = xx + yy;
  return uint64_t(__double_as_longlong(p));
}

// Histogram of digit (key >> shift) & (bins - 1) over the keys whose bits
// under `mask` equal `prefix`.
template <typename C>
__global__ void __launch_bounds__(256)
    topk_hist_kernel(const C* __restrict__ a, uint64_t count, uint64_t mask,
                     uint64_t prefix, int shift, int bins,
                     unsigned long long* __restrict__ hist) {
  __shared__ unsigned int h[kTopkBins];
  for (int b = threadIdx.x; b < kTopkBins; b += 256) h[b] = 0;
  __syncthreads();
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < count;
       i += stride) {
    const uint64_t k = topk_key(a[i]);
    if ((k & mask) == prefix)
      atomicAdd(&h[(k >> shift) & uint64_t(bins - 1)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < bins; b += 256)
    if (h[b]) atomicAdd(&hist[b], (unsigned long long)h[b]);
}

// Gather (key, index) of every element with (key & mask) > prefix, or >=
// prefix when `ge`; positions come from an integer counter (order is fixed
// afterwards by sorting on (key, index)).
template <typename C>
__global__ void __launch_bounds__(256)
    topk_collect_kernel(const C* __restrict__ a, uint64_t count,
                        uint64_t mask, uint64_t prefix, int ge,
                        unsigned long long* __restrict__ counter, uint64_t cap,
                        uint64_t* __restrict__ out_key,
                        uint64_t* __restrict__ out_idx) {
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < count;
       i += stride) {
    const uint64_t k = topk_key(a[i]);
    const uint64_t m = k & mask;
    if (ge ? m >= prefix : m > prefix) {
      const unsigned long long slot = atomicAdd(counter, 1ull);
      if (slot < cap) {
        out_key[slot] = k;
        out_idx[slot] = i;
      }
    }
  }
}

// Elements equal to the threshold key in each block's contiguous range.
template <typename C>
__global__ void __launch_bounds__(256)
    topk_tie_count_kernel(const C* __restrict__ a, uint64_t count,
                          uint64_t chunk, uint64_t key,
                          unsigned long long* __restrict__ counts) {
  __shared__ unsigned int tot;
  if (threadIdx.x == 0) tot = 0;
  __syncthreads();
  const uint64_t lo = uint64_t(blockIdx.x) * chunk;
  const uint64_t hi = lo + chunk < count ? lo + chunk : count;
  unsigned int c = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += 256)
    c += topk_key(a[i]) == key ? 1u : 0u;
  atomicAdd(&tot, c);
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// The first `need` elements equal to the threshold key, in index order:
// block b starts at rank offsets[b] and ranks its own equal elements in
// index order (wave ballots, then waves in order).
template <typename C>
__global__ void __launch_bounds__(256)
    topk_tie_collect_kernel(const C* __restrict__ a, uint64_t count,
                            uint64_t chunk, uint64_t key,
                            const unsigned long long* __restrict__ offsets,
                            uint64_t need, uint64_t* __restrict__ out_idx) {
  __shared__ unsigned int wave_cnt[4];
  const uint64_t base = offsets[blockIdx.x];
  if (base >= need) return;  // uniform over the block
  const uint64_t lo = uint64_t(blockIdx.x) * chunk;
  const uint64_t hi = lo + chunk < count ? lo + chunk : count;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t run = base;
  for (uint64_t s = lo; s < hi && run < need; s += 256) {
    const uint64_t i = s + threadIdx.x;
    const bool eq = i < hi && topk_key(a[i]) == key;
    const uint64_t bal = __ballot(eq);
    if (lane == 0) wave_cnt[wv] = __popcll(bal);
    __syncthreads();
    uint64_t before = 0;
    for (int w = 0; w < wv; ++w) before += wave_cnt[w];
    const uint64_t mine = __popcll(bal & ((uint64_t(1) << lane) - 1));
    const uint64_t rank = run + before + mine;
    if (eq && rank < need) out_idx[rank] = i;
    uint64_t total = 0;
    for (int w = 0; w < 4; ++w) total += wave_cnt[w];
    __syncthreads();
    run += total;
  }
}

template <typename C>
static const C* as(const void* p) {
  return static_cast<const C*>(p);
}

unsigned topk_grid(uint64_t count) {
  const uint64_t g = (count + 255) / 256;
  return unsigned(g < 4096 ? g : 4096);
}

hipError_t launch_topk_hist(int prec, const void* amp, uint64_t count,
                            uint64_t mask, uint64_t prefix, int shift,
                            int bins, unsigned long long* hist,
                            hipStream_t stream) {
  const unsigned g = topk_grid(count);
  if (prec == 1)
    topk_hist_kernel<float2><<<g, 256, 0, stream>>>(
        as<float2>(amp), count, mask, prefix, shift, bins, hist);
  else
    topk_hist_kernel<double2><<<g, 256, 0, stream>>>(
        as<double2>(amp), count, mask, prefix, shift, bins, hist);
  return hipGetLastError();
}

hipError_t launch_topk_collect(int prec, const void* amp, uint64_t count,
                               uint64_t mask, uint64_t prefix, int ge,
                               unsigned long long* counter, uint64_t cap,
                               uint64_t* out_key, uint64_t* out_idx,
                               hipStream_t stream) {
  const unsigned g = topk_grid(count);
  if (prec == 1)
    topk_collect_kernel<float2><<<g, 256, 0, stream>>>(
        as<float2>(amp), count, mask, prefix, ge, counter, cap, out_key,
        out_idx);
  else
    topk_collect_kernel<double2><<<g, 256, 0, stream>>>(
        as<double2>(amp), count, mask, prefix, ge, counter, cap, out_key,
        out_idx);
  return hipGetLastError();
}

hipError_t launch_topk_ties(int prec, const void* amp, uint64_t count,
                            uint64_t key, unsigned blocks, uint64_t chunk,
                            unsigned long long* counts,
                            const unsigned long long* offsets, uint64_t need,
                            uint64_t* out_idx, hipStream_t stream) {
  if (!offsets) {
    if (prec == 1)
      topk_tie_count_kernel<float2><<<blocks, 256, 0, stream>>>(
          as<float2>(amp), count, chunk, key, counts);
    else
      topk_tie_count_kernel<double2><<<blocks, 256, 0, stream>>>(
          as<double2>(amp), count, chunk, key, counts);
  } else {
    if (prec == 1)
      topk_tie_collect_kernel<float2><<<blocks, 256, 0, stream>>>(
          as<float2>(amp), count, chunk, key, offsets, need, out_idx);
    else
      topk_tie_collect_kernel<double2><<<blocks, 256, 0, stream>>>(
          as<double2>(amp), count, chunk, key, offsets, need, out_idx);
  }
  return hipGetLastError();
}

// ------------------------------------------------------ Pauli expectations
//
// For P = i^{|x & z|} X^x Z^z (x: qubits with X or Y, z: qubits with Z or
// Y), P|i> = i^{|x & z|} (-1)^{|i & z|} |i ^ x>, so
// <psi|P|psi> = Re(i^{|x & z|} S), S = sum_i conj(a_{i^x}) a_i (-1)^{|i & z|}.
// Each block sums 4096 terms of S (real and imaginary parts, FP64 with
// Neumaier compensation, fixed order); one block then sums the blocks.

constexpr int kPauliChunkLog = 12;

template <typename C>
__global__ void __launch_bounds__(256)
    pauli_partial_kernel(const C* __restrict__ a, uint64_t count, uint64_t xm,
                         uint64_t zm, double* __restrict__ partial) {
  __shared__ double sh[512];
  const uint64_t start = uint64_t(blockIdx.x) << kPauliChunkLog;
  double sr = 0, cr = 0, si = 0, ci = 0;
  for (int it = 0; it < (1 << kPauliChunkLog) / 256; ++it) {
    const uint64_t i = start + uint64_t(it) * 256 + threadIdx.x;
    if (i < count) {
      const C ai = a[i], aj = a[i ^ xm];
      const double xr = double(aj.x), xi = double(aj.y);
      const double yr = double(ai.x), yi = double(ai.y);
      double re = xr * yr + xi * yi;
      double im = xr * yi - xi * yr;
      if (__popcll(i & zm) & 1) {
        re = -re;
        im = -im;
      }
      nadd(sr, cr, re);
      nadd(si, ci, im);
    }
  }
  block_reduce_pair(sr, cr, sh);
  __syncthreads();
  block_reduce_pair(si, ci, sh);
  if (threadIdx.x == 0) {
    double* p = partial + 4 * uint64_t(blockIdx.x);
    p[0] = sr;
    p[1] = cr;
    p[2] = si;
    p[3] = ci;
  }
}

__global__ void __launch_bounds__(256)
    pauli_final_kernel(const double* __restrict__ partial, uint64_t blocks,
                       double* __restrict__ out) {
  __shared__ double sh[512];
  double sr = 0, cr = 0, si = 0, ci = 0;
  for (uint64_t b = threadIdx.x; b < blocks; b += 256) {
    nadd(sr, cr, partial[4 * b]);
    cr += partial[4 * b + 1];
    nadd(si, ci, partial[4 * b + 2]);
    ci += partial[4 * b + 3];
  }
  block_reduce_pair(sr, cr, sh);
  __syncthreads();
  block_reduce_pair(si, ci, sh);
  if (threadIdx.x == 0) {
    out[0] = sr + cr;
    out[1] = si + ci;
  }
}

size_t pauli_scratch_bytes(int n) {
  const uint64_t blocks =
      ((uint64_t(1) << n) + (1u << kPauliChunkLog) - 1) >> kPauliChunkLog;
  return size_t(blocks) * 4 * sizeof(double);
}

hipError_t launch_pauli(int prec, const void* amp, int n, uint64_t xm,
                        uint64_t zm, double* scratch, double* out_dev,
                        hipStream_t stream) {
  const uint64_t count = uint64_t(1) << n;
  const uint64_t blocks =
      (count + (1u << kPauliChunkLog) - 1) >> kPauliChunkLog;
  if (prec == 1)
    pauli_partial_kernel<float2><<<unsigned(blocks), 256, 0, stream>>>(
        as<float2>(amp), count, xm, zm, scratch);
  else
    pauli_partial_kernel<double2><<<unsigned(blocks), 256, 0, stream>>>(
        as<double2>(amp), count, xm, zm, scratch);
  pauli_final_kernel<<<1, 256, 0, stream>>>(scratch, blocks, out_dev);
  return hipGetLastError();
}

}  // namespace qsv
