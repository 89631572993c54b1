// Qubit relabelling pass: qubit q of the state becomes qubit perm[q].
//
// This is the data movement of the paper's swap insertion (Section III.B):
// one pass moves busy high qubits to low positions, where later tiles and
// coalesced runs cover them.  A work-group takes one tile of source indices
// spanned by the source bits S = {0..m-1} + {perm^-1(0..m-1)}: its reads
// are contiguous runs of the m lowest source qubits and its writes
// contiguous runs of the m lowest destination qubits, with the tile
// transposed through LDS in between.
#include "device_common.h"

namespace qsv {

constexpr int kPermMaxTileBits = 10;

// Spread the low bits of x over the listed positions (ascending count k).
__device__ __forceinline__ uint64_t spread_bits(uint32_t x, const int* pos,
                                                int k) {
  uint64_t v = 0;
  for (int j = 0; j < k; ++j) v |= uint64_t((x >> j) & 1u) << pos[j];
  return v;
}

template <typename C>
__global__ void __launch_bounds__(256)
    permute_kernel(const C* __restrict__ src, C* __restrict__ dst,
                   PermArgs p) {
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  const uint32_t tile_amps = 1u << p.s;
  // tile index -> source base (outer source bits) and its destination
  uint64_t t = blockIdx.x;
  uint64_t sb = 0, db = 0;
  for (int j = 0; j < p.n_outer; ++j) {
    const uint64_t bit = (t >> j) & 1;
    sb |= bit << p.outer_src[j];
    db |= bit << p.outer_dst[j];
  }
  for (uint32_t r = tid; r < tile_amps; r += blockDim.x)
    lds[r] = src[sb | spread_bits(r, p.s_bits, p.s)];
  __syncthreads();
  for (uint32_t rd = tid; rd < tile_amps; rd += blockDim.x) {
    // destination tile-local bit j holds source tile-local bit src_of[j]
    uint32_t r = 0;
    for (int j = 0; j < p.s; ++j) r |= ((rd >> j) & 1u) << p.src_of[j];
    dst[db | spread_bits(rd, p.d_bits, p.s)] = lds[r];
  }
}

hipError_t launch_permute(int prec, const void* src, void* dst, int n,
                          const PermArgs& p, hipStream_t stream) {
  if (p.s < 0 || p.s > kPermMaxTileBits || p.s > n) return hipErrorInvalidValue;
  const uint64_t tiles = uint64_t(1) << (n - p.s);
  const unsigned threads = (1u << p.s) < 256u ? (1u << p.s) : 256u;
  if (prec == 1)
    permute_kernel<float2><<<unsigned(tiles), threads,
                             sizeof(float2) << p.s, stream>>>(
        static_cast<const float2*>(src), static_cast<float2*>(dst), p);
  else
    permute_kernel<double2><<<unsigned(tiles), threads,
                              sizeof(double2) << p.s, stream>>>(
        static_cast<const double2*>(src), static_cast<double2*>(dst), p);
  return hipGetLastError();
}

}  // namespace qsv
