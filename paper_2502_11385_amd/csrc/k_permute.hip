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

// LDS slot of tile-local index r: its bits m.. folded onto bits 0..m-1 so
// that both the loads (r consecutive) and the stores (r varying in the
// bits that land on the lowest destination qubits) spread over banks.
__device__ __forceinline__ uint32_t perm_slot(uint32_t r, int m) {
  return r ^ ((r >> m) & ((1u << m) - 1u));
}

// Work-group g takes tiles g, g + gridDim.x, ... (the grid is capped so
// that grid x block stays far below 2^32 threads at 34 qubits).
template <typename C>
__global__ void __launch_bounds__(256)
    permute_kernel(const C* __restrict__ src, C* __restrict__ dst,
                   PermArgs p, uint64_t tiles) {
  extern __shared__ double lds_raw[];
  C* lds = reinterpret_cast<C*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  const uint32_t step = blockDim.x;
  // Spreading and the destination-to-source bit map are linear, and the
  // thread and step parts of r = tid + e * step have disjoint bits, so each
  // splits into a per-thread term and a per-step (uniform) term.
  const uint64_t s_thr = spread_bits(tid, p.s_bits, p.s);
  const uint64_t d_thr = spread_bits(tid, p.d_bits, p.s);
  uint32_t g_thr = 0;
  for (int j = 0; j < p.s; ++j) g_thr |= ((tid >> j) & 1u) << p.src_of[j];
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    // tile index -> source base (outer source bits) and its destination
    uint64_t sb = 0, db = 0;
    for (int j = 0; j < p.n_outer; ++j) {
      const uint64_t bit = (t >> j) & 1;
      sb |= bit << p.outer_src[j];
      db |= bit << p.outer_dst[j];
    }
    for (int e = 0; e < p.ne; ++e) {
      const uint32_t r = uint32_t(e) * step + tid;
      lds[perm_slot(r, p.m)] = src[sb | s_thr | p.se[e]];
    }
    __syncthreads();
    for (int e = 0; e < p.ne; ++e)
      dst[db | d_thr | p.de[e]] = lds[perm_slot(g_thr | p.ge[e], p.m)];
    __syncthreads();  // the next tile reuses the LDS
  }
}

hipError_t launch_permute(int prec, const void* src, void* dst, int n,
                          const PermArgs& p, hipStream_t stream) {
  if (p.s < 0 || p.s > kPermMaxTileBits || p.s > n || p.m < 0 || p.m > p.s ||
      p.ne < 1 || p.ne > 16 ||
      uint64_t(p.ne) * ((1u << p.s) < 256u ? (1u << p.s) : 256u) != (1ull << p.s))
    return hipErrorInvalidValue;
  if (p.n_outer != n - p.s) return hipErrorInvalidValue;
  const uint64_t tiles = uint64_t(1) << (n - p.s);
  const unsigned threads = (1u << p.s) < 256u ? (1u << p.s) : 256u;
  const unsigned grid = unsigned(tiles < (1u << 20) ? tiles : (1u << 20));
  if (prec == 1)
    permute_kernel<float2><<<grid, threads, sizeof(float2) << p.s, stream>>>(
        static_cast<const float2*>(src), static_cast<float2*>(dst), p, tiles);
  else
    permute_kernel<double2><<<grid, threads, sizeof(double2) << p.s, stream>>>(
        static_cast<const double2*>(src), static_cast<double2*>(dst), p,
        tiles);
  return hipGetLastError();
}

}  // namespace qsv
