// Cut reconstruction kernels (Section III.A).
//
// Step 1 builds, for every subcircuit, the term vectors of the one-cut
// identity applied to each of its cut ends: a downstream end contributes
// p(|0>), p(|1>), 2p(|+>) - p(|0>) - p(|1>) or 2p(|+i>) - p(|0>) - p(|1>)
// (eqs 3.3-3.6); an upstream end contributes, by shot attribution (eq 3.7),
// I + Z and I - Z from the I-basis readout (2 p(0) and 2 p(1)), or the
// signed X or Y readout p(0) - p(1).  Step 2 forms, for every outcome x of
// the uncut circuit, (1/2)^K times the sum over all 4^K joint term choices
// of the product of the subcircuits' term vectors at x's bits.
#include "cut_internal.h"
#include "device_common.h"

namespace qsv {

__device__ __forceinline__ double cut_prob(const CutArgs& a, uint64_t i) {
  return a.probs_fp64 ? static_cast<const double*>(a.probs)[i]
                      : double(static_cast<const float*>(a.probs)[i]);
}

__global__ void __launch_bounds__(256)
    cut_terms_kernel(CutArgs a) {
  const uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= a.total_entries) return;
  int s = 0;
  while (s + 1 < a.n_sub && a.subs[s + 1].entry_begin <= g) ++s;
  const CutSubDev& sd = a.subs[s];
  const uint64_t local = g - sd.entry_begin;
  const uint32_t t = uint32_t(local >> sd.eff);
  const uint64_t y = local & ((uint64_t(1) << sd.eff) - 1);
  uint64_t idx0 = 0;
  for (int i = 0; i < sd.eff; ++i) idx0 |= ((y >> i) & 1) << sd.out_pos[i];
  // choices per end: downstream ends with term 0/1 read one variant, with
  // term 2/3 three; upstream ends with term 0/1 read one outcome, with
  // term 2/3 both
  int nch[kCutMaxEnds];
  uint32_t total = 1;
  for (int e = 0; e < sd.n_ends; ++e) {
    const int d = (t >> (2 * e)) & 3;
    nch[e] = d < 2 ? 1 : (sd.end_kind[e] == 0 ? 3 : 2);
    total *= uint32_t(nch[e]);
  }
  const uint64_t* vo = a.voff + sd.v_offset;
  double acc = 0.0;
  for (uint32_t c = 0; c < total; ++c) {
    uint32_t r = c;
    uint64_t v = 0, idx = idx0;
    double coef = 1.0;
    for (int e = 0; e < sd.n_ends; ++e) {
      const int d = (t >> (2 * e)) & 3;
      const int k = int(r % uint32_t(nch[e]));
      r /= uint32_t(nch[e]);
      if (sd.end_kind[e] == 0) {
        // initial state label and its coefficient
        int label = d;
        if (d >= 2) {
          label = k == 0 ? d : k - 1;
          coef *= k == 0 ? 2.0 : -1.0;
        }
        v += uint64_t(label) * uint64_t(sd.end_mult[e]);
      } else {
        // readout basis I (terms 0, 1), X (2) or Y (3), and the outcome
        const int basis = d < 2 ? 0 : d - 1;
        v += uint64_t(basis) * uint64_t(sd.end_mult[e]);
        int m;
        if (d < 2) {
          m = d;
          coef *= 2.0;
        } else {
          m = k;
          coef *= k ? -1.0 : 1.0;
        }
        idx |= uint64_t(m) << sd.end_pos[e];
      }
    }
    acc += coef * cut_prob(a, vo[v] + idx);
  }
  a.T[sd.t_offset + local] = acc;
}

// The subcircuit's output index of outcome x (bit i = its i-th output).
__device__ __forceinline__ uint64_t cut_gather(const CutSubDev& sd,
                                               uint64_t x) {
  uint64_t v = 0;
  for (int r = 0; r < sd.n_runs; ++r)
    v |= ((x >> sd.run_src[r]) & ((uint64_t(1) << sd.run_len[r]) - 1))
         << sd.run_dst[r];
  return v;
}

// One thread per outcome x: the sum over all 4^K term choices of the
// product of the subcircuits' entries.
__global__ void __launch_bounds__(256)
    cut_kron_simple_kernel(CutArgs a, const double* __restrict__ T,
                           double* __restrict__ out) {
  const uint64_t x = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= (uint64_t(1) << a.n_qubits)) return;
  uint64_t y[kCutMaxSub];
  for (int s = 0; s < a.n_sub; ++s) y[s] = cut_gather(a.subs[s], x);
  double acc = 0.0;
  for (uint64_t t = 0; t < a.n_terms; ++t) {
    const uint64_t* row = a.tt + t * uint64_t(a.n_sub);
    double prod = 1.0;
    for (int s = 0; s < a.n_sub; ++s) prod *= T[row[s] + y[s]];
    acc += prod;
  }
  out[x] = acc * ldexp(1.0, -a.n_cuts);
}


// One wave per nb blocks of 64 consecutive outcomes (n_qubits >= 6).
// Within a block the uniform subcircuits' entries are the same for every
// lane, so the sum factors: p(x) = (1/2)^K sum_c W[c] prod_{varying s}
// T_s(c)[y_s(x)], with W[c] = sum_u prod_{uniform s} T_s(c, u)[y_s].  The
// wave first forms every block's products over the uniform subcircuits for
// all (c, u) in parallel, then W[c] by summing over u in increasing order,
// then each lane sums over c in increasing order for its outcomes.
constexpr int kCutWaveLds = 512;  // doubles of LDS per wave

__global__ void __launch_bounds__(256)
    cut_kron_wave_kernel(CutArgs a, const double* __restrict__ T,
                         double* __restrict__ out, int nb) {
  __shared__ double lds[4][kCutWaveLds];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t nx = uint64_t(1) << a.n_qubits;
  const uint64_t x0 = (uint64_t(blockIdx.x) * 4 + wv) * 64 * uint64_t(nb);
  if (x0 >= nx) return;  // whole waves exit
  double* P = lds[wv];                               // [nb][n_c][n_u]
  double* W = P + uint64_t(nb) * a.n_c * a.n_u;      // [nb][n_c]
  const uint64_t ncu = a.n_c * a.n_u;
  for (uint64_t i = lane; i < uint64_t(nb) * ncu; i += 64) {
    const uint64_t blk = i / ncu, cu = i - blk * ncu;
    const uint64_t xb = x0 + blk * 64;
    const uint64_t* row = a.ttu + cu * uint64_t(a.n_uni);
    double prod = 1.0;
    for (int k = 0; k < a.n_uni; ++k)
      prod *= T[row[k] + cut_gather(a.subs[a.uni_sub[k]], xb)];
    P[i] = prod;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (uint64_t i = lane; i < uint64_t(nb) * a.n_c; i += 64) {
    double sum = 0.0;
    for (uint64_t u = 0; u < a.n_u; ++u) sum += P[i * a.n_u + u];
    W[i] = sum;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const double scale = ldexp(1.0, -a.n_cuts);
  for (int blk = 0; blk < nb; ++blk) {
    const uint64_t x = x0 + uint64_t(blk) * 64 + uint64_t(lane);
    uint64_t yv[kCutMaxVary];
#pragma unroll
    for (int k = 0; k < kCutMaxVary; ++k)
      yv[k] = k < a.n_vary ? cut_gather(a.subs[a.vary_sub[k]], x) : 0;
    double acc = 0.0;
    for (uint64_t c = 0; c < a.n_c; ++c) {
      const uint64_t* row = a.ttv + c * uint64_t(a.n_vary);
      double prod = W[uint64_t(blk) * a.n_c + c];
#pragma unroll
      for (int k = 0; k < kCutMaxVary; ++k)
        if (k < a.n_vary) prod *= T[row[k] + yv[k]];
      acc += prod;
    }
    out[x] = acc * scale;
  }
}

hipError_t launch_cut(const CutArgs& a, double* out, hipStream_t stream) {
  if (a.total_entries) {
    const uint64_t blocks = (a.total_entries + 255) / 256;
    cut_terms_kernel<<<unsigned(blocks), 256, 0, stream>>>(a);
  }
  const uint64_t nx = uint64_t(1) << a.n_qubits;
  // blocks of 64 outcomes per wave: up to 16, within the wave's LDS share
  // (nb * n_c * (n_u + 1) doubles) and the number of blocks
  int nb = 16;
  while (nb > 1 && (uint64_t(nb) * a.n_c * (a.n_u + 1) > uint64_t(kCutWaveLds) ||
                    uint64_t(nb) * 64 > nx))
    nb >>= 1;
  if (a.n_qubits >= 6 && a.n_vary <= kCutMaxVary &&
      a.n_c * (a.n_u + 1) <= uint64_t(kCutWaveLds)) {
    const uint64_t waves = nx / (64 * uint64_t(nb));
    cut_kron_wave_kernel<<<unsigned((waves + 3) / 4), 256, 0, stream>>>(
        a, a.T, out, nb);
  } else
    cut_kron_simple_kernel<<<unsigned((nx + 255) / 256), 256, 0, stream>>>(
        a, a.T, out);
  return hipGetLastError();
}

}  // namespace qsv
