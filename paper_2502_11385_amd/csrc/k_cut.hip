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

__global__ void __launch_bounds__(256)
    cut_kron_kernel(CutArgs a, double* __restrict__ out) {
  const uint64_t x = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= (uint64_t(1) << a.n_qubits)) return;
  uint64_t y[kCutMaxSub];
  for (int s = 0; s < a.n_sub; ++s) {
    const CutSubDev& sd = a.subs[s];
    uint64_t v = 0;
    for (int i = 0; i < sd.eff; ++i) v |= ((x >> sd.out_uncut[i]) & 1) << i;
    y[s] = v;
  }
  double acc = 0.0;
  for (uint64_t t = 0; t < a.n_terms; ++t) {
    const uint64_t* row = a.tt + t * uint64_t(a.n_sub);
    double prod = 1.0;
    for (int s = 0; s < a.n_sub; ++s) prod *= a.T[row[s] + y[s]];
    acc += prod;
  }
  out[x] = acc * ldexp(1.0, -a.n_cuts);
}

hipError_t launch_cut(const CutArgs& a, double* out, hipStream_t stream) {
  if (a.total_entries) {
    const uint64_t blocks = (a.total_entries + 255) / 256;
    cut_terms_kernel<<<unsigned(blocks), 256, 0, stream>>>(a);
  }
  const uint64_t nx = uint64_t(1) << a.n_qubits;
  cut_kron_kernel<<<unsigned((nx + 255) / 256), 256, 0, stream>>>(a, out);
  return hipGetLastError();
}

}  // namespace qsv
