// Cut reconstruction: host validation, tables and launch (Section III.A).
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "cut_internal.h"
#include "qsv.h"

namespace qsv {
qsv_status set_error(qsv_status st, const std::string& msg);
hipError_t launch_cut(const CutArgs& a, double* out, hipStream_t stream);
}  // namespace qsv

using namespace qsv;

namespace {

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Validated problem with its host tables and workspace layout.
struct CutPlan {
  std::vector<CutSubDev> subs;
  std::vector<uint64_t> n_variants;   // per subcircuit
  std::vector<uint64_t> tt;           // [4^K][n_sub]
  std::vector<std::vector<int>> end_cut;  // per subcircuit, cut of each end
  std::vector<int> vary, uni;         // wave-kernel split of subcircuits
  std::vector<uint64_t> ttv, ttu;     // its term-vector start tables
  uint64_t n_c = 1, n_u = 1, o_ttv = 0, o_ttu = 0;
  uint64_t total_variants = 0, total_entries = 0, n_terms = 1;
  uint64_t o_voff = 0, o_tt = 0, o_T = 0, bytes = 0;
};

std::string plan_cut(const qsv_cut_spec* sp, CutPlan* P) {
  if (!sp) return "null specification";
  const int S = sp->n_sub, K = sp->n_cuts, n = sp->n_qubits;
  if (S < 1 || S > kCutMaxSub) return "n_sub must be 1..16";
  if (K < 0 || K > kCutMaxCuts) return "n_cuts must be 0..8";
  if (n < 1 || n > kCutMaxQubits) return "n_qubits must be 1..30";
  if (!sp->widths || !sp->out_qubit || !sp->cut_in || !sp->cut_out)
    return "null specification array";
  std::vector<int> seen_q(n, 0), seen_in(K, -1), seen_out(K, -1);
  P->subs.assign(S, CutSubDev{});
  P->n_variants.assign(S, 0);
  P->end_cut.assign(S, {});
  int base = 0;
  for (int s = 0; s < S; ++s) {
    const int w = sp->widths[s];
    if (w < 1 || w > kCutMaxWidth) return "subcircuit width must be 1..24";
    CutSubDev& d = P->subs[s];
    std::memset(&d, 0, sizeof d);
    d.width = w;
    uint64_t mult = 1;
    for (int j = 0; j < w; ++j) {
      const int oq = sp->out_qubit[base + j];
      const int ci = sp->cut_in[base + j];
      const int co = sp->cut_out[base + j];
      if (oq < -1 || oq >= n) return "out_qubit out of range";
      if (ci < -1 || ci >= K || co < -1 || co >= K) return "cut id out of range";
      if ((oq >= 0) == (co >= 0))
        return "every local qubit must be measured exactly once "
               "(as an output or as a cut's upstream end)";
      if (oq >= 0) {
        if (seen_q[oq]++) return "uncut qubit measured twice";
        d.out_uncut[d.eff] = oq;
        d.out_pos[d.eff++] = j;
      }
      if (ci >= 0) {
        if (seen_in[ci] >= 0) return "cut has two downstream ends";
        seen_in[ci] = s;
        if (d.n_ends >= kCutMaxEnds) return "more than 6 cut ends in a subcircuit";
        d.end_kind[d.n_ends] = 0;
        d.end_pos[d.n_ends] = j;
        d.end_mult[d.n_ends] = int32_t(mult);
        P->end_cut[s].push_back(ci);
        ++d.n_ends;
        mult *= 4;
      }
      if (co >= 0) {
        if (seen_out[co] >= 0) return "cut has two upstream ends";
        seen_out[co] = s;
        if (d.n_ends >= kCutMaxEnds) return "more than 6 cut ends in a subcircuit";
        d.end_kind[d.n_ends] = 1;
        d.end_pos[d.n_ends] = j;
        d.end_mult[d.n_ends] = int32_t(mult);
        P->end_cut[s].push_back(co);
        ++d.n_ends;
        mult *= 3;
      }
    }
    P->n_variants[s] = mult;
    base += w;
  }
  for (int q = 0; q < n; ++q)
    if (!seen_q[q]) return "an uncut qubit is never measured";
  for (int s = 0; s < S; ++s) {  // outputs as runs of consecutive uncut qubits
    CutSubDev& d = P->subs[s];
    for (int i = 0; i < d.eff; ++i) {
      if (d.n_runs > 0 && d.out_uncut[i] == d.run_src[d.n_runs - 1] +
                                                 d.run_len[d.n_runs - 1]) {
        ++d.run_len[d.n_runs - 1];
        continue;
      }
      d.run_src[d.n_runs] = d.out_uncut[i];
      d.run_dst[d.n_runs] = i;
      d.run_len[d.n_runs] = 1;
      ++d.n_runs;
    }
  }
  for (int k = 0; k < K; ++k) {
    if (seen_in[k] < 0 || seen_out[k] < 0)
      return "every cut needs one upstream and one downstream end";
    if (seen_in[k] == seen_out[k])
      return "a cut's two ends must be in different subcircuits";
  }
  for (int k = 0; k < K; ++k) P->n_terms *= 4;
  uint64_t toff = 0, voff = 0, ent = 0;
  for (int s = 0; s < S; ++s) {
    CutSubDev& d = P->subs[s];
    d.n_entries = (uint64_t(1) << (2 * d.n_ends)) << d.eff;
    d.entry_begin = ent;
    d.t_offset = toff;
    d.v_offset = voff;
    ent += d.n_entries;
    toff += d.n_entries;
    voff += P->n_variants[s];
  }
  if (ent > (uint64_t(1) << 32))
    return "term vectors exceed 2^32 entries (too many cut ends or outputs)";
  P->total_entries = ent;
  P->total_variants = voff;
  P->tt.assign(P->n_terms * uint64_t(S), 0);
  auto term_start = [&](int s, uint64_t t) {
    const CutSubDev& d = P->subs[s];
    uint64_t ti = 0;
    for (int e = 0; e < d.n_ends; ++e)
      ti |= ((t >> (2 * P->end_cut[s][e])) & 3) << (2 * e);
    return d.t_offset + (ti << d.eff);
  };
  for (uint64_t t = 0; t < P->n_terms; ++t)
    for (int s = 0; s < S; ++s) P->tt[t * S + s] = term_start(s, t);
  // wave kernel split: subcircuits with an output among uncut qubits 0..5
  // vary across a wave's lanes; cuts touching them index c, the rest u
  P->vary.clear();
  P->uni.clear();
  std::vector<int> cut_vary(K, 0);
  for (int s = 0; s < S; ++s) {
    const CutSubDev& d = P->subs[s];
    bool vary = false;
    for (int i = 0; i < d.eff; ++i) vary = vary || d.out_uncut[i] < 6;
    (vary ? P->vary : P->uni).push_back(s);
    if (vary)
      for (int k : P->end_cut[s]) cut_vary[k] = 1;
  }
  std::vector<int> cv, cu;
  for (int k = 0; k < K; ++k) (cut_vary[k] ? cv : cu).push_back(k);
  P->n_c = uint64_t(1) << (2 * cv.size());
  P->n_u = uint64_t(1) << (2 * cu.size());
  auto compose = [&](uint64_t c, uint64_t u) {
    uint64_t t = 0;
    for (size_t i = 0; i < cv.size(); ++i) t |= ((c >> (2 * i)) & 3) << (2 * cv[i]);
    for (size_t i = 0; i < cu.size(); ++i) t |= ((u >> (2 * i)) & 3) << (2 * cu[i]);
    return t;
  };
  P->ttv.assign(P->n_c * P->vary.size(), 0);
  P->ttu.assign(P->n_c * P->n_u * P->uni.size(), 0);
  for (uint64_t c = 0; c < P->n_c; ++c) {
    for (size_t k = 0; k < P->vary.size(); ++k)
      P->ttv[c * P->vary.size() + k] = term_start(P->vary[k], compose(c, 0));
    for (uint64_t u = 0; u < P->n_u; ++u)
      for (size_t k = 0; k < P->uni.size(); ++k)
        P->ttu[(c * P->n_u + u) * P->uni.size() + k] =
            term_start(P->uni[k], compose(c, u));
  }
  P->o_voff = align256(sizeof(CutSubDev) * S);
  P->o_tt = P->o_voff + align256(8 * P->total_variants);
  P->o_ttv = P->o_tt + align256(8 * P->tt.size());
  P->o_ttu = P->o_ttv + align256(8 * P->ttv.size());
  P->o_T = P->o_ttu + align256(8 * P->ttu.size());
  P->bytes = P->o_T + align256(8 * P->total_entries);
  return "";
}

}  // namespace

extern "C" {

qsv_status qsv_cut_workspace_bytes(const qsv_cut_spec* spec, uint64_t* bytes) {
  if (!bytes) return set_error(QSV_ERR_INVALID_ARG, "null output");
  CutPlan P;
  const std::string e = plan_cut(spec, &P);
  if (!e.empty()) return set_error(QSV_ERR_INVALID_ARG, e);
  *bytes = P.bytes;
  return set_error(QSV_OK, "");
}

qsv_status qsv_cut_reconstruct(const qsv_cut_spec* spec, const void* probs_dev,
                               int32_t probs_fp64, uint64_t probs_elems,
                               const uint64_t* offsets, void* workspace,
                               uint64_t workspace_bytes, double* out_dev,
                               void* hip_stream) {
  CutPlan P;
  const std::string e = plan_cut(spec, &P);
  if (!e.empty()) return set_error(QSV_ERR_INVALID_ARG, e);
  if (!probs_dev || !offsets || !workspace || !out_dev)
    return set_error(QSV_ERR_INVALID_ARG, "null pointer argument");
  if (probs_fp64 != 0 && probs_fp64 != 1)
    return set_error(QSV_ERR_INVALID_ARG, "probs_fp64 must be 0 or 1");
  if (workspace_bytes < P.bytes)
    return set_error(QSV_ERR_INVALID_ARG, "workspace too small");
  // every variant vector must lie inside the caller's buffer
  uint64_t vi = 0;
  for (int s = 0; s < spec->n_sub; ++s) {
    const uint64_t len = uint64_t(1) << P.subs[s].width;
    for (uint64_t v = 0; v < P.n_variants[s]; ++v, ++vi) {
      const uint64_t o = offsets[vi];
      if (o > probs_elems || len > probs_elems - o)
        return set_error(QSV_ERR_INVALID_ARG,
                         "a variant vector lies outside probs_elems");
    }
  }
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  // tables: subcircuits, variant offsets, term-vector starts
  std::vector<char> host(P.o_T, 0);
  std::memcpy(host.data(), P.subs.data(), sizeof(CutSubDev) * P.subs.size());
  std::memcpy(host.data() + P.o_voff, offsets, 8 * P.total_variants);
  std::memcpy(host.data() + P.o_tt, P.tt.data(), 8 * P.tt.size());
  std::memcpy(host.data() + P.o_ttv, P.ttv.data(), 8 * P.ttv.size());
  std::memcpy(host.data() + P.o_ttu, P.ttu.data(), 8 * P.ttu.size());
  char* ws = static_cast<char*>(workspace);
  hipError_t he = hipMemcpyAsync(ws, host.data(), host.size(),
                                 hipMemcpyHostToDevice, stream);
  if (he == hipSuccess) he = hipStreamSynchronize(stream);
  if (he != hipSuccess)
    return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
  CutArgs a = {};
  a.n_sub = spec->n_sub;
  a.n_cuts = spec->n_cuts;
  a.n_qubits = spec->n_qubits;
  a.probs_fp64 = probs_fp64;
  a.n_terms = P.n_terms;
  a.total_entries = P.total_entries;
  a.subs = reinterpret_cast<const CutSubDev*>(ws);
  a.voff = reinterpret_cast<const uint64_t*>(ws + P.o_voff);
  a.tt = reinterpret_cast<const uint64_t*>(ws + P.o_tt);
  a.T = reinterpret_cast<double*>(ws + P.o_T);
  a.probs = probs_dev;
  a.ttv = reinterpret_cast<const uint64_t*>(ws + P.o_ttv);
  a.ttu = reinterpret_cast<const uint64_t*>(ws + P.o_ttu);
  a.n_vary = int32_t(P.vary.size());
  a.n_uni = int32_t(P.uni.size());
  for (int k = 0; k < a.n_vary; ++k) a.vary_sub[k] = P.vary[k];
  for (int k = 0; k < a.n_uni; ++k) a.uni_sub[k] = P.uni[k];
  a.n_c = P.n_c;
  a.n_u = P.n_u;
  he = launch_cut(a, out_dev, stream);
  if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
  return set_error(QSV_OK, "");
}

}  // extern "C"
