// Batched subcircuit variants: host planning, program upload, autotuning and
// the persistent launch (optionally replayed from a hipGraph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "batch_internal.h"

using namespace qsv;

namespace {

// Standard one-qubit matrices for the cut preparations and readouts.
const double kR2 = 0.70710678118654752440;
const double kX[8] = {0, 0, 1, 0, 1, 0, 0, 0};
const double kH[8] = {kR2, 0, kR2, 0, kR2, 0, -kR2, 0};
const double kS[8] = {1, 0, 0, 0, 0, 0, 0, 1};
const double kSdg[8] = {1, 0, 0, 0, 0, 0, 0, -1};

std::string variant_gates(const qsv_variant& v, std::vector<HostGate>* G) {
  const int w = v.width;
  G->clear();
  auto add1 = [&](int q, const double* m) -> std::string {
    HostGate g;
    int32_t qq = q;
    std::string e = make_gate(w, 1, 0, &qq, m, &g);
    if (e.empty()) G->push_back(std::move(g));
    return e;
  };
  uint64_t seen = 0;
  for (int i = 0; i < v.n_inputs; ++i) {
    const int q = v.input_qubits[i], lab = v.input_labels[i];
    if (q < 0 || q >= w) return "cut-input qubit out of range";
    if (seen >> q & 1) return "duplicate cut-input qubit";
    seen |= uint64_t(1) << q;
    std::string e;
    if (lab == 1) e = add1(q, kX);
    else if (lab == 2) e = add1(q, kH);
    else if (lab == 3) {
      e = add1(q, kH);
      if (e.empty()) e = add1(q, kS);
    } else if (lab != 0) return "cut-input label must be 0..3";
    if (!e.empty()) return e;
  }
  const qsv_circuit& c = v.body;
  if (c.n_gates && (!c.k || !c.c || !c.qubits || !c.matrices))
    return "null body array";
  size_t qo = 0, mo = 0;
  for (size_t i = 0; i < c.n_gates; ++i) {
    HostGate g;
    std::string e = make_gate(w, c.k[i], c.c[i], c.qubits + qo,
                              c.matrices + mo, &g);
    if (!e.empty()) return "gate " + std::to_string(i) + ": " + e;
    qo += size_t(c.k[i] + c.c[i]);
    mo += size_t(2) << (2 * c.k[i]);
    G->push_back(std::move(g));
  }
  seen = 0;
  for (int i = 0; i < v.n_outputs; ++i) {
    const int q = v.output_qubits[i], bas = v.output_bases[i];
    if (q < 0 || q >= w) return "cut-output qubit out of range";
    if (seen >> q & 1) return "duplicate cut-output qubit";
    seen |= uint64_t(1) << q;
    std::string e;
    if (bas == 1) e = add1(q, kH);
    else if (bas == 2) {
      e = add1(q, kSdg);
      if (e.empty()) e = add1(q, kH);
    } else if (bas != 0) return "cut-output basis must be 0..2";
    if (!e.empty()) return e;
  }
  return "";
}

std::string build_program(const qsv_variant* vars, size_t count, int b,
                          int L, int RB, HostProgram* hp) {
  *hp = HostProgram();
  hp->out_offsets.assign(1, 0);
  std::vector<double> cost(count);
  std::vector<HostGate> G;
  for (size_t i = 0; i < count; ++i) {
    const qsv_variant& v = vars[i];
    if (v.width < RB + 2 || v.width > QSV_BATCH_MAX_WIDTH)
      return "variant " + std::to_string(i) + ": width out of range";
    if ((v.n_inputs && (!v.input_qubits || !v.input_labels)) ||
        (v.n_outputs && (!v.output_qubits || !v.output_bases)) ||
        v.n_inputs < 0 || v.n_outputs < 0)
      return "variant " + std::to_string(i) + ": bad cut lists";
    std::string e = variant_gates(v, &G);
    if (!e.empty()) return "variant " + std::to_string(i) + ": " + e;
    e = append_variant(v.width, G, b, L, RB, hp, &cost[i]);
    if (!e.empty()) return "variant " + std::to_string(i) + ": " + e;
  }
  hp->order.resize(count);
  std::iota(hp->order.begin(), hp->order.end(), 0);
  std::stable_sort(hp->order.begin(), hp->order.end(),
                   [&](int a, int c) { return cost[a] > cost[c]; });
  finalize_program(hp);
  return "";
}

}  // namespace

namespace qsv {

std::string append_variant(int w, const std::vector<HostGate>& G, int b,
                           int L, int RB, HostProgram* hp, double* cost) {
  const size_t i = hp->circs.size();
  std::string e;
  {
    PlanOptions po;
    po.strategy = 2;
    po.tile_log2 = std::min(L, w);
    po.low_qubits = std::min(4, po.tile_log2 - 1);
    po.reg_log2 = RB;
    Plan plan;
    make_plan(G, w, b, po, &plan);
    BatchCircuit bc = {};
    bc.w = w;
    bc.pass_begin = int32_t(hp->passes.size());
    for (const Pass& p : plan.passes) {
      if (p.kind != kPassTile)
        return "gate not supported in batched tiles (dense k >= 2)";
      e = emit_tile_pass(p, G, RB, &hp->passes, &hp->segs, &hp->ops);
      if (!e.empty()) return e;
      hp->tiles += uint64_t(1) << (w - p.L);
    }
    bc.n_passes = int32_t(hp->passes.size()) - bc.pass_begin;
    if (bc.n_passes == 0) {
      // an empty variant still needs one pass to write |0...0>'s vector
      Pass p;
      p.kind = kPassTile;
      p.L = std::min(L, w);
      for (int q = 0; q < p.L; ++q) {
        p.q[q] = q;
        p.qubits |= uint64_t(1) << q;
      }
      Pass::Seg sg;
      for (int j = 0; j < RB; ++j) sg.reg_bits[j] = p.L - RB + j;
      p.segs.push_back(sg);
      e = emit_tile_pass(p, G, RB, &hp->passes, &hp->segs, &hp->ops);
      if (!e.empty()) return e;
      hp->tiles += uint64_t(1) << (w - p.L);
      bc.n_passes = 1;
    }
    if (hp->out_offsets.empty()) hp->out_offsets.push_back(0);
    bc.out_offset = hp->out_offsets[i];
    hp->out_offsets.push_back(hp->out_offsets[i] + (uint64_t(1) << w));
    if (bc.n_passes == 1) hp->single_tile++;
    hp->amp_updates += (uint64_t(1) << w) * G.size();
    if (cost)
      *cost = double(uint64_t(1) << w) * (double(G.size()) + 4.0 * bc.n_passes);
    hp->circs.push_back(bc);
  }
  return "";
}

void finalize_program(HostProgram* hp) {
  const size_t n = hp->circs.size();
  std::vector<int32_t> ord = hp->order;
  if (ord.size() != n) {
    ord.resize(n);
    std::iota(ord.begin(), ord.end(), 0);
  }
  // states of multi-pass variants, one after another
  hp->state_amps = 0;
  int phases = 0;
  for (BatchCircuit& c : hp->circs) {
    c.state_offset = 0;
    if (c.n_passes > 1) {
      c.state_offset = hp->state_amps;
      hp->state_amps += uint64_t(1) << c.w;
    }
    phases = std::max(phases, int(c.n_passes));
  }
  // phase p: pass p of every variant that has one, in the given order
  hp->work.clear();
  hp->phase_work_begin.assign(1, 0);
  hp->phase_tiles.clear();
  hp->phase_cost.clear();
  for (int p = 0; p < phases; ++p) {
    uint64_t tiles = 0, cost = 0;
    for (int32_t ci : ord) {
      const BatchCircuit& c = hp->circs[ci];
      if (p >= c.n_passes) continue;
      const TilePass& tp = hp->passes[c.pass_begin + p];
      // a tile's cost: its ops (a phase block as three), plus one per
      // segment change and one for the HBM transfers
      uint32_t ops = 1;
      for (int k = 0; k < tp.nseg; ++k) {
        const TileSeg& sg = hp->segs[tp.seg_begin + k];
        for (int oi = sg.op_begin; oi < sg.op_end; ++oi)
          ops += hp->ops[oi].kind == kOpPhaseBlock ? 3 : 1;
        ops += 1;
      }
      BatchWork wk = {};
      wk.circ = ci;
      wk.tile_cost = ops;
      wk.tile_begin = tiles;
      wk.cost_begin = cost;
      hp->work.push_back(wk);
      const uint64_t nt = uint64_t(1) << (c.w - tp.L);
      tiles += nt;
      cost += nt * ops;
    }
    hp->phase_work_begin.push_back(hp->work.size());
    hp->phase_tiles.push_back(tiles);
    hp->phase_cost.push_back(cost);
  }
}

}  // namespace qsv

namespace {

template <class T>
size_t put(std::vector<char>& buf, const std::vector<T>& v) {
  size_t off = (buf.size() + 255) & ~size_t(255);
  buf.resize(off + sizeof(T) * v.size());
  if (!v.empty()) std::memcpy(buf.data() + off, v.data(), sizeof(T) * v.size());
  return off;
}

}  // namespace

struct qsv_batch_s {
  int prec = 1, b = 8, out_fp64 = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t count = 0;
  int L = 12, RB = 4, grid = 0;
  int user_grid = 0;  // 0: as many work-groups as stay resident
  int cus = 0;
  bool use_graph = false;
  HostProgram hp;
  char* prog = nullptr;
  size_t o_circ = 0, o_work = 0, o_pass = 0, o_seg = 0, o_op = 0;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_out = nullptr;
};

namespace {

void release_device(qsv_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_out = nullptr;
  if (b->prog) (void)hipFree(b->prog);
  if (b->scratch) (void)hipFree(b->scratch);
  b->prog = nullptr;
  b->scratch = nullptr;
}

qsv_status upload_program(qsv_batch b, const qsv_variant* vars, int L, int RB) {
  std::string e = build_program(vars, b->count, b->b, L, RB, &b->hp);
  if (!e.empty()) return set_error(QSV_ERR_INVALID_ARG, e);
  hipError_t he = hipStreamSynchronize(b->stream);
  if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
  release_device(b);
  b->L = L;
  b->RB = RB;
  if (b->user_grid) {
    b->grid = b->user_grid;
  } else {
    const int per_cu = batch_blocks_per_cu(b->prec, b->out_fp64, RB, L);
    b->grid = std::max(1, per_cu) * std::max(1, b->cus);
  }
  std::vector<char> buf;
  b->o_circ = put(buf, b->hp.circs);
  b->o_work = put(buf, b->hp.work);
  b->o_pass = put(buf, b->hp.passes);
  b->o_seg = put(buf, b->hp.segs);
  b->o_op = put(buf, b->hp.ops);
  if (hipMalloc(&b->prog, std::max<size_t>(buf.size(), 256)) != hipSuccess) {
    b->prog = nullptr;
    (void)hipGetLastError();
    return set_error(QSV_ERR_OUT_OF_MEMORY, "batch program allocation failed");
  }
  he = hipMemcpy(b->prog, buf.data(), buf.size(), hipMemcpyHostToDevice);
  if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
  b->scratch_bytes = size_t(b->hp.state_amps) * size_t(b->b);
  if (b->scratch_bytes) {
    if (hipMalloc(&b->scratch, b->scratch_bytes) != hipSuccess) {
      b->scratch = nullptr;
      (void)hipGetLastError();
      return set_error(QSV_ERR_OUT_OF_MEMORY, "batch scratch allocation failed");
    }
  }
  return QSV_OK;
}

hipError_t launch_direct(qsv_batch b, void* out) {
  return launch_batch(
      b->prec, b->out_fp64, b->RB,
      reinterpret_cast<const BatchCircuit*>(b->prog + b->o_circ),
      reinterpret_cast<const TilePass*>(b->prog + b->o_pass),
      reinterpret_cast<const TileSeg*>(b->prog + b->o_seg),
      reinterpret_cast<const TileOp*>(b->prog + b->o_op),
      reinterpret_cast<const BatchWork*>(b->prog + b->o_work), b->hp, out,
      b->scratch, b->L, b->grid, b->stream);
}

}  // namespace

extern "C" {

qsv_status qsv_batch_create(const qsv_variant* vars, size_t count,
                            int32_t prec, const qsv_batch_opts* opts,
                            void* stream, qsv_batch* out) {
  if (!out) return set_error(QSV_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  if (prec != QSV_C64 && prec != QSV_C128)
    return set_error(QSV_ERR_UNSUPPORTED, "unknown precision");
  if (count == 0 || !vars)
    return set_error(QSV_ERR_INVALID_ARG, "empty batch");
  const int b = prec == QSV_C64 ? 8 : 16;
  qsv_batch_opts o = {};
  if (opts) o = *opts;
  int L = o.tile_log2 ? o.tile_log2 : (b == 8 ? 12 : 11);
  int RB = o.reg_log2 ? o.reg_log2 : 4;
  if (L < 8 || L > 12) return set_error(QSV_ERR_INVALID_ARG, "tile_log2 must be 8..12");
  if (RB != 4 && !(RB == 5 && b == 8))
    return set_error(QSV_ERR_INVALID_ARG, "reg_log2 must be 4 (or 5 for c64)");
  if (L - RB > 8) return set_error(QSV_ERR_INVALID_ARG, "tile_log2 - reg_log2 must be <= 8");
  if (o.grid < 0) return set_error(QSV_ERR_INVALID_ARG, "negative grid");
  {  // validate every variant before touching the device
    HostProgram tmp;
    std::string e = build_program(vars, count, b, L, RB, &tmp);
    if (!e.empty()) return set_error(QSV_ERR_INVALID_ARG, e);
  }
  int dev = 0, cus = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he == hipSuccess)
    he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
  qsv_batch bt = new qsv_batch_s;
  bt->prec = prec;
  bt->b = b;
  bt->out_fp64 = o.out_fp64 != 0;
  bt->stream = static_cast<hipStream_t>(stream);
  bt->device = dev;
  bt->count = count;
  bt->user_grid = o.grid;
  bt->cus = cus;
  bt->use_graph = o.use_graph != 0;
  qsv_status st = upload_program(bt, vars, L, RB);
  if (st != QSV_OK) {
    release_device(bt);
    delete bt;
    return st;
  }
  if (o.autotune) {
    // Time each candidate twice on a scratch output and keep the fastest.
    struct Cand { int L, RB; };
    std::vector<Cand> cands = b == 8
        ? std::vector<Cand>{{12, 4}, {11, 4}, {10, 4}, {12, 5}, {11, 5}}
        : std::vector<Cand>{{11, 4}, {10, 4}, {12, 4}};
    void* tmp = nullptr;
    const size_t ob = (bt->out_fp64 ? 8 : 4) * bt->hp.out_offsets[count];
    hipEvent_t e0, e1;
    if (hipMalloc(&tmp, ob) != hipSuccess) {
      (void)hipGetLastError();
      release_device(bt);
      delete bt;
      return set_error(QSV_ERR_OUT_OF_MEMORY, "autotune output allocation failed");
    }
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    Cand pick = {L, RB};
    for (const Cand& c : cands) {
      if (upload_program(bt, vars, c.L, c.RB) != QSV_OK) continue;
      float ms = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, bt->stream);
        if (launch_direct(bt, tmp) != hipSuccess) break;
        (void)hipEventRecord(e1, bt->stream);
        (void)hipEventSynchronize(e1);
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        ms = std::min(ms, t);
      }
      if (ms < best) {
        best = ms;
        pick = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(tmp);
    st = upload_program(bt, vars, pick.L, pick.RB);
    if (st != QSV_OK) {
      release_device(bt);
      delete bt;
      return st;
    }
  }
  *out = bt;
  return QSV_OK;
}

qsv_status qsv_batch_out_offsets(qsv_batch b, uint64_t* offsets) {
  if (!b || !offsets) return set_error(QSV_ERR_INVALID_ARG, "null argument");
  std::copy(b->hp.out_offsets.begin(), b->hp.out_offsets.end(), offsets);
  return QSV_OK;
}

qsv_status qsv_batch_launch(qsv_batch b, void* out_dev) {
  if (!b || !out_dev) return set_error(QSV_ERR_INVALID_ARG, "null argument");
  hipError_t he;
  if (!b->use_graph) {
    he = launch_direct(b, out_dev);
    if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
    return QSV_OK;
  }
  if (!b->exec || b->graph_out != out_dev) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipStream_t cap = nullptr;
    he = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
    he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
      hipStream_t saved = b->stream;
      b->stream = cap;
      hipError_t le = launch_direct(b, out_dev);
      b->stream = saved;
      he = hipStreamEndCapture(cap, &b->graph);
      if (le != hipSuccess) he = le;
    }
    if (he == hipSuccess)
      he = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
    b->graph_out = out_dev;
  }
  he = hipGraphLaunch(b->exec, b->stream);
  if (he != hipSuccess) return set_error(QSV_ERR_DEVICE, hipGetErrorString(he));
  return QSV_OK;
}

qsv_status qsv_batch_stats(qsv_batch b, uint64_t* out, int32_t n) {
  if (!b || !out || n < 0 || n > 10)
    return set_error(QSV_ERR_INVALID_ARG, "bad arguments");
  const uint64_t v[10] = {b->count, b->hp.passes.size(), b->hp.tiles,
                          b->hp.ops.size(), b->scratch_bytes, uint64_t(b->L),
                          uint64_t(b->RB), uint64_t(b->grid), b->hp.single_tile,
                          b->hp.amp_updates};
  for (int i = 0; i < n; ++i) out[i] = v[i];
  return QSV_OK;
}

qsv_status qsv_batch_free(qsv_batch b) {
  if (!b) return QSV_OK;
  (void)hipStreamSynchronize(b->stream);
  release_device(b);
  delete b;
  return QSV_OK;
}

}  // extern "C"
