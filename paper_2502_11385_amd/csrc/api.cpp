// C ABI of libqsv: state lifecycle, argument validation, program upload and
// pass dispatch.  Every argument check runs on the host before any device
// call, so a rejected call leaves the state untouched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "device_common.h"
#include "planner.h"
#include "program.h"
#include "qsv.h"

using namespace qsv;

struct qsv_state_s {
  int n = 0;
  int prec = 0;
  int b = 0;  // bytes per amplitude
  void* amp = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int device = 0;
  bool failed = false;
  // program buffer (device) and its pinned host staging copy
  char* prog_dev = nullptr;
  size_t prog_cap = 0;
  char* prog_host = nullptr;
  size_t host_cap = 0;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  // second state-sized buffer for out-of-place relabelling (on demand)
  void* spare = nullptr;
  // reduction scratch
  char* scratch = nullptr;
  size_t scratch_cap = 0;
  uint64_t stats[13] = {0};
  // per-pass timing
  bool profiling = false;
  std::vector<hipEvent_t> evs;
  std::vector<int32_t> ev_kinds;
  int32_t ev_used = 0;
};

namespace {

thread_local std::string g_err;

qsv_status fail(qsv_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

qsv_status device_fail(qsv_state s, hipError_t e, const char* what) {
  if (s) s->failed = true;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? QSV_ERR_OUT_OF_MEMORY : QSV_ERR_DEVICE;
}

// Failure injection (qsv_debug_inject): counts of allocations and of
// state device calls still to fail.
std::atomic<int> g_inject_alloc{0}, g_inject_call{0};

bool take_injected(std::atomic<int>& c) {
  int v = c.load();
  while (v > 0)
    if (c.compare_exchange_weak(v, v - 1)) return true;
  return false;
}

hipError_t dev_malloc(void** p, size_t bytes) {
  if (take_injected(g_inject_alloc)) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

#define QSV_HIP(s, call)                                             \
  do {                                                               \
    if (take_injected(g_inject_call))                                \
      return device_fail(s, hipErrorLaunchFailure, "injected: " #call); \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) return device_fail(s, e_, #call);          \
  } while (0)

qsv_status check_state(qsv_state s) {
  if (!s) return fail(QSV_ERR_INVALID_ARG, "null state");
  if (s->failed)
    return fail(QSV_ERR_DEVICE, "state is in a failed state after a device error");
  return QSV_OK;
}

qsv_status select_device(qsv_state s) {
  int cur = -1;
  QSV_HIP(s, hipGetDevice(&cur));
  if (cur != s->device) QSV_HIP(s, hipSetDevice(s->device));
  return QSV_OK;
}

int bytes_of(int prec) { return prec == QSV_C64 ? 8 : 16; }

qsv_status ensure_scratch(qsv_state s, size_t bytes) {
  if (bytes <= s->scratch_cap) return QSV_OK;
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  if (s->scratch) QSV_HIP(s, hipFree(s->scratch));
  s->scratch = nullptr;
  s->scratch_cap = 0;
  size_t cap = std::max(bytes, size_t(1) << 16);
  hipError_t e = dev_malloc(reinterpret_cast<void**>(&s->scratch), cap);
  if (e != hipSuccess) {
    s->scratch = nullptr;
    (void)hipGetLastError();
    return fail(QSV_ERR_OUT_OF_MEMORY, "scratch allocation failed");
  }
  s->scratch_cap = cap;
  return QSV_OK;
}

// Copy `bytes` of host data into the state's device program buffer, in
// stream order (kernels already enqueued keep reading the previous
// program until the copy runs).
qsv_status upload(qsv_state s, const void* data, size_t bytes) {
  if (bytes == 0) return QSV_OK;
  if (bytes > s->prog_cap) {
    const size_t old = s->prog_cap;
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    if (s->prog_dev) QSV_HIP(s, hipFree(s->prog_dev));
    s->prog_dev = nullptr;
    s->prog_cap = 0;
    size_t cap = std::max(bytes, std::max(size_t(1) << 16, 2 * old));
    hipError_t e = dev_malloc(reinterpret_cast<void**>(&s->prog_dev), cap);
    if (e != hipSuccess) {
      s->prog_dev = nullptr;
      (void)hipGetLastError();
      return fail(QSV_ERR_OUT_OF_MEMORY, "program buffer allocation failed");
    }
    s->prog_cap = cap;
  }
  if (s->upload_pending) {
    QSV_HIP(s, hipEventSynchronize(s->upload_done));
    s->upload_pending = false;
  }
  if (bytes > s->host_cap) {
    if (s->prog_host) QSV_HIP(s, hipHostFree(s->prog_host));
    s->prog_host = nullptr;
    s->host_cap = 0;
    size_t cap = std::max(bytes, size_t(1) << 16);
    hipError_t e = hipHostMalloc(&s->prog_host, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      s->prog_host = nullptr;
      (void)hipGetLastError();
      return fail(QSV_ERR_OUT_OF_MEMORY, "pinned staging allocation failed");
    }
    s->host_cap = cap;
  }
  std::memcpy(s->prog_host, data, bytes);
  QSV_HIP(s, hipMemcpyAsync(s->prog_dev, s->prog_host, bytes,
                            hipMemcpyHostToDevice, s->stream));
  QSV_HIP(s, hipEventRecord(s->upload_done, s->stream));
  s->upload_pending = true;
  return QSV_OK;
}

qsv_status parse_circuit(const qsv_circuit* circ, int n,
                         std::vector<HostGate>* out) {
  if (!circ) return fail(QSV_ERR_INVALID_ARG, "null circuit");
  out->clear();
  if (circ->n_gates == 0) return QSV_OK;
  if (!circ->k || !circ->c || !circ->qubits || !circ->matrices)
    return fail(QSV_ERR_INVALID_ARG, "null circuit array");
  out->resize(circ->n_gates);
  size_t qo = 0, mo = 0;
  for (size_t i = 0; i < circ->n_gates; ++i) {
    const int k = circ->k[i], c = circ->c[i];
    std::string err = make_gate(n, k, c, circ->qubits + qo,
                                circ->matrices + mo, &(*out)[i]);
    if (!err.empty())
      return fail(QSV_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": " + err);
    qo += size_t(k + c);
    mo += size_t(2) << (2 * k);
  }
  return QSV_OK;
}

template <class T>
size_t put(std::vector<char>& buf, const T* data, size_t count) {
  size_t off = (buf.size() + 255) & ~size_t(255);
  buf.resize(off + sizeof(T) * count);
  if (count) std::memcpy(buf.data() + off, data, sizeof(T) * count);
  return off;
}

}  // namespace

namespace qsv {
// Error reporting shared with the batch and server front ends.
qsv_status set_error(qsv_status st, const std::string& msg) {
  return fail(st, msg);
}

// Draw shots into a device buffer without waiting (used by the server).
qsv_status state_sample_async(qsv_state s, uint64_t shots, uint64_t seed,
                              uint64_t* dev_out) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if ((st = ensure_scratch(s, sample_scratch_bytes(s->n, 0))) != QSV_OK)
    return st;
  QSV_HIP(s, launch_sample(s->prec, s->amp, s->n, shots, seed, s->scratch,
                           dev_out, s->stream));
  return QSV_OK;
}

// Device bytes a state holds: its amplitudes (when the library allocated
// them), program buffer, reduction scratch and relabelling buffer.
size_t state_device_bytes(qsv_state s) {
  if (!s) return 0;
  const size_t amps = size_t(s->b) << s->n;
  return (s->owned ? amps : 0) + s->prog_cap + s->scratch_cap +
         (s->spare ? amps : 0);
}
}  // namespace qsv

// ======================================================================

extern "C" {

const char* qsv_last_error(void) { return g_err.c_str(); }

const char* qsv_version(void) { return "qsv 0.1 (gfx950)"; }

qsv_status qsv_debug_inject(int32_t kind, int32_t count) {
  if (count < 0) return fail(QSV_ERR_INVALID_ARG, "negative count");
  if (kind == 1)
    g_inject_alloc.store(count);
  else if (kind == 2)
    g_inject_call.store(count);
  else
    return fail(QSV_ERR_INVALID_ARG, "kind must be 1 or 2");
  return QSV_OK;
}

qsv_status qsv_alloc(int32_t n, int32_t prec, void* stream, qsv_state* out) {
  if (!out) return fail(QSV_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  if (prec != QSV_C64 && prec != QSV_C128)
    return fail(QSV_ERR_UNSUPPORTED, "unknown precision");
  if (n < 1 || n > QSV_MAX_QUBITS)
    return fail(QSV_ERR_INVALID_ARG, "n_qubits must be 1..34");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(nullptr, e, "hipGetDevice");
  const size_t bytes = size_t(bytes_of(prec)) << n;
  void* p = nullptr;
  e = dev_malloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(QSV_ERR_OUT_OF_MEMORY,
                "state allocation of " + std::to_string(bytes) + " bytes failed");
  }
  qsv_state s = new qsv_state_s;
  s->n = n;
  s->prec = prec;
  s->b = bytes_of(prec);
  s->amp = p;
  s->owned = true;
  s->stream = static_cast<hipStream_t>(stream);
  s->device = dev;
  e = hipEventCreateWithFlags(&s->upload_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipFree(p);
    delete s;
    return device_fail(nullptr, e, "hipEventCreate");
  }
  *out = s;
  return QSV_OK;
}

qsv_status qsv_wrap(int32_t n, int32_t prec, void* ptr, size_t bytes,
                    void* stream, qsv_state* out) {
  if (!out) return fail(QSV_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  if (prec != QSV_C64 && prec != QSV_C128)
    return fail(QSV_ERR_UNSUPPORTED, "unknown precision");
  if (n < 1 || n > QSV_MAX_QUBITS)
    return fail(QSV_ERR_INVALID_ARG, "n_qubits must be 1..34");
  if (!ptr) return fail(QSV_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(ptr) % 16)
    return fail(QSV_ERR_INVALID_ARG, "device pointer not 16-byte aligned");
  if (bytes < (size_t(bytes_of(prec)) << n))
    return fail(QSV_ERR_INVALID_ARG, "buffer smaller than 2^n amplitudes");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(nullptr, e, "hipGetDevice");
  qsv_state s = new qsv_state_s;
  s->n = n;
  s->prec = prec;
  s->b = bytes_of(prec);
  s->amp = ptr;
  s->owned = false;
  s->stream = static_cast<hipStream_t>(stream);
  s->device = dev;
  e = hipEventCreateWithFlags(&s->upload_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete s;
    return device_fail(nullptr, e, "hipEventCreate");
  }
  *out = s;
  return QSV_OK;
}

qsv_status qsv_free(qsv_state s) {
  if (!s) return QSV_OK;
  (void)select_device(s);
  hipError_t e = hipStreamSynchronize(s->stream);
  if (s->owned && s->amp) (void)hipFree(s->amp);
  if (s->prog_dev) (void)hipFree(s->prog_dev);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->spare) (void)hipFree(s->spare);
  if (s->prog_host) (void)hipHostFree(s->prog_host);
  if (s->upload_done) (void)hipEventDestroy(s->upload_done);
  for (hipEvent_t e2 : s->evs) (void)hipEventDestroy(e2);
  delete s;
  if (e != hipSuccess) return device_fail(nullptr, e, "hipStreamSynchronize");
  return QSV_OK;
}

qsv_status qsv_info(qsv_state s, void** ptr, int32_t* n, int32_t* prec) {
  if (!s) return fail(QSV_ERR_INVALID_ARG, "null state");
  if (ptr) *ptr = s->amp;
  if (n) *n = s->n;
  if (prec) *prec = s->prec;
  return QSV_OK;
}

qsv_status qsv_sync(qsv_state s) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if ((st = select_device(s)) != QSV_OK) return st;
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  return QSV_OK;
}

qsv_status qsv_init_basis(qsv_state s, uint64_t index) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (index >= (uint64_t(1) << s->n))
    return fail(QSV_ERR_INVALID_ARG, "basis index >= 2^n");
  if ((st = select_device(s)) != QSV_OK) return st;
  QSV_HIP(s, launch_fill_basis(s->prec, s->amp, s->n, index, s->stream));
  return QSV_OK;
}

// A control-free dense gate as a block for the matrix-core kernel: q gets
// its targets in ascending order (block bit j = j-th smallest target) and
// m its matrix re-indexed to that order.
static void block_matrix(const HostGate& g, int32_t* q,
                         std::vector<double>* m) {
  const int d = 1 << g.k;
  for (int j = 0; j < g.k; ++j) q[j] = g.t[j];
  std::sort(q, q + g.k);
  int pos[kMaxK] = {0};
  for (int i = 0; i < g.k; ++i)
    for (int j = 0; j < g.k; ++j)
      if (q[j] == g.t[i]) pos[i] = j;
  auto perm = [&](int r) {
    int v = 0;
    for (int i = 0; i < g.k; ++i) v |= ((r >> i) & 1) << pos[i];
    return v;
  };
  m->assign(size_t(2) * d * d, 0.0);
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      const size_t src = size_t(2) * (r * d + c);
      const size_t dst = size_t(2) * (perm(r) * d + perm(c));
      (*m)[dst] = g.m[src];
      (*m)[dst + 1] = g.m[src + 1];
    }
}

// Gates that take the matrix-core path when run on their own (controls
// restrict the groups the kernel visits).
static bool block_gate(const HostGate& g) {
  return !g.diagonal && g.k >= 4;
}

qsv_status qsv_apply_gate(qsv_state s, const int32_t* targets, int32_t k,
                          const int32_t* controls, int32_t c,
                          const double* matrix) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (k < 1 || k > QSV_MAX_TARGETS)
    return fail(QSV_ERR_INVALID_ARG, "k must be 1..5");
  if (!targets) return fail(QSV_ERR_INVALID_ARG, "null targets");
  if (c < 0) return fail(QSV_ERR_INVALID_ARG, "negative control count");
  if (c > 0 && !controls) return fail(QSV_ERR_INVALID_ARG, "null controls");
  if (k + c > s->n)
    return fail(QSV_ERR_INVALID_ARG, "too many targets + controls for n");
  std::vector<int32_t> qs(targets, targets + k);
  if (c > 0) qs.insert(qs.end(), controls, controls + c);
  HostGate g;
  std::string err = make_gate(s->n, k, c, qs.data(), matrix, &g);
  if (!err.empty()) return fail(QSV_ERR_INVALID_ARG, err);
  if ((st = select_device(s)) != QSV_OK) return st;
  if (g.diagonal) {
    QSV_HIP(s, launch_diag(s->prec, s->amp, s->n, g, s->stream));
  } else if (block_gate(g)) {
    // 4-5 targets: the matrix-core block kernel of the fused plans (the
    // matrix rounded once to FP32 for complex64), over the groups whose
    // control qubits are 1
    int32_t q[kMaxK];
    std::vector<double> mp;
    block_matrix(g, q, &mp);
    if (s->prec == QSV_C64) {
      std::vector<float> mf(mp.begin(), mp.end());
      if ((st = upload(s, mf.data(), mf.size() * sizeof(float))) != QSV_OK)
        return st;
    } else if ((st = upload(s, mp.data(), mp.size() * sizeof(double))) != QSV_OK) {
      return st;
    }
    QSV_HIP(s, launch_fused_apply(s->prec, s->amp, s->n, g.k, q, s->prog_dev,
                                  g.cmask, s->stream));
  } else if (g.k <= 2) {
    QSV_HIP(s, launch_dense(s->prec, s->amp, s->n, g, nullptr, s->stream));
  } else {
    if ((st = upload(s, g.m.data(), g.m.size() * sizeof(double))) != QSV_OK)
      return st;
    QSV_HIP(s, launch_dense(s->prec, s->amp, s->n, g,
                            reinterpret_cast<const double*>(s->prog_dev),
                            s->stream));
  }
  return QSV_OK;
}

static qsv_status plan_for(const qsv_circuit* circ, int n, int prec,
                           const qsv_fuse_opts* opts,
                           std::vector<HostGate>* G, PlanOptions* po,
                           Plan* plan) {
  qsv_status st = parse_circuit(circ, n, G);
  if (st != QSV_OK) return st;
  int v[5] = {0, 0, 0, 0, 0};
  if (opts) {
    v[0] = opts->strategy;
    v[1] = opts->tile_log2;
    v[2] = opts->k_max;
    v[3] = opts->low_qubits;
    v[4] = opts->reg_log2;
  }
  std::string err = resolve_options(n, bytes_of(prec), v, po);
  if (!err.empty())
    return fail(v[0] < 0 || v[0] > 3 ? QSV_ERR_UNSUPPORTED : QSV_ERR_INVALID_ARG,
                err);
  make_plan(*G, n, bytes_of(prec), *po, plan);
  return QSV_OK;
}

// Outputs requested with qsv_apply_fused_outputs, checked and laid out in
// the state's scratch buffer.  A key's tile-local mask and bit count refer
// to the circuit's last tile pass; fold_* says which outputs that pass
// computes (the others run as separate kernels after the passes).
struct OutPlan {
  const qsv_outputs* o = nullptr;
  bool fold_probs = false, fold_marg = false, fold_shots = false;
  int last_tile = -1;         // index into the tile passes
  uint32_t km = 0, ks = 0;    // key masks (tile-local bits)
  int kbm = 0, kbs = 0;
  size_t off_mpart = 0, off_mout = 0, off_blocks = 0, off_shots = 0,
         off_spart = 0, off_other = 0, total = 0;
};

static qsv_status check_outputs(qsv_state s, const qsv_outputs* o) {
  if (!o) return QSV_OK;
  if (o->probs_fp64 != 0 && o->probs_fp64 != 1)
    return fail(QSV_ERR_INVALID_ARG, "probs_fp64 must be 0 or 1");
  if (o->marg_m < 0 || o->marg_m > 20 || o->marg_m > s->n)
    return fail(QSV_ERR_INVALID_ARG, "marg_m must be 0..min(20, n)");
  if (o->marg_m) {
    if (!o->marg_qubits || !o->marg_out)
      return fail(QSV_ERR_INVALID_ARG, "null marginal argument");
    uint64_t seen = 0;
    for (int l = 0; l < o->marg_m; ++l) {
      const int q = o->marg_qubits[l];
      if (q < 0 || q >= s->n)
        return fail(QSV_ERR_INVALID_ARG, "marginal qubit out of range");
      if (seen >> q & 1)
        return fail(QSV_ERR_INVALID_ARG, "duplicate marginal qubit");
      seen |= uint64_t(1) << q;
    }
  }
  if (o->n_shots > (uint64_t(1) << 32))
    return fail(QSV_ERR_INVALID_ARG, "n_shots must be <= 2^32");
  if (o->n_shots && !o->shots_out)
    return fail(QSV_ERR_INVALID_ARG, "null shots output");
  return QSV_OK;
}

static qsv_status apply_fused_impl(qsv_state s, const qsv_circuit* circ,
                                   const qsv_fuse_opts* opts,
                                   const qsv_outputs* outs);

qsv_status qsv_apply_fused(qsv_state s, const qsv_circuit* circ,
                           const qsv_fuse_opts* opts) {
  return apply_fused_impl(s, circ, opts, nullptr);
}

qsv_status qsv_apply_fused_outputs(qsv_state s, const qsv_circuit* circ,
                                   const qsv_fuse_opts* opts,
                                   const qsv_outputs* outs) {
  if (!outs) return fail(QSV_ERR_INVALID_ARG, "null outputs");
  return apply_fused_impl(s, circ, opts, outs);
}

static qsv_status apply_fused_impl(qsv_state s, const qsv_circuit* circ,
                                   const qsv_fuse_opts* opts,
                                   const qsv_outputs* outs) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if ((st = check_outputs(s, outs)) != QSV_OK) return st;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<HostGate> G;
  PlanOptions po;
  Plan plan;
  if ((st = plan_for(circ, s->n, s->prec, opts, &G, &po, &plan)) != QSV_OK)
    return st;
  const int n = s->n;

  // ---- serialise the program
  std::vector<TilePass> tpasses;
  std::vector<TileSeg> tsegs;
  std::vector<TileOp> tops;
  TileEmitStats est;
  std::vector<FusedBlock> fblocks;
  std::vector<FusedGate> fgates;
  std::vector<double> mats;             // gate matrices (FP64)
  std::vector<int64_t> plain_moff(plan.passes.size(), -1);
  // plain passes run as one-gate matrix-core blocks (k = 0: not one)
  std::vector<FusedBlock> plain_block(plan.passes.size(), FusedBlock{});
  std::vector<float> plain32;  // their FP32 matrices, after the fused ones
  size_t u64_total = 0, u32_total = 0;  // fused outputs (in doubles/floats)

  for (size_t pi = 0; pi < plan.passes.size(); ++pi) {
    const Pass& p = plan.passes[pi];
    if (p.kind == kPassTile) {
      std::string err = emit_tile_pass(p, G, po.reg_log2, &tpasses, &tsegs,
                                       &tops, &est);
      if (!err.empty()) return fail(QSV_ERR_DEVICE, err);
    } else if (p.kind == kPassPlain) {
      const HostGate& g = G[p.gates[0]];
      if (block_gate(g)) {
        // as a single-gate block on the matrix cores, like qsv_apply_gate
        std::vector<double> mp;
        FusedBlock fb = {};
        fb.k = g.k;
        fb.cmask = g.cmask;
        block_matrix(g, fb.q, &mp);
        fb.u64_offset = int64_t(mats.size());
        fb.u32_offset = int64_t(plain32.size());
        mats.insert(mats.end(), mp.begin(), mp.end());
        plain32.insert(plain32.end(), mp.begin(), mp.end());
        plain_block[pi] = fb;
      } else if (!g.diagonal && g.k >= 3) {
        plain_moff[pi] = int64_t(mats.size());
        mats.insert(mats.end(), g.m.begin(), g.m.end());
      }
    } else {
      FusedBlock fb = {};
      fb.k = p.fk;
      fb.n_gates = int32_t(p.gates.size());
      fb.gate_begin = int32_t(fgates.size());
      int local_of[64];
      for (int j = 0; j < p.fk; ++j) {
        fb.q[j] = p.fq[j];
        local_of[p.fq[j]] = j;
      }
      for (int gi : p.gates) {
        const HostGate& g = G[gi];
        FusedGate fg = {};
        fg.k = g.k;
        fg.c = g.c;
        for (int j = 0; j < g.k; ++j) fg.t[j] = local_of[g.t[j]];
        for (int j = 0; j < g.c; ++j) fg.ctl[j] = local_of[g.ctl[j]];
        fg.m_offset = int64_t(mats.size());
        mats.insert(mats.end(), g.m.begin(), g.m.end());
        fgates.push_back(fg);
      }
      const size_t dd = size_t(2) << (2 * p.fk);
      fb.u64_offset = int64_t(u64_total);
      fb.u32_offset = int64_t(u32_total);
      u64_total += dd;
      u32_total += dd;
      fblocks.push_back(fb);
    }
  }
  // Outputs: which ones the last tile pass folds (the last pass of the plan
  // must be a tile pass; a key may span at most L - reg_log2 tile bits, so
  // that each thread's registers fall in one group), and the scratch
  // layout: per-tile partial sums, the marginal, the sampler's block sums
  // and scan, the shots, and the scratch of unfolded reductions.
  OutPlan op;
  op.o = outs;
  if (outs) {
    const bool last_is_tile =
        !plan.passes.empty() && plan.passes.back().kind == kPassTile;
    op.last_tile = last_is_tile ? int(tpasses.size()) - 1 : -1;
    const int L = last_is_tile ? plan.passes.back().L : 0;
    const int RB = po.reg_log2;
    if (last_is_tile) {
      const Pass& lp = plan.passes.back();
      op.fold_probs = outs->probs_dev != nullptr;
      if (outs->marg_m) {
        for (int l = 0; l < outs->marg_m; ++l)
          for (int b = 0; b < L; ++b)
            if (lp.q[b] == outs->marg_qubits[l]) op.km |= 1u << b;
        op.kbm = __builtin_popcount(op.km);
        op.fold_marg = op.kbm <= L - RB;
      }
      if (outs->n_shots && n > 10) {
        for (int b = 0; b < L; ++b)
          if (lp.q[b] >= 10) op.ks |= 1u << b;
        op.kbs = __builtin_popcount(op.ks);
        op.fold_shots = op.kbs <= L - RB;
      }
    }
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 0;
    const uint64_t tiles = last_is_tile ? uint64_t(1) << (n - L) : 0;
    op.off_mpart = off;
    if (op.fold_marg) off = al(off + (tiles << op.kbm) * sizeof(double));
    op.off_mout = off;
    if (outs->marg_m) off = al(off + (sizeof(double) << outs->marg_m));
    op.off_blocks = off;
    if (outs->n_shots) off = al(off + sample_scratch_bytes(n, 0));
    op.off_shots = off;
    if (outs->n_shots) off = al(off + outs->n_shots * sizeof(uint64_t));
    op.off_spart = off;
    if (op.fold_shots) off = al(off + (tiles << op.kbs) * sizeof(double));
    op.off_other = off;
    size_t other = 0;
    if (outs->probs_dev && !op.fold_probs)
      other = std::max(other, norm_scratch_bytes(n));
    if (outs->marg_m && !op.fold_marg)
      other = std::max(other, marginal_scratch_bytes(n, outs->marg_m));
    op.total = off + al(other);
    if ((st = select_device(s)) != QSV_OK) return st;
    if ((st = ensure_scratch(s, op.total)) != QSV_OK) return st;
  }

  // Fused outputs follow the gate matrices in the FP64 region.
  const size_t gate_doubles = mats.size();
  for (auto& fb : fblocks) fb.u64_offset += int64_t(gate_doubles);
  mats.resize(gate_doubles + u64_total, 0.0);
  std::vector<float> mats32(u32_total, 0.0f);
  for (auto& fb : plain_block)
    if (fb.k) fb.u32_offset += int64_t(u32_total);
  mats32.insert(mats32.end(), plain32.begin(), plain32.end());

  std::vector<char> buf;
  const size_t o_tp = put(buf, tpasses.data(), tpasses.size());
  const size_t o_ts = put(buf, tsegs.data(), tsegs.size());
  const size_t o_to = put(buf, tops.data(), tops.size());
  const size_t o_fb = put(buf, fblocks.data(), fblocks.size());
  const size_t o_fg = put(buf, fgates.data(), fgates.size());
  const size_t o_m64 = put(buf, mats.data(), mats.size());
  const size_t o_m32 = put(buf, mats32.data(), mats32.size());
  if (outs && op.last_tile >= 0 &&
      (op.fold_probs || op.fold_marg || op.fold_shots)) {
    // the last tile pass's output record, after everything else
    const TilePass& lp = tpasses[size_t(op.last_tile)];
    const int L = lp.L, RB = po.reg_log2, W = L - RB;
    OutSpec os = {};
    os.probs = op.fold_probs ? uint64_t(uintptr_t(outs->probs_dev)) : 0;
    os.probs_fp64 = outs->probs_fp64;
    auto add_key = [&](uint32_t K, int kb, size_t part_off) {
      const int k = os.n_keys++;
      os.part[k] = uint64_t(uintptr_t(s->scratch + part_off));
      os.key_bits[k] = kb;
      // position term of tile bit c in group-major order
      auto term = [&](int c) -> uint32_t {
        const uint32_t below = (1u << c) - 1;
        return (K >> c & 1) ? 1u << (L - kb + __builtin_popcount(K & below))
                            : 1u << __builtin_popcount(~K & below);
      };
      for (int b = 0; b < W; ++b) os.thr_pos[k][b] = term(b);
      for (int j = 0; j < (1 << RB); ++j) {
        uint32_t v = 0;
        for (int i = 0; i < RB; ++i)
          if (j >> i & 1) v += term(W + i);
        os.reg_pos[k][j] = v;
      }
    };
    if (op.fold_marg) add_key(op.km, op.kbm, op.off_mpart);
    if (op.fold_shots) add_key(op.ks, op.kbs, op.off_spart);
    const size_t o_os = put(buf, &os, 1);
    const size_t o_lp = o_tp + size_t(op.last_tile) * sizeof(TilePass);
    TilePass* hp = reinterpret_cast<TilePass*>(buf.data() + o_lp);
    hp->flags |= kPassOutputs;
    hp->out_spec = int32_t(o_os - o_lp);
    tpasses[size_t(op.last_tile)].flags |= kPassOutputs;
  }
  const auto t1 = std::chrono::steady_clock::now();

  if ((st = select_device(s)) != QSV_OK) return st;
  if ((st = upload(s, buf.data(), buf.size())) != QSV_OK) return st;
  char* dev = s->prog_dev;
  const TilePass* d_tp = reinterpret_cast<const TilePass*>(dev + o_tp);
  const TileSeg* d_ts = reinterpret_cast<const TileSeg*>(dev + o_ts);
  const TileOp* d_to = reinterpret_cast<const TileOp*>(dev + o_to);
  double* d_m64 = reinterpret_cast<double*>(dev + o_m64);
  float* d_m32 = reinterpret_cast<float*>(dev + o_m32);

  if (!fblocks.empty())
    QSV_HIP(s, launch_fused_build(
                   reinterpret_cast<const FusedBlock*>(dev + o_fb),
                   int(fblocks.size()),
                   reinterpret_cast<const FusedGate*>(dev + o_fg), d_m64,
                   d_m32, s->stream));

  if (s->profiling) {
    const size_t need = 2 * plan.passes.size();
    while (s->evs.size() < need) {
      hipEvent_t e2;
      QSV_HIP(s, hipEventCreate(&e2));
      s->evs.push_back(e2);
    }
    s->ev_kinds.assign(plan.passes.size(), 0);
    s->ev_used = int32_t(plan.passes.size());
  } else {
    s->ev_used = 0;
  }
  size_t ti = 0, fi = 0;
  for (size_t pi = 0; pi < plan.passes.size(); ++pi) {
    const Pass& p = plan.passes[pi];
    if (s->profiling) {
      s->ev_kinds[pi] = p.kind;
      QSV_HIP(s, hipEventRecord(s->evs[2 * pi], s->stream));
    }
    if (p.kind == kPassTile) {
      QSV_HIP(s, launch_tile(s->prec, po.reg_log2, s->amp, n, tpasses[ti],
                             d_tp + ti, d_ts, d_to, s->stream));
      ++ti;
    } else if (p.kind == kPassPlain) {
      const HostGate& g = G[p.gates[0]];
      const FusedBlock& pb = plain_block[pi];
      if (g.diagonal) {
        QSV_HIP(s, launch_diag(s->prec, s->amp, n, g, s->stream));
      } else if (pb.k) {
        const void* u = s->prec == QSV_C64
                            ? static_cast<const void*>(d_m32 + pb.u32_offset)
                            : static_cast<const void*>(d_m64 + pb.u64_offset);
        QSV_HIP(s, launch_fused_apply(s->prec, s->amp, n, pb.k, pb.q, u,
                                      pb.cmask, s->stream));
      } else
        QSV_HIP(s, launch_dense(s->prec, s->amp, n, g,
                                plain_moff[pi] >= 0 ? d_m64 + plain_moff[pi]
                                                    : nullptr,
                                s->stream));
    } else {
      const FusedBlock& fb = fblocks[fi++];
      const void* u = (s->prec == QSV_C64 && fb.k >= 4)
                          ? static_cast<const void*>(d_m32 + fb.u32_offset)
                          : static_cast<const void*>(d_m64 + fb.u64_offset);
      QSV_HIP(s, launch_fused_apply(s->prec, s->amp, n, fb.k, fb.q, u,
                                    fb.cmask, s->stream));
    }
    if (s->profiling)
      QSV_HIP(s, hipEventRecord(s->evs[2 * pi + 1], s->stream));
  }
  s->stats[0] = plan.passes.size();
  s->stats[1] = G.size();
  s->stats[2] = plan.alg_bytes;
  s->stats[3] = uint64_t(plan.tile_passes);
  s->stats[4] = uint64_t(plan.plain_passes);
  s->stats[5] = uint64_t(plan.fused_passes);
  s->stats[6] = uint64_t(plan.segments);
  s->stats[7] = uint64_t(
      std::chrono::duration_cast<std::chrono::nanoseconds>(t1 - t0).count());
  s->stats[8] = est.ops;
  s->stats[9] = est.blocks;
  s->stats[10] = est.block_gates;
  s->stats[11] = 0;
  s->stats[12] = uint64_t(std::ldexp(est.flops_per_amp, n) + 0.5);
  if (!outs) return QSV_OK;

  // ---- outputs: finish the folded reductions, run the others
  s->stats[11] = (op.fold_probs ? 1 : 0) | (op.fold_marg ? 2 : 0) |
                 (op.fold_shots ? 4 : 0);
  const Pass* lp = op.last_tile >= 0 ? &plan.passes.back() : nullptr;
  // tile-index bit of each outer qubit of the last tile pass
  int tbit[64];
  if (lp) {
    uint64_t tq = 0;
    for (int b = 0; b < lp->L; ++b) tq |= uint64_t(1) << lp->q[b];
    for (int q = 0, r = 0; q < n; ++q) tbit[q] = (tq >> q & 1) ? -1 : r++;
  }
  auto local_of = [&](int q) -> int {
    for (int b = 0; b < lp->L; ++b)
      if (lp->q[b] == q) return b;
    return -1;
  };
  char* sc = s->scratch;
  if (outs->probs_dev && !op.fold_probs)
    QSV_HIP(s, launch_probs(s->prec, s->amp, n, outs->probs_dev,
                            outs->probs_fp64,
                            reinterpret_cast<double*>(sc + op.off_other),
                            nullptr, s->stream));
  const int m = outs->marg_m;
  double* mout = reinterpret_cast<double*>(sc + op.off_mout);
  if (m && op.fold_marg) {
    MargTileArgs a = {};
    a.m = m;
    a.kb = op.kbm;
    uint64_t used = 0;
    for (int l = 0; l < m; ++l) {
      const int q = outs->marg_qubits[l];
      const int b = local_of(q);
      a.gpos[l] = b >= 0 ? __builtin_popcount(op.km & ((1u << b) - 1)) : -1;
      a.tpos[l] = b >= 0 ? -1 : tbit[q];
      if (b < 0) used |= uint64_t(1) << tbit[q];
    }
    for (int q = 0; q < n; ++q)
      if (tbit[q] >= 0 && !(used >> tbit[q] & 1))
        a.free_pos[a.free_bits++] = tbit[q];
    a.n_enum = uint64_t(1) << a.free_bits;
    QSV_HIP(s, launch_marg_tiles(reinterpret_cast<double*>(sc + op.off_mpart),
                                 a, mout, s->stream));
  } else if (m) {
    QSV_HIP(s, launch_marginal(s->prec, s->amp, n, outs->marg_qubits, m,
                               reinterpret_cast<double*>(sc + op.off_other),
                               mout, s->stream));
  }
  uint64_t* sout = reinterpret_cast<uint64_t*>(sc + op.off_shots);
  if (outs->n_shots && op.fold_shots) {
    BlockTileArgs a = {};
    a.nblocks = uint64_t(1) << (n - 10);
    a.kb = op.kbs;
    a.nhi = n - 10;
    for (int i = 0; i < a.nhi; ++i) {
      const int q = 10 + i;
      const int b = local_of(q);
      a.hi_g[i] = b >= 0 ? __builtin_popcount(op.ks & ((1u << b) - 1)) : -1;
      a.hi_t[i] = b >= 0 ? -1 : tbit[q];
    }
    for (int q = 0; q < 10; ++q)
      if (tbit[q] >= 0) a.free_pos[a.free_bits++] = tbit[q];
    double* P = reinterpret_cast<double*>(sc + op.off_blocks);
    QSV_HIP(s, launch_blocks_tiles(reinterpret_cast<double*>(sc + op.off_spart),
                                   a, P, s->stream));
    QSV_HIP(s, launch_sample_from_blocks(s->prec, s->amp, n, outs->n_shots,
                                         outs->shot_seed, P, sout,
                                         s->stream));
  } else if (outs->n_shots) {
    QSV_HIP(s, launch_sample(s->prec, s->amp, n, outs->n_shots,
                             outs->shot_seed, sc + op.off_blocks, sout,
                             s->stream));
  }
  if (m)
    QSV_HIP(s, hipMemcpyAsync(outs->marg_out, mout, sizeof(double) << m,
                              hipMemcpyDeviceToHost, s->stream));
  if (outs->n_shots)
    QSV_HIP(s, hipMemcpyAsync(outs->shots_out, sout,
                              outs->n_shots * sizeof(uint64_t),
                              hipMemcpyDeviceToHost, s->stream));
  if (m || outs->n_shots) QSV_HIP(s, hipStreamSynchronize(s->stream));
  return QSV_OK;
}

qsv_status qsv_set_profiling(qsv_state s, int32_t enable) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  s->profiling = enable != 0;
  return QSV_OK;
}

qsv_status qsv_pass_times(qsv_state s, float* ms_out, int32_t* kinds_out,
                          int32_t cap, int32_t* count) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!count || cap < 0 || (cap > 0 && !ms_out))
    return fail(QSV_ERR_INVALID_ARG, "bad output arguments");
  if ((st = select_device(s)) != QSV_OK) return st;
  const int32_t m = std::min(cap, s->ev_used);
  if (s->ev_used > 0)
    QSV_HIP(s, hipEventSynchronize(s->evs[2 * (s->ev_used - 1) + 1]));
  for (int32_t i = 0; i < m; ++i) {
    float ms = 0;
    QSV_HIP(s, hipEventElapsedTime(&ms, s->evs[2 * i], s->evs[2 * i + 1]));
    ms_out[i] = ms;
    if (kinds_out) kinds_out[i] = s->ev_kinds[i];
  }
  *count = s->ev_used;
  return QSV_OK;
}

// ---- autotuning of the blocking parameters

namespace {

// Structure of a circuit: what the plan depends on (gate shapes, qubits,
// diagonal form), not the matrix values.  FNV-1a over those fields.
uint64_t circuit_signature(const std::vector<HostGate>& G) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xFF;
      h *= 1099511628211ull;
    }
  };
  mix(G.size());
  for (const HostGate& g : G) {
    mix(uint64_t(g.k) | uint64_t(g.c) << 8 | uint64_t(g.diagonal) << 16 |
        uint64_t(g.masked_phase) << 17);
    for (int i = 0; i < g.k; ++i) mix(uint64_t(g.t[i]));
    for (int i = 0; i < g.c; ++i) mix(uint64_t(g.ctl[i]));
  }
  return h;
}

struct TuneKey {
  int device, n, prec, strategy, k_max;
  uint64_t sig;
  bool operator==(const TuneKey& o) const {
    return device == o.device && n == o.n && prec == o.prec &&
           strategy == o.strategy && k_max == o.k_max && sig == o.sig;
  }
};
struct TuneKeyHash {
  size_t operator()(const TuneKey& k) const {
    return size_t(k.sig ^ (uint64_t(k.n) << 40) ^ (uint64_t(k.prec) << 48) ^
                  (uint64_t(k.device) << 52) ^ (uint64_t(k.strategy) << 56) ^
                  (uint64_t(k.k_max) << 60));
  }
};
struct TuneEntry {
  qsv_fuse_opts best;
  float best_ms, default_ms;
};
std::mutex g_tune_mu;
std::unordered_map<TuneKey, TuneEntry, TuneKeyHash> g_tune;

// Modelled time of a plan (seconds), for ranking candidates before any is
// timed: a tile pass costs the larger of its HBM time and its vector-ALU
// issue time (eight FMA instructions per amplitude and dense op, a
// re-layout per segment, a fixed part), a fused or plain pass its HBM time.
double plan_model_s(const std::vector<HostGate>& G, const Plan& plan, int n,
                    int bytes, const PlanOptions& po) {
  const double state = std::ldexp(double(bytes), n);
  const double hbm = 6.0e12, issue = 1024 * 2.4e9 * 0.85;
  const double amps_per_thread = double(1 << po.reg_log2);
  const double waves = std::ldexp(1.0, n) / amps_per_thread / 64;
  double t = 0;
  for (const Pass& p : plan.passes) {
    double tp = double(p.alg_bytes) / hbm;
    if (p.kind == kPassTile) {
      std::vector<TilePass> tps;
      std::vector<TileSeg> tss;
      std::vector<TileOp> tos;
      TileEmitStats e;
      if (!emit_tile_pass(p, G, po.reg_log2, &tps, &tss, &tos, &e).empty())
        return 1e30;
      const double insts = double(e.ops) * amps_per_thread * 8 * (bytes / 8) +
                           double(p.segs.size() + 1) * amps_per_thread * 6 +
                           250;
      tp = std::max(2 * state / hbm, waves * insts * 4 / issue);
    }
    t += tp + 4e-6;
  }
  return t;
}

}  // namespace

qsv_status qsv_autotune_fused(qsv_state s, const qsv_circuit* circ,
                              const qsv_fuse_opts* base, int32_t max_timed,
                              qsv_fuse_opts* best, float* best_ms,
                              float* default_ms, int32_t* from_cache) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!best) return fail(QSV_ERR_INVALID_ARG, "null best");
  if (max_timed < 0 || max_timed > 64)
    return fail(QSV_ERR_INVALID_ARG, "max_timed must be 0..64");
  if (max_timed == 0) max_timed = 6;
  std::vector<HostGate> G;
  if ((st = parse_circuit(circ, s->n, &G)) != QSV_OK) return st;
  qsv_fuse_opts b0 = {};
  if (base) {
    b0.strategy = base->strategy;
    b0.k_max = base->k_max;
  }
  PlanOptions pdef;
  {
    int v[5] = {b0.strategy, 0, b0.k_max, 0, 0};
    std::string err = resolve_options(s->n, s->b, v, &pdef);
    if (!err.empty())
      return fail(b0.strategy < 0 || b0.strategy > 3 ? QSV_ERR_UNSUPPORTED
                                                     : QSV_ERR_INVALID_ARG,
                  err);
  }
  const TuneKey key{s->device, s->n, s->prec, pdef.strategy, pdef.k_max,
                    circuit_signature(G)};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *best = it->second.best;
      if (best_ms) *best_ms = it->second.best_ms;
      if (default_ms) *default_ms = it->second.default_ms;
      if (from_cache) *from_cache = 1;
      return QSV_OK;
    }
  }
  // candidates: the defaults first, then every valid (tile_log2,
  // low_qubits, reg_log2) ranked by the model; the plain and fused
  // strategies have no tile parameters to choose
  struct Cand {
    qsv_fuse_opts o;
    double model;
  };
  std::vector<Cand> cands;
  const qsv_fuse_opts def = {pdef.strategy, pdef.tile_log2, pdef.k_max,
                             pdef.low_qubits, pdef.reg_log2};
  cands.push_back({def, 0});
  if (pdef.strategy == QSV_PLAN_AUTO || pdef.strategy == QSV_PLAN_TILED) {
    std::vector<Cand> more;
    for (int L = 10; L <= 13; ++L)
      for (int rb = 3; rb <= 5; ++rb)
        for (int low = 2; low <= 6; ++low) {
          const int v[5] = {pdef.strategy, L, pdef.k_max, low, rb};
          PlanOptions po;
          if (!resolve_options(s->n, s->b, v, &po).empty()) continue;
          if (L == pdef.tile_log2 && rb == pdef.reg_log2 &&
              low == pdef.low_qubits)
            continue;
          Plan plan;
          make_plan(G, s->n, s->b, po, &plan);
          more.push_back({{pdef.strategy, L, pdef.k_max, low, rb},
                          plan_model_s(G, plan, s->n, s->b, po)});
        }
    std::sort(more.begin(), more.end(),
              [](const Cand& a, const Cand& c) { return a.model < c.model; });
    for (size_t i = 0; i < more.size() && int(cands.size()) < max_timed; ++i)
      cands.push_back(more[i]);
  }
  // time each candidate once (kernel time of its passes, HIP events), after
  // one untimed run of the defaults; the state's contents are overwritten
  const bool prof = s->profiling;
  s->profiling = true;
  std::vector<float> ms(cands.size(), 0.0f);
  for (size_t i = 0; i <= cands.size() && st == QSV_OK; ++i) {
    const qsv_fuse_opts& o = cands[i == 0 ? 0 : i - 1].o;
    st = apply_fused_impl(s, circ, &o, nullptr);
    if (st != QSV_OK || i == 0) continue;
    std::vector<float> pm(size_t(std::max(s->ev_used, 1)));
    int32_t cnt = 0;
    st = qsv_pass_times(s, pm.data(), nullptr, int32_t(pm.size()), &cnt);
    float tot = 0;
    for (int32_t j = 0; j < cnt; ++j) tot += pm[size_t(j)];
    ms[i - 1] = tot;
  }
  s->profiling = prof;
  if (st != QSV_OK) return st;
  // the defaults stay unless a candidate is at least 2 % faster
  size_t bi = 0;
  for (size_t i = 1; i < cands.size(); ++i)
    if (ms[i] < ms[bi] && ms[i] < 0.98f * ms[0]) bi = i;
  const TuneEntry e{cands[bi].o, ms[bi], ms[0]};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = e;
  }
  *best = e.best;
  if (best_ms) *best_ms = e.best_ms;
  if (default_ms) *default_ms = e.default_ms;
  if (from_cache) *from_cache = 0;
  return QSV_OK;
}

qsv_status qsv_last_plan_stats(qsv_state s, uint64_t* out, int32_t n_out) {
  if (!s) return fail(QSV_ERR_INVALID_ARG, "null state");
  if (!out || n_out < 0 || n_out > 13)
    return fail(QSV_ERR_INVALID_ARG, "bad stats buffer");
  for (int i = 0; i < n_out; ++i) out[i] = s->stats[i];
  return QSV_OK;
}

qsv_status qsv_plan_describe(const qsv_circuit* circ, int32_t n, int32_t prec,
                             const qsv_fuse_opts* opts, int32_t* gate_pass,
                             int32_t* gate_order, int32_t* pass_kind,
                             uint64_t* pass_qubits, int32_t* n_passes) {
  if (prec != QSV_C64 && prec != QSV_C128)
    return fail(QSV_ERR_UNSUPPORTED, "unknown precision");
  if (n < 1 || n > QSV_MAX_QUBITS)
    return fail(QSV_ERR_INVALID_ARG, "n_qubits must be 1..34");
  if (!n_passes) return fail(QSV_ERR_INVALID_ARG, "null n_passes");
  std::vector<HostGate> G;
  PlanOptions po;
  Plan plan;
  qsv_status st = plan_for(circ, n, prec, opts, &G, &po, &plan);
  if (st != QSV_OK) return st;
  if (!G.empty() && (!gate_pass || !gate_order || !pass_kind || !pass_qubits))
    return fail(QSV_ERR_INVALID_ARG, "null output array");
  size_t j = 0;
  for (size_t pi = 0; pi < plan.passes.size(); ++pi) {
    const Pass& p = plan.passes[pi];
    pass_kind[pi] = p.kind;
    pass_qubits[pi] = p.qubits;
    for (int gi : p.gates) {
      gate_pass[gi] = int32_t(pi);
      gate_order[j++] = gi;
    }
  }
  *n_passes = int32_t(plan.passes.size());
  return QSV_OK;
}

qsv_status qsv_plan_program_stats(const qsv_circuit* circ, int32_t n,
                                  int32_t prec, const qsv_fuse_opts* opts,
                                  uint64_t* out, int32_t n_out) {
  if (prec != QSV_C64 && prec != QSV_C128)
    return fail(QSV_ERR_UNSUPPORTED, "unknown precision");
  if (n < 1 || n > QSV_MAX_QUBITS)
    return fail(QSV_ERR_INVALID_ARG, "n_qubits must be 1..34");
  if (!out || n_out < 0 || n_out > 7)
    return fail(QSV_ERR_INVALID_ARG, "bad stats buffer");
  std::vector<HostGate> G;
  PlanOptions po;
  Plan plan;
  qsv_status st = plan_for(circ, n, prec, opts, &G, &po, &plan);
  if (st != QSV_OK) return st;
  std::vector<TilePass> tp;
  std::vector<TileSeg> ts;
  std::vector<TileOp> to;
  TileEmitStats est;
  for (const Pass& p : plan.passes) {
    if (p.kind != kPassTile) continue;
    std::string err = emit_tile_pass(p, G, po.reg_log2, &tp, &ts, &to, &est);
    if (!err.empty()) return fail(QSV_ERR_DEVICE, err);
  }
  const uint64_t v[7] = {plan.passes.size(), tp.size(), ts.size(), est.ops,
                         est.blocks, est.block_gates,
                         uint64_t(std::ldexp(est.flops_per_amp, n) + 0.5)};
  for (int i = 0; i < n_out; ++i) out[i] = v[i];
  return QSV_OK;
}

qsv_status qsv_debug_emulate_tiled(const qsv_circuit* circ, int32_t n,
                                   const qsv_fuse_opts* opts, double* state) {
  if (n < 6 || n > 16) return fail(QSV_ERR_INVALID_ARG, "n must be 6..16");
  if (!state) return fail(QSV_ERR_INVALID_ARG, "null state");
  qsv_fuse_opts o = {};
  if (opts) o = *opts;
  o.strategy = QSV_PLAN_TILED;
  std::vector<HostGate> G;
  PlanOptions po;
  Plan plan;
  // the complex64 option set (it allows reg_log2 = 5); the host
  // execution below is complex128 either way
  qsv_status st = plan_for(circ, n, QSV_C64, &o, &G, &po, &plan);
  if (st != QSV_OK) return st;
  const uint64_t dim = uint64_t(1) << n;
  auto C = [&](uint64_t i) { return std::complex<double>(state[2 * i], state[2 * i + 1]); };
  auto put = [&](uint64_t i, std::complex<double> v) {
    state[2 * i] = v.real();
    state[2 * i + 1] = v.imag();
  };
  for (const Pass& p : plan.passes) {
    if (p.kind != kPassTile) {  // plain gate: apply directly
      const HostGate& g = G[p.gates[0]];
      const int d = 1 << g.k;
      std::vector<std::complex<double>> v(d);
      for (uint64_t i = 0; i < dim; ++i) {
        if ((i & g.tmask) || (i & g.cmask) != g.cmask) continue;
        std::vector<uint64_t> idx(d);
        for (int r = 0; r < d; ++r) {
          uint64_t x = i;
          for (int j = 0; j < g.k; ++j)
            if (r >> j & 1) x |= uint64_t(1) << g.t[j];
          idx[r] = x;
          v[r] = C(x);
        }
        for (int r = 0; r < d; ++r) {
          std::complex<double> acc = 0;
          for (int c = 0; c < d; ++c)
            acc += std::complex<double>(g.m[2 * (r * d + c)],
                                        g.m[2 * (r * d + c) + 1]) * v[c];
          put(idx[r], acc);
        }
      }
      continue;
    }
    std::vector<TilePass> tp;
    std::vector<TileSeg> ts;
    std::vector<TileOp> to;
    std::string err = emit_tile_pass(p, G, po.reg_log2, &tp, &ts, &to);
    if (!err.empty()) return fail(QSV_ERR_DEVICE, err);
    const int L = p.L;
    const uint64_t tiles = uint64_t(1) << (n - L);
    for (uint64_t tix = 0; tix < tiles; ++tix) {
      uint64_t base = tix;
      for (int b = 0; b < L; ++b) {
        const int q = p.q[b];
        base = ((base >> q) << (q + 1)) | (base & ((uint64_t(1) << q) - 1));
      }
      auto gidx = [&](uint32_t r) {
        uint64_t x = base;
        for (int b = 0; b < L; ++b)
          if (r >> b & 1) x |= uint64_t(1) << p.q[b];
        return x;
      };
      for (const TileSeg& sg : ts) {
        for (int oi = sg.op_begin; oi < sg.op_end; ++oi) {
          const TileOp& op = to[oi];
          // the kernels trust mux_reg to name the mux bit's register
          const bool mux_in_reg = op.kind == kOpDense1 && op.mux >= 0 &&
                                  [&] {
                                    for (int i = 0; i < po.reg_log2; ++i)
                                      if (sg.reg_bits[i] == op.mux) return true;
                                    return false;
                                  }();
          if ((op.mux_reg >= 0) != mux_in_reg ||
              (op.mux_reg >= 0 && sg.reg_bits[op.mux_reg] != op.mux))
            return fail(QSV_ERR_DEVICE, "tile op has an inconsistent mux_reg");
          // the ops run by their dispatch codes, as the kernels run them
          const int cls = op.code >> 3, creg = op.code & 7;
          const bool dense = cls <= kCodeCtrlMux;
          if (dense != (op.kind == kOpDense1) ||
              (dense && (creg != op.reg || creg >= po.reg_log2)) ||
              (cls == kCodePhase && op.kind != kOpPhase) ||
              (cls == kCodeDiag && op.kind != kOpDiag) ||
              (cls == kCodePhaseBlock && op.kind != kOpPhaseBlock) ||
              ((cls == kCodeUniform || cls == kCodeRegMux ||
                cls == kCodeThreadMux) && op.lctrl != 0) ||
              ((cls == kCodeUniform || cls == kCodeCtrl) &&
               (op.arg < 0 || op.arg > 63)) ||
              (cls == kCodeRegMux &&
               (op.arg < 0 || op.arg >= po.reg_log2 || op.arg == creg)) ||
              (cls == kCodeThreadMux &&
               [&] {  // a thread bit: no register bit of the segment
                 for (int i = 0; i < po.reg_log2; ++i)
                   if (sg.reg_bits[i] == op.arg) return true;
                 return op.arg < 0 || op.arg >= L;
               }()))
            return fail(QSV_ERR_DEVICE, "tile op has an inconsistent code");
          if ((base & op.gctrl) != op.gctrl) continue;
          for (uint32_t r = 0; r < (1u << L); ++r) {
            if ((r & op.lctrl) != op.lctrl) continue;
            if (dense) {
              const int tb = sg.reg_bits[creg];
              if (r >> tb & 1) continue;
              const uint32_t r1 = r | (1u << tb);
              bool second = false;
              if (cls == kCodeUniform || cls == kCodeCtrl)
                second = (base >> op.arg) & 1;
              else if (cls == kCodeRegMux)
                second = (r >> sg.reg_bits[op.arg]) & 1;
              else
                second = (r >> op.arg) & 1;
              const double* m = second ? op.m2 : op.m;
              const std::complex<double> x0 = C(gidx(r)), x1 = C(gidx(r1));
              const std::complex<double> m00(m[0], m[1]), m01(m[2], m[3]),
                  m10(m[4], m[5]), m11(m[6], m[7]);
              put(gidx(r), m00 * x0 + m01 * x1);
              put(gidx(r1), m10 * x0 + m11 * x1);
            } else if (op.kind == kOpPhaseBlock) {
              const int RB = po.reg_log2;
              const PhaseBlock* pb = reinterpret_cast<const PhaseBlock*>(
                  reinterpret_cast<const char*>(&op) + op.blob);
              const PhaseTerm* t = reinterpret_cast<const PhaseTerm*>(pb + 1);
              uint32_t regmask = 0, j = 0;
              for (int i = 0; i < RB; ++i) {
                regmask |= 1u << sg.reg_bits[i];
                j |= ((r >> sg.reg_bits[i]) & 1u) << i;
              }
              const uint32_t thr = r & ~regmask;
              uint64_t sum = 0;
              for (int k = 0; k <= RB; ++k) {
                const bool reg_on = k == 0 || (j >> (k - 1) & 1);
                for (int i = 0; i < pb->n_uni[k] + pb->n_thr[k]; ++i, ++t) {
                  if ((t->tmask == 0) != (i < pb->n_uni[k]) || (t->tmask & regmask))
                    return fail(QSV_ERR_DEVICE, "inconsistent phase block");
                  if (reg_on && (base & t->gmask) == t->gmask &&
                      (thr & t->tmask) == t->tmask)
                    sum += t->turns;
                }
              }
              const double ang = std::ldexp(double(sum), -64) * 2.0 * M_PI;
              std::complex<double> f(std::cos(ang), std::sin(ang));
              if (pb->has_table)
                f *= std::complex<double>(pb->td[2 * j], pb->td[2 * j + 1]);
              put(gidx(r), C(gidx(r)) * f);
            } else if (op.kind == kOpPhase) {
              put(gidx(r), C(gidx(r)) * std::complex<double>(op.m[0], op.m[1]));
            } else {
              auto bit = [&](int db) -> int {
                return db >= 0 ? int(r >> db & 1) : int(base >> (-1 - db) & 1);
              };
              int e = bit(op.dbit0);
              if (op.arg > 1) e |= bit(op.dbit1) << 1;
              put(gidx(r), C(gidx(r)) *
                               std::complex<double>(op.m[2 * e], op.m[2 * e + 1]));
            }
          }
        }
      }
    }
  }
  return QSV_OK;
}

qsv_status qsv_gate_matrix(const char* name, const double* params,
                           int32_t n_params, double* out, int32_t* k_out) {
  if (!name || !out || !k_out)
    return fail(QSV_ERR_INVALID_ARG, "null argument");
  const std::string nm(name);
  auto need = [&](int cnt) -> bool { return n_params >= cnt && (cnt == 0 || params); };
  double m[8] = {1, 0, 0, 0, 0, 0, 1, 0};
  const double r2 = std::sqrt(0.5);
  if (nm == "id") {
  } else if (nm == "h") {
    double v[8] = {r2, 0, r2, 0, r2, 0, -r2, 0};
    std::memcpy(m, v, sizeof m);
  } else if (nm == "x") {
    double v[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    std::memcpy(m, v, sizeof m);
  } else if (nm == "y") {
    double v[8] = {0, 0, 0, -1, 0, 1, 0, 0};
    std::memcpy(m, v, sizeof m);
  } else if (nm == "z") {
    m[6] = -1;
  } else if (nm == "s") {
    m[6] = 0;
    m[7] = 1;
  } else if (nm == "sdg") {
    m[6] = 0;
    m[7] = -1;
  } else if (nm == "p") {
    if (!need(1)) return fail(QSV_ERR_INVALID_ARG, "p needs 1 parameter");
    m[6] = std::cos(params[0]);
    m[7] = std::sin(params[0]);
  } else if (nm == "u3") {
    if (!need(3)) return fail(QSV_ERR_INVALID_ARG, "u3 needs 3 parameters");
    const double th = params[0], ph = params[1], la = params[2];
    const double c = std::cos(th / 2), sn = std::sin(th / 2);
    // [[c, -e^{i la} s], [e^{i ph} s, e^{i (ph + la)} c]]
    m[0] = c;
    m[1] = 0;
    m[2] = -std::cos(la) * sn;
    m[3] = -std::sin(la) * sn;
    m[4] = std::cos(ph) * sn;
    m[5] = std::sin(ph) * sn;
    m[6] = std::cos(ph + la) * c;
    m[7] = std::sin(ph + la) * c;
  } else {
    return fail(QSV_ERR_UNSUPPORTED, "unknown gate name " + nm);
  }
  std::memcpy(out, m, sizeof m);
  *k_out = 1;
  return QSV_OK;
}

qsv_status qsv_gate_matrices(const char* name, const double* params,
                             int32_t n_params, size_t count, double* out) {
  if (!out || (count && n_params > 0 && !params))
    return fail(QSV_ERR_INVALID_ARG, "null argument");
  if (n_params < 0) return fail(QSV_ERR_INVALID_ARG, "negative n_params");
  int32_t k = 0;
  for (size_t i = 0; i < count; ++i) {
    qsv_status st = qsv_gate_matrix(
        name, n_params ? params + i * size_t(n_params) : nullptr, n_params,
        out + 8 * i, &k);
    if (st != QSV_OK) return st;
  }
  return QSV_OK;
}

qsv_status qsv_probabilities(qsv_state s, void* out_dev, int32_t out_fp64) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!out_dev) return fail(QSV_ERR_INVALID_ARG, "null output buffer");
  if ((st = select_device(s)) != QSV_OK) return st;
  if ((st = ensure_scratch(s, norm_scratch_bytes(s->n))) != QSV_OK) return st;
  QSV_HIP(s, launch_probs(s->prec, s->amp, s->n, out_dev, out_fp64 != 0,
                          reinterpret_cast<double*>(s->scratch), nullptr,
                          s->stream));
  return QSV_OK;
}

static qsv_status norm_dev(qsv_state s, double** where) {
  const size_t part = norm_scratch_bytes(s->n);
  qsv_status st = ensure_scratch(s, part + 256);
  if (st != QSV_OK) return st;
  double* nd = reinterpret_cast<double*>(s->scratch + ((part + 255) & ~size_t(255)));
  QSV_HIP(s, launch_probs(s->prec, s->amp, s->n, nullptr, 1,
                          reinterpret_cast<double*>(s->scratch), nd,
                          s->stream));
  *where = nd;
  return QSV_OK;
}

qsv_status qsv_norm(qsv_state s, double* out) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!out) return fail(QSV_ERR_INVALID_ARG, "null output");
  if ((st = select_device(s)) != QSV_OK) return st;
  double* nd = nullptr;
  if ((st = norm_dev(s, &nd)) != QSV_OK) return st;
  QSV_HIP(s, hipMemcpyAsync(out, nd, sizeof(double), hipMemcpyDeviceToHost,
                            s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  return QSV_OK;
}

qsv_status qsv_renormalize(qsv_state s, double* norm_out) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if ((st = select_device(s)) != QSV_OK) return st;
  double* nd = nullptr;
  if ((st = norm_dev(s, &nd)) != QSV_OK) return st;
  double h = 0;
  QSV_HIP(s, hipMemcpyAsync(&h, nd, sizeof(double), hipMemcpyDeviceToHost,
                            s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  if (!(h > 0.0) || !std::isfinite(h))
    return fail(QSV_ERR_INVALID_ARG, "state norm is zero or not finite");
  QSV_HIP(s, launch_scale(s->prec, s->amp, s->n, nd, s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  if (norm_out) *norm_out = h;
  return QSV_OK;
}

qsv_status qsv_renormalize_noalloc(qsv_state s, double* norm_out) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  const size_t part = (norm_scratch_bytes(s->n) + 255) & ~size_t(255);
  if (part + sizeof(double) > fixed_scratch_bytes())
    return fail(QSV_ERR_INVALID_ARG,
                "state too large for the fixed scratch (at most 30 qubits)");
  if ((st = select_device(s)) != QSV_OK) return st;
  void* base = nullptr;
  QSV_HIP(s, fixed_scratch(s->device, &base));
  double* pairs = static_cast<double*>(base);
  double* nd = reinterpret_cast<double*>(static_cast<char*>(base) + part);
  QSV_HIP(s, launch_probs(s->prec, s->amp, s->n, nullptr, 1, pairs, nd,
                          s->stream));
  double h = 0;
  QSV_HIP(s, hipMemcpyAsync(&h, nd, sizeof(double), hipMemcpyDeviceToHost,
                            s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  if (!(h > 0.0) || !std::isfinite(h))
    return fail(QSV_ERR_INVALID_ARG, "state norm is zero or not finite");
  QSV_HIP(s, launch_scale(s->prec, s->amp, s->n, nd, s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  if (norm_out) *norm_out = h;
  return QSV_OK;
}

// -------------------------------------------------- qubit relabelling

qsv_status qsv_permute_qubits(qsv_state s, const int32_t* perm) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!perm) return fail(QSV_ERR_INVALID_ARG, "null permutation");
  const int n = s->n;
  std::vector<int> inv(n, -1);
  for (int q = 0; q < n; ++q) {
    if (perm[q] < 0 || perm[q] >= n || inv[perm[q]] >= 0)
      return fail(QSV_ERR_INVALID_ARG, "perm must be a permutation of 0..n-1");
    inv[perm[q]] = q;
  }
  bool identity = true;
  for (int q = 0; q < n; ++q) identity = identity && perm[q] == q;
  if (identity) return QSV_OK;
  if ((st = select_device(s)) != QSV_OK) return st;
  // tile source bits: the m lowest, and those that land on the m lowest
  const int m = std::min(n, s->b == 8 ? 5 : 4);
  uint64_t smask = 0;
  for (int q = 0; q < m; ++q) smask |= (uint64_t(1) << q) | (uint64_t(1) << inv[q]);
  PermArgs pa = {};
  pa.m = m;
  for (int q = 0; q < n; ++q)
    if (smask >> q & 1) pa.s_bits[pa.s++] = q;
    else {
      pa.outer_src[pa.n_outer] = q;
      pa.outer_dst[pa.n_outer++] = perm[q];
    }
  std::vector<int> d(pa.s_bits, pa.s_bits + pa.s);
  for (int& x : d) x = perm[x];
  std::sort(d.begin(), d.end());
  for (int j = 0; j < pa.s; ++j) {
    pa.d_bits[j] = d[j];
    const int q = inv[d[j]];
    for (int k = 0; k < pa.s; ++k)
      if (pa.s_bits[k] == q) pa.src_of[j] = k;
  }
  // uniform per-step parts of the tile index maps (see the kernel)
  const uint32_t step = std::min(256u, 1u << pa.s);
  pa.ne = int32_t((1u << pa.s) / step);
  for (int e = 0; e < pa.ne; ++e) {
    const uint32_t r = uint32_t(e) * step;
    uint64_t sv = 0, dv = 0;
    uint32_t gv = 0;
    for (int j = 0; j < pa.s; ++j) {
      const uint32_t bit = (r >> j) & 1u;
      sv |= uint64_t(bit) << pa.s_bits[j];
      dv |= uint64_t(bit) << pa.d_bits[j];
      gv |= bit << pa.src_of[j];
    }
    pa.se[e] = sv;
    pa.de[e] = dv;
    pa.ge[e] = gv;
  }
  const size_t bytes = size_t(s->b) << n;
  if (!s->spare) {
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    hipError_t e = dev_malloc(&s->spare, bytes);
    if (e != hipSuccess) {
      s->spare = nullptr;
      (void)hipGetLastError();
      return fail(QSV_ERR_OUT_OF_MEMORY, "no room for the relabelling buffer");
    }
  }
  QSV_HIP(s, launch_permute(s->prec, s->amp, s->spare, n, pa, s->stream));
  if (s->owned) {
    std::swap(s->amp, s->spare);
  } else {
    QSV_HIP(s, hipMemcpyAsync(s->amp, s->spare, bytes, hipMemcpyDeviceToDevice,
                              s->stream));
  }
  return QSV_OK;
}

// ------------------------------------------------------------- top-k

qsv_status qsv_top_k(qsv_state s, uint32_t k, uint64_t* idx_out,
                     double* p_out) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!idx_out || !p_out) return fail(QSV_ERR_INVALID_ARG, "null argument");
  const uint64_t count = uint64_t(1) << s->n;
  if (k < 1 || k > 65536 || uint64_t(k) > count)
    return fail(QSV_ERR_INVALID_ARG, "k must be 1..min(65536, 2^n)");
  if ((st = select_device(s)) != QSV_OK) return st;
  // scratch: histogram, counter, k keys, k indices, tie counts/offsets
  const unsigned tie_blocks = 1024;
  const uint64_t chunk = (count + tie_blocks - 1) / tie_blocks;
  const size_t o_cnt = 4096 * 8, o_key = o_cnt + 256, o_idx = o_key + 8 * size_t(k);
  const size_t o_tc = (o_idx + 8 * size_t(k) + 255) & ~size_t(255);
  const size_t o_to = o_tc + 8 * tie_blocks;
  if ((st = ensure_scratch(s, o_to + 8 * tie_blocks)) != QSV_OK) return st;
  char* sc = s->scratch;
  auto* hist = reinterpret_cast<unsigned long long*>(sc);
  auto* counter = reinterpret_cast<unsigned long long*>(sc + o_cnt);
  auto* dkey = reinterpret_cast<uint64_t*>(sc + o_key);
  auto* didx = reinterpret_cast<uint64_t*>(sc + o_idx);
  auto* tcount = reinterpret_cast<unsigned long long*>(sc + o_tc);
  auto* toff = reinterpret_cast<unsigned long long*>(sc + o_to);
  // radix select of the k-th largest key, 12 bits per pass from the top
  uint64_t prefix = 0, mask = 0, need = k, above = 0;
  int fixed = 0;
  bool whole_bin = false;
  std::vector<unsigned long long> h(4096);
  while (fixed < 64) {
    const int wd = std::min(12, 64 - fixed);
    const int shift = 64 - fixed - wd;
    const int bins = 1 << wd;
    QSV_HIP(s, hipMemsetAsync(hist, 0, 8 * size_t(bins), s->stream));
    QSV_HIP(s, launch_topk_hist(s->prec, s->amp, count, mask, prefix, shift,
                                bins, hist, s->stream));
    QSV_HIP(s, hipMemcpyAsync(h.data(), hist, 8 * size_t(bins),
                              hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    uint64_t cum = 0;
    int b = bins - 1;
    for (; b > 0; --b) {
      if (cum + h[b] >= need) break;
      cum += h[b];
    }
    above += cum;
    need -= cum;
    prefix |= uint64_t(b) << shift;
    mask |= uint64_t(bins - 1) << shift;
    fixed += wd;
    if (h[b] == need) {  // the whole bin is taken: keys >= its lower bound
      whole_bin = true;
      break;
    }
  }
  std::vector<uint64_t> keys, idx;
  if (whole_bin) {
    QSV_HIP(s, hipMemsetAsync(counter, 0, 8, s->stream));
    QSV_HIP(s, launch_topk_collect(s->prec, s->amp, count, mask, prefix, 1,
                                   counter, k, dkey, didx, s->stream));
    keys.resize(k);
    idx.resize(k);
    QSV_HIP(s, hipMemcpyAsync(keys.data(), dkey, 8 * size_t(k),
                              hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(s, hipMemcpyAsync(idx.data(), didx, 8 * size_t(k),
                              hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(s, hipStreamSynchronize(s->stream));
  } else {
    // prefix is the exact k-th key: `above` keys exceed it, `need` of the
    // keys equal to it complete the k, in index order
    keys.resize(k);
    idx.resize(k);
    if (above) {
      QSV_HIP(s, hipMemsetAsync(counter, 0, 8, s->stream));
      QSV_HIP(s, launch_topk_collect(s->prec, s->amp, count, ~uint64_t(0),
                                     prefix, 0, counter, above, dkey, didx,
                                     s->stream));
      QSV_HIP(s, hipMemcpyAsync(keys.data(), dkey, 8 * above,
                                hipMemcpyDeviceToHost, s->stream));
      QSV_HIP(s, hipMemcpyAsync(idx.data(), didx, 8 * above,
                                hipMemcpyDeviceToHost, s->stream));
    }
    QSV_HIP(s, launch_topk_ties(s->prec, s->amp, count, prefix, tie_blocks,
                                chunk, tcount, nullptr, 0, nullptr,
                                s->stream));
    std::vector<unsigned long long> tc(tie_blocks), to(tie_blocks);
    QSV_HIP(s, hipMemcpyAsync(tc.data(), tcount, 8 * tie_blocks,
                              hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    unsigned long long run = 0;
    for (unsigned b = 0; b < tie_blocks; ++b) {
      to[b] = run;
      run += tc[b];
    }
    QSV_HIP(s, hipMemcpyAsync(toff, to.data(), 8 * tie_blocks,
                              hipMemcpyHostToDevice, s->stream));
    QSV_HIP(s, launch_topk_ties(s->prec, s->amp, count, prefix, tie_blocks,
                                chunk, tcount, toff, need, didx + above,
                                s->stream));
    QSV_HIP(s, hipMemcpyAsync(idx.data() + above, didx + above, 8 * need,
                              hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(s, hipStreamSynchronize(s->stream));
    for (uint64_t i = above; i < k; ++i) keys[i] = prefix;
  }
  std::vector<uint32_t> ord(k);
  for (uint32_t i = 0; i < k; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) {
    if (keys[x] != keys[y]) return keys[x] > keys[y];
    return idx[x] < idx[y];
  });
  for (uint32_t i = 0; i < k; ++i) {
    idx_out[i] = idx[ord[i]];
    const uint64_t kb = keys[ord[i]];
    std::memcpy(&p_out[i], &kb, 8);
  }
  return QSV_OK;
}

// ------------------------------------------------- Pauli expectations

qsv_status qsv_expectation_pauli(qsv_state s, int32_t n_terms,
                                 const uint64_t* x_masks,
                                 const uint64_t* z_masks, double* out) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (n_terms < 1 || !x_masks || !z_masks || !out)
    return fail(QSV_ERR_INVALID_ARG, "need n_terms >= 1 and non-null arrays");
  const uint64_t full = (s->n >= 64) ? ~uint64_t(0)
                                     : ((uint64_t(1) << s->n) - 1);
  for (int t = 0; t < n_terms; ++t)
    if ((x_masks[t] | z_masks[t]) & ~full)
      return fail(QSV_ERR_INVALID_ARG, "Pauli mask names a qubit >= n");
  if ((st = select_device(s)) != QSV_OK) return st;
  const size_t part = (pauli_scratch_bytes(s->n) + 255) & ~size_t(255);
  const size_t outb = 16 * size_t(n_terms);
  if ((st = ensure_scratch(s, part + outb)) != QSV_OK) return st;
  double* od = reinterpret_cast<double*>(s->scratch + part);
  for (int t = 0; t < n_terms; ++t)
    QSV_HIP(s, launch_pauli(s->prec, s->amp, s->n, x_masks[t], z_masks[t],
                            reinterpret_cast<double*>(s->scratch), od + 2 * t,
                            s->stream));
  std::vector<double> sri(2 * size_t(n_terms));
  QSV_HIP(s, hipMemcpyAsync(sri.data(), od, outb, hipMemcpyDeviceToHost,
                            s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  for (int t = 0; t < n_terms; ++t) {
    const double re = sri[2 * t], im = sri[2 * t + 1];
    switch (__builtin_popcountll(x_masks[t] & z_masks[t]) & 3) {
      case 0: out[t] = re; break;
      case 1: out[t] = -im; break;
      case 2: out[t] = -re; break;
      default: out[t] = im; break;
    }
  }
  return QSV_OK;
}

qsv_status qsv_marginal(qsv_state s, const int32_t* qubits, int32_t m,
                        double* out_host) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!qubits || !out_host) return fail(QSV_ERR_INVALID_ARG, "null argument");
  if (m < 1 || m > 20 || m > s->n)
    return fail(QSV_ERR_INVALID_ARG, "m must be 1..min(20, n)");
  uint64_t seen = 0;
  for (int l = 0; l < m; ++l) {
    if (qubits[l] < 0 || qubits[l] >= s->n)
      return fail(QSV_ERR_INVALID_ARG, "qubit index out of range");
    if (seen >> qubits[l] & 1)
      return fail(QSV_ERR_INVALID_ARG, "duplicate marginal qubit");
    seen |= uint64_t(1) << qubits[l];
  }
  if ((st = select_device(s)) != QSV_OK) return st;
  const size_t part = (marginal_scratch_bytes(s->n, m) + 255) & ~size_t(255);
  const size_t outb = sizeof(double) << m;
  if ((st = ensure_scratch(s, part + outb)) != QSV_OK) return st;
  double* od = reinterpret_cast<double*>(s->scratch + part);
  QSV_HIP(s, launch_marginal(s->prec, s->amp, s->n, qubits, m,
                             reinterpret_cast<double*>(s->scratch), od,
                             s->stream));
  QSV_HIP(s, hipMemcpyAsync(out_host, od, outb, hipMemcpyDeviceToHost,
                            s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  return QSV_OK;
}

qsv_status qsv_sample(qsv_state s, uint64_t shots, uint64_t seed,
                      uint64_t* out_host) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (shots > (uint64_t(1) << 32))
    return fail(QSV_ERR_INVALID_ARG, "n_shots must be <= 2^32");
  if (shots && !out_host) return fail(QSV_ERR_INVALID_ARG, "null output");
  if (shots == 0) return QSV_OK;
  if ((st = select_device(s)) != QSV_OK) return st;
  const size_t head = (sample_scratch_bytes(s->n, 0) + 255) & ~size_t(255);
  if ((st = ensure_scratch(s, head + shots * sizeof(uint64_t))) != QSV_OK)
    return st;
  uint64_t* od = reinterpret_cast<uint64_t*>(s->scratch + head);
  QSV_HIP(s, launch_sample(s->prec, s->amp, s->n, shots, seed, s->scratch, od,
                           s->stream));
  QSV_HIP(s, hipMemcpyAsync(out_host, od, shots * sizeof(uint64_t),
                            hipMemcpyDeviceToHost, s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  return QSV_OK;
}

qsv_status qsv_get_amplitudes(qsv_state s, void* host_out) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!host_out) return fail(QSV_ERR_INVALID_ARG, "null output");
  if ((st = select_device(s)) != QSV_OK) return st;
  QSV_HIP(s, hipMemcpyAsync(host_out, s->amp, size_t(s->b) << s->n,
                            hipMemcpyDeviceToHost, s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  return QSV_OK;
}

qsv_status qsv_set_amplitudes(qsv_state s, const void* host_in) {
  qsv_status st = check_state(s);
  if (st != QSV_OK) return st;
  if (!host_in) return fail(QSV_ERR_INVALID_ARG, "null input");
  if ((st = select_device(s)) != QSV_OK) return st;
  QSV_HIP(s, hipMemcpyAsync(s->amp, host_in, size_t(s->b) << s->n,
                            hipMemcpyHostToDevice, s->stream));
  QSV_HIP(s, hipStreamSynchronize(s->stream));
  return QSV_OK;
}

}  // extern "C"
