// Request server: admission by HBM bytes and continuous batching.
//
// The evaluator of the paper's cutting pipeline sizes its process pool by
// the memory each worker needs and the memory available (Section IV.A).  On
// one GPU the equivalent resource is HBM: a scheduler thread admits queued
// requests first-come first-served while the bytes they need (state plus
// output) fit the budget.  Admitted small requests become slots of one
// persistent batch launch; wide ones get their own state.  Each group runs
// on one of a few streams and is retired by polling its event, so new work
// is admitted and launched while earlier work is still on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_internal.h"

namespace qsv {
qsv_status state_sample_async(qsv_state s, uint64_t shots, uint64_t seed,
                              uint64_t* dev_out);
size_t state_device_bytes(qsv_state s);
}

using namespace qsv;

namespace {

double now_s() {
  return std::chrono::duration<double>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Size class of a pooled block: at least 64 KiB, then eight classes per
// power of two, so a block wastes at most 1/8 of its size.
size_t pool_round(size_t b) {
  size_t p = size_t(1) << 16;
  if (b <= p) return p;
  while (p < b) p <<= 1;        // p / 2 < b <= p
  const size_t step = p >> 4;   // (p / 2) / 8
  return (b + step - 1) / step * step;
}

// Device blocks kept for reuse, so that steady-state serving calls neither
// hipMalloc nor hipFree (both can stall other streams).  Idle blocks are
// counted, and trimmed when admission needs their bytes.
class DevicePool {
 public:
  void* get(size_t bytes) {
    const size_t sz = pool_round(bytes);
    auto& fl = free_[sz];
    if (!fl.empty()) {
      void* p = fl.back();
      fl.pop_back();
      idle_ -= sz;
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void* p, size_t bytes) {
    if (!p) return;
    const size_t sz = pool_round(bytes);
    free_[sz].push_back(p);
    idle_ += sz;
  }
  size_t idle() const { return idle_; }
  void clear() {
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipFree(p);
    free_.clear();
    idle_ = 0;
  }

 private:
  std::map<size_t, std::vector<void*>> free_;
  size_t idle_ = 0;
};

// Used by client threads (results) and the scheduler (staging): locked.
class HostPool {
 public:
  void* get(size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    const size_t sz = pool_round(bytes);
    auto& fl = free_[sz];
    if (!fl.empty()) {
      void* p = fl.back();
      fl.pop_back();
      return p;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void* p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    if (p) free_[pool_round(bytes)].push_back(p);
  }
  void clear() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipHostFree(p);
    free_.clear();
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void*>> free_;
};

struct Req {
  uint64_t ticket = 0;
  int w = 0, prec = 1, b = 8;
  bool samples = false;
  uint64_t shots = 0, seed = 0;
  std::vector<HostGate> G;
  std::vector<int32_t> k, c, q;  // flat copy for the single-state path
  std::vector<double> m;
  bool batched = false;
  size_t need = 0;
  double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  int status = QSV_OK;
  std::string err;
  void* host = nullptr;
  size_t host_bytes = 0;
  uint64_t n_out = 0;
  bool done = false;
};

struct Buf {
  void* p;
  size_t bytes;
  bool host;
};

struct Group {
  int stream_idx = 0;
  hipEvent_t ev = nullptr;
  std::vector<Req*> reqs;
  std::vector<Buf> bufs;
  qsv_state state = nullptr;
  int state_key = -1;
};

}  // namespace

struct qsv_server_s {
  qsv_server_opts o = {};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, Req*> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  // submit-side counters (under mu)
  uint64_t submitted = 0, rejected = 0, completed = 0;
  // scheduler-owned
  bool hip_ready = false;
  int device = 0;
  std::vector<hipStream_t> streams;
  int rr = 0;
  DevicePool dpool;
  HostPool hpool;
  size_t reserved = 0, peak_reserved = 0;
  std::vector<Group*> running;
  std::vector<hipEvent_t> free_events;
  std::map<int, std::vector<qsv_state>> states;  // key: (w, prec, stream)
  size_t idle_state_bytes = 0;  // device bytes of the cached idle states
  uint64_t n_batches = 0, n_single = 0, max_inflight = 0, trims = 0;
  uint64_t cancelled = 0;  // under mu
};

namespace {

int state_key(int w, int prec, int stream) {
  return (w * 4 + prec) * 64 + stream;
}

bool init_hip(qsv_server s, std::string* err) {
  if (s->hip_ready) return true;
  if (hipGetDevice(&s->device) != hipSuccess) {
    *err = "no device";
    return false;
  }
  s->streams.resize(s->o.n_streams);
  for (auto& st : s->streams)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      *err = "stream creation failed";
      return false;
    }
  s->hip_ready = true;
  return true;
}

hipEvent_t take_event(qsv_server s) {
  if (!s->free_events.empty()) {
    hipEvent_t e = s->free_events.back();
    s->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
  return e;
}

template <class T>
size_t put_vec(std::vector<char>& buf, const std::vector<T>& v) {
  size_t off = (buf.size() + 255) & ~size_t(255);
  buf.resize(off + sizeof(T) * v.size());
  if (!v.empty()) std::memcpy(buf.data() + off, v.data(), sizeof(T) * v.size());
  return off;
}

void fail_group(Group* g, const std::string& msg) {
  for (Req* r : g->reqs) {
    r->status = QSV_ERR_DEVICE;
    r->err = msg;
  }
}

// Resident work-groups of the batch kernel on this device (cached).
int batch_grid(int prec, int RB, int L) {
  static int cache[3][6][14] = {};
  int& g = cache[prec][RB][L];
  if (!g) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess) {
      (void)hipGetLastError();
      cus = 1;
    }
    g = std::max(1, batch_blocks_per_cu(prec, prec == QSV_C128, RB, L)) *
        std::max(1, cus);
  }
  return g;
}

// Launch one group of batch-slot requests (same precision).
void launch_batched(qsv_server s, Group* g, int prec) {
  const int b = prec == QSV_C64 ? 8 : 16;
  const int L = b == 8 ? 12 : 11, RB = 4;
  hipStream_t st = s->streams[g->stream_idx];
  HostProgram hp;
  hp.out_offsets.assign(1, 0);
  for (Req* r : g->reqs) {
    std::string e = append_variant(r->w, r->G, b, L, RB, &hp, nullptr);
    if (!e.empty()) {
      fail_group(g, e);
      return;
    }
  }
  finalize_program(&hp);  // variants in submission order
  std::vector<char> img;
  const size_t o_c = put_vec(img, hp.circs), o_w = put_vec(img, hp.work),
               o_p = put_vec(img, hp.passes), o_s = put_vec(img, hp.segs),
               o_op = put_vec(img, hp.ops);
  const int grid = batch_grid(prec, RB, L);
  const size_t outb = size_t(hp.out_offsets.back()) * (b == 8 ? 4 : 8);
  const size_t scrb = size_t(hp.state_amps) * size_t(b);
  void* hstage = s->hpool.get(img.size());
  char* prog = static_cast<char*>(s->dpool.get(img.size()));
  void* out = s->dpool.get(outb);
  void* scr = scrb ? s->dpool.get(scrb) : nullptr;
  g->bufs.push_back({hstage, img.size(), true});
  g->bufs.push_back({prog, img.size(), false});
  g->bufs.push_back({out, outb, false});
  if (scrb) g->bufs.push_back({scr, scrb, false});
  if (!hstage || !prog || !out || (scrb && !scr)) {
    fail_group(g, "out of memory");
    return;
  }
  std::memcpy(hstage, img.data(), img.size());
  hipError_t e = hipMemcpyAsync(prog, hstage, img.size(),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = launch_batch(prec, b == 16, RB,
                     reinterpret_cast<const BatchCircuit*>(prog + o_c),
                     reinterpret_cast<const TilePass*>(prog + o_p),
                     reinterpret_cast<const TileSeg*>(prog + o_s),
                     reinterpret_cast<const TileOp*>(prog + o_op),
                     reinterpret_cast<const BatchWork*>(prog + o_w), hp, out,
                     scr, L, grid, st);
  for (size_t i = 0; i < g->reqs.size() && e == hipSuccess; ++i) {
    Req* r = g->reqs[i];
    const size_t esz = b == 8 ? 4 : 8;
    char* pr = static_cast<char*>(out) + esz * hp.out_offsets[i];
    if (r->samples) {
      const size_t sb = sample_scratch_bytes(r->w, 0);
      void* ss = s->dpool.get(sb + r->shots * 8 + 256);
      g->bufs.push_back({ss, sb + r->shots * 8 + 256, false});
      if (!ss) {
        e = hipErrorOutOfMemory;
        break;
      }
      uint64_t* dsm = reinterpret_cast<uint64_t*>(
          static_cast<char*>(ss) + ((sb + 255) & ~size_t(255)));
      e = launch_sample_probs(b == 16, pr, r->w, r->shots, r->seed, ss, dsm,
                              st);
      if (e == hipSuccess && r->shots)
        e = hipMemcpyAsync(r->host, dsm, r->shots * 8, hipMemcpyDeviceToHost,
                           st);
    } else {
      e = hipMemcpyAsync(r->host, pr, esz << r->w, hipMemcpyDeviceToHost, st);
    }
  }
  if (e != hipSuccess) fail_group(g, hipGetErrorString(e));
  s->n_batches++;
}

// Launch one wide request on its own state.
void launch_single(qsv_server s, Group* g) {
  Req* r = g->reqs[0];
  hipStream_t st = s->streams[g->stream_idx];
  const int key = state_key(r->w, r->prec, g->stream_idx);
  qsv_state state = nullptr;
  auto& fl = s->states[key];
  if (!fl.empty()) {
    state = fl.back();
    fl.pop_back();
    s->idle_state_bytes -= state_device_bytes(state);
  } else if (qsv_alloc(r->w, r->prec, st, &state) != QSV_OK) {
    fail_group(g, qsv_last_error());
    return;
  }
  g->state = state;
  g->state_key = key;
  qsv_circuit circ = {r->k.size(), r->k.data(), r->c.data(), r->q.data(),
                      r->m.data()};
  qsv_status stt = qsv_init_basis(state, 0);
  if (stt == QSV_OK) stt = qsv_apply_fused(state, &circ, nullptr);
  const size_t esz = r->b == 8 ? 4 : 8;
  if (stt == QSV_OK) {
    if (r->samples) {
      void* dsm = s->dpool.get(r->shots * 8 + 8);
      g->bufs.push_back({dsm, r->shots * 8 + 8, false});
      if (!dsm) {
        fail_group(g, "out of memory");
        return;
      }
      stt = state_sample_async(state, r->shots, r->seed,
                               static_cast<uint64_t*>(dsm));
      if (stt == QSV_OK && r->shots &&
          hipMemcpyAsync(r->host, dsm, r->shots * 8, hipMemcpyDeviceToHost,
                         st) != hipSuccess)
        stt = QSV_ERR_DEVICE;
    } else {
      void* dp = s->dpool.get(esz << r->w);
      g->bufs.push_back({dp, esz << r->w, false});
      if (!dp) {
        fail_group(g, "out of memory");
        return;
      }
      stt = qsv_probabilities(state, dp, r->b == 16);
      if (stt == QSV_OK &&
          hipMemcpyAsync(r->host, dp, esz << r->w, hipMemcpyDeviceToHost,
                         st) != hipSuccess)
        stt = QSV_ERR_DEVICE;
    }
  }
  if (stt != QSV_OK) fail_group(g, qsv_last_error());
  s->n_single++;
}

void finish(qsv_server s, Group* g) {
  const double t = now_s();
  for (const Buf& b : g->bufs) {
    if (b.host)
      s->hpool.put(b.p, b.bytes);
    else
      s->dpool.put(b.p, b.bytes);
  }
  if (g->state) {
    s->idle_state_bytes += state_device_bytes(g->state);
    s->states[g->state_key].push_back(g->state);
  }
  s->free_events.push_back(g->ev);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Req* r : g->reqs) {
      r->t_done = t;
      r->done = true;
      s->reserved -= r->need;
      s->completed++;
    }
  }
  s->cv_done.notify_all();
  delete g;
}

// Free every idle device block and cached state (work in flight keeps
// its own).  hipFree waits for the device, so this runs only when
// admission would otherwise exceed the budget.
void trim_idle(qsv_server s) {
  s->dpool.clear();
  for (auto& kv : s->states)
    for (qsv_state st : kv.second) (void)qsv_free(st);
  s->states.clear();
  s->idle_state_bytes = 0;
  s->trims++;
}

void scheduler(qsv_server s) {
  std::string init_err;
  for (;;) {
    bool progress = false;
    // 1. retire finished groups
    for (size_t i = 0; i < s->running.size();) {
      Group* g = s->running[i];
      const hipError_t q = hipEventQuery(g->ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) fail_group(g, hipGetErrorString(q));
      s->running.erase(s->running.begin() + long(i));
      finish(s, g);
      progress = true;
    }
    // 2. admit first-come first-served while the budget allows and the
    // requests form no more groups than there are idle streams (one group
    // per stream: requests overlap on the device without the whole backlog
    // sharing it, which would delay every request)
    std::vector<Req*> ready;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      const size_t slots =
          s->o.serial ? (s->running.empty() ? 1 : 0)
                      : (s->running.size() < size_t(s->o.n_streams)
                             ? size_t(s->o.n_streams) - s->running.size()
                             : 0);
      size_t groups = 0;
      int in_batch[3] = {0, 0, 0};  // requests in the open batch group
      while (!s->pending.empty() &&
             s->reserved + s->pending.front()->need <= s->o.budget_bytes) {
        Req* r = s->pending.front();
        // idle blocks and cached states hold device memory too: drop them
        // before an admission that would not fit beside them
        if (s->reserved + r->need + s->dpool.idle() + s->idle_state_bytes >
            s->o.budget_bytes)
          trim_idle(s);
        const bool opens = !r->batched || in_batch[r->prec] == 0 ||
                           in_batch[r->prec] >= s->o.max_batch;
        if (opens && groups + 1 > slots) break;
        // the pinned result buffer is taken at admission, so that a long
        // queue holds no pinned memory; the client's release returns it
        r->host = s->hpool.get(std::max<size_t>(r->host_bytes, 8));
        if (!r->host) {
          s->pending.pop_front();
          r->status = QSV_ERR_OUT_OF_MEMORY;
          r->err = "pinned result buffer allocation failed";
          r->t_admit = r->t_done = now_s();
          r->done = true;
          s->completed++;
          s->cv_done.notify_all();
          continue;
        }
        if (opens) {
          ++groups;
          if (r->batched) in_batch[r->prec] = 0;
        }
        if (r->batched) ++in_batch[r->prec];
        s->pending.pop_front();
        r->t_admit = now_s();
        s->reserved += r->need;
        s->peak_reserved = std::max(s->peak_reserved, s->reserved);
        ready.push_back(r);
        if (s->o.serial) break;
      }
      if (ready.empty() && s->running.empty() && s->pending.empty()) {
        if (s->stop) return;
        s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        continue;
      }
    }
    // 3. launch: batch slots by precision, wide requests alone
    if (!ready.empty()) {
      if (!init_hip(s, &init_err)) {
        Group tmp;
        tmp.reqs = ready;
        fail_group(&tmp, init_err);
        std::lock_guard<std::mutex> lk(s->mu);
        for (Req* r : ready) {
          r->done = true;
          r->t_done = now_s();
          s->reserved -= r->need;
          s->completed++;
        }
        s->cv_done.notify_all();
        continue;
      }
      (void)hipSetDevice(s->device);
      std::vector<Group*> groups;
      for (int prec : {QSV_C64, QSV_C128}) {
        Group* cur = nullptr;
        for (Req* r : ready)
          if (r->batched && r->prec == prec) {
            if (!cur || int(cur->reqs.size()) >= s->o.max_batch) {
              cur = new Group;
              groups.push_back(cur);
            }
            cur->reqs.push_back(r);
          }
      }
      for (Req* r : ready)
        if (!r->batched) {
          Group* g = new Group;
          g->reqs.push_back(r);
          groups.push_back(g);
        }
      std::vector<char> busy(s->o.n_streams, 0);
      for (Group* g : s->running) busy[g->stream_idx] = 1;
      for (Group* g : groups) {
        // an idle stream (round-robin among them), else the next one
        int pick = -1;
        for (int k = 0; k < s->o.n_streams && pick < 0; ++k) {
          const int c = (s->rr + k) % s->o.n_streams;
          if (!busy[c]) pick = c;
        }
        if (pick < 0) pick = s->rr % s->o.n_streams;
        s->rr = pick + 1;
        busy[pick] = 1;
        g->stream_idx = pick;
        const double t = now_s();
        for (Req* r : g->reqs) r->t_start = t;
        if (g->reqs[0]->batched)
          launch_batched(s, g, g->reqs[0]->prec);
        else
          launch_single(s, g);
        g->ev = take_event(s);
        (void)hipEventRecord(g->ev, s->streams[g->stream_idx]);
        s->running.push_back(g);
      }
      s->max_inflight = std::max<uint64_t>(s->max_inflight, s->running.size());
      progress = true;
    }
    if (!progress) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

// Device bytes a request may hold while it runs (host buffers are not
// HBM): its state, its output on the device, the sampling scratch, and an
// allowance for its program and reduction scratch.  Pooled blocks (the
// batch path) are rounded to their size class, which wastes at most 1/8
// of a block, and a group's blocks hold the sums of its requests' parts,
// so 9/8 of each part bounds its share.
size_t device_need(const Req& r) {
  const size_t esz = r.b == 8 ? 4 : 8;
  const size_t state = size_t(r.b) << r.w;
  const size_t out = r.samples ? size_t(r.shots) * 8 + 256 : esz << r.w;
  const size_t smp = r.samples ? sample_scratch_bytes(r.w, 0) +
                                     (esz << r.w) : 0;
  const size_t prog = (size_t(64) << 10) + r.G.size() * 1024;
  const size_t red = (state >> 10) + (size_t(64) << 10);
  const size_t parts = state + out + smp + 2 * prog + red;
  return parts + parts / 8;
}

}  // namespace

extern "C" {

double qsv_clock(void) { return now_s(); }

qsv_status qsv_server_create(const qsv_server_opts* opts, qsv_server* out) {
  if (!out) return set_error(QSV_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  qsv_server_opts o = {};
  if (opts) o = *opts;
  if (!o.budget_bytes) o.budget_bytes = uint64_t(256e9);
  if (!o.max_batch) o.max_batch = 256;
  if (!o.small_width) o.small_width = 20;
  if (!o.n_streams) o.n_streams = 4;
  if (o.max_batch < 1 || o.small_width < 0 || o.small_width > QSV_BATCH_MAX_WIDTH ||
      o.n_streams < 1 || o.n_streams > 16)
    return set_error(QSV_ERR_INVALID_ARG, "bad server options");
  qsv_server s = new qsv_server_s;
  s->o = o;
  s->th = std::thread(scheduler, s);
  *out = s;
  return QSV_OK;
}

qsv_status qsv_server_submit(qsv_server s, const qsv_request* rq,
                             uint64_t* ticket) {
  if (!s || !rq || !ticket) return set_error(QSV_ERR_INVALID_ARG, "null argument");
  if (rq->prec != QSV_C64 && rq->prec != QSV_C128)
    return set_error(QSV_ERR_UNSUPPORTED, "unknown precision");
  if (rq->width < 1 || rq->width > QSV_MAX_QUBITS)
    return set_error(QSV_ERR_INVALID_ARG, "width must be 1..34");
  if (rq->want_samples && rq->shots > (uint64_t(1) << 32))
    return set_error(QSV_ERR_INVALID_ARG, "shots must be <= 2^32");
  Req* r = new Req;
  r->w = rq->width;
  r->prec = rq->prec;
  r->b = rq->prec == QSV_C64 ? 8 : 16;
  r->samples = rq->want_samples != 0;
  r->shots = rq->shots;
  r->seed = rq->seed;
  const qsv_circuit& c = rq->body;
  if (c.n_gates && (!c.k || !c.c || !c.qubits || !c.matrices)) {
    delete r;
    return set_error(QSV_ERR_INVALID_ARG, "null circuit array");
  }
  size_t qo = 0, mo = 0;
  r->G.resize(c.n_gates);
  for (size_t i = 0; i < c.n_gates; ++i) {
    std::string e = make_gate(r->w, c.k[i], c.c[i], c.qubits + qo,
                              c.matrices + mo, &r->G[i]);
    if (!e.empty()) {
      delete r;
      return set_error(QSV_ERR_INVALID_ARG, "gate " + std::to_string(i) + ": " + e);
    }
    qo += size_t(c.k[i] + c.c[i]);
    mo += size_t(2) << (2 * c.k[i]);
  }
  r->k.assign(c.k, c.k + c.n_gates);
  r->c.assign(c.c, c.c + c.n_gates);
  r->q.assign(c.qubits, c.qubits + qo);
  r->m.assign(c.matrices, c.matrices + mo);
  r->batched = r->w >= 6 && r->w <= s->o.small_width && batchable(r->G);
  const size_t esz = r->b == 8 ? 4 : 8;
  r->n_out = r->samples ? r->shots : (uint64_t(1) << r->w);
  r->host_bytes = r->samples ? size_t(r->shots) * 8 : (esz << r->w);
  r->need = device_need(*r);
  std::lock_guard<std::mutex> lk(s->mu);
  if (r->need > s->o.budget_bytes) {
    s->rejected++;
    delete r;
    return set_error(QSV_ERR_BUDGET, "request needs more HBM than the budget");
  }
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  s->all[r->ticket] = r;
  s->pending.push_back(r);
  s->submitted++;
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return QSV_OK;
}

static qsv_status wait_impl(qsv_server s, uint64_t ticket, double timeout_s,
                            qsv_result* out) {
  if (!s || !out) return set_error(QSV_ERR_INVALID_ARG, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return set_error(QSV_ERR_INVALID_ARG, "unknown ticket");
  Req* r = it->second;
  if (timeout_s < 0) {
    s->cv_done.wait(lk, [r] { return r->done; });
  } else if (!s->cv_done.wait_for(
                 lk, std::chrono::duration<double>(timeout_s),
                 [r] { return r->done; })) {
    return set_error(QSV_ERR_TIMEOUT, "request not finished within the timeout");
  }
  out->status = r->status;
  out->width = r->w;
  out->prec = r->prec;
  out->is_samples = r->samples;
  out->batched = r->batched;
  out->pad = 0;
  out->n_out = r->n_out;
  out->data = r->host;
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_start = r->t_start;
  out->t_done = r->t_done;
  if (r->status != QSV_OK) return set_error(qsv_status(r->status), r->err);
  return QSV_OK;
}

qsv_status qsv_server_wait(qsv_server s, uint64_t ticket, qsv_result* out) {
  return wait_impl(s, ticket, -1.0, out);
}

qsv_status qsv_server_wait_timeout(qsv_server s, uint64_t ticket,
                                   double timeout_s, qsv_result* out) {
  if (!(timeout_s >= 0) || !std::isfinite(timeout_s))
    return set_error(QSV_ERR_INVALID_ARG, "timeout must be finite and >= 0");
  return wait_impl(s, ticket, timeout_s, out);
}

qsv_status qsv_server_cancel(qsv_server s, uint64_t ticket) {
  if (!s) return set_error(QSV_ERR_INVALID_ARG, "null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end())
      return set_error(QSV_ERR_INVALID_ARG, "unknown ticket");
    Req* r = it->second;
    auto q = std::find(s->pending.begin(), s->pending.end(), r);
    if (q == s->pending.end())
      return set_error(QSV_ERR_INVALID_ARG,
                       "request already admitted or finished");
    s->pending.erase(q);
    r->status = QSV_ERR_CANCELLED;
    r->err = "request cancelled";
    r->t_admit = r->t_start = r->t_done = now_s();
    r->done = true;
    s->completed++;
    s->cancelled++;
  }
  s->cv_done.notify_all();
  return QSV_OK;
}

qsv_status qsv_server_release(qsv_server s, uint64_t ticket) {
  if (!s) return set_error(QSV_ERR_INVALID_ARG, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return set_error(QSV_ERR_INVALID_ARG, "unknown ticket");
  Req* r = it->second;
  if (!r->done) return set_error(QSV_ERR_INVALID_ARG, "request still running");
  s->hpool.put(r->host, std::max<size_t>(r->host_bytes, 8));
  s->all.erase(it);
  delete r;
  return QSV_OK;
}

qsv_status qsv_server_stats(qsv_server s, uint64_t* out, int32_t n) {
  if (!s || !out || n < 0 || n > 8) return set_error(QSV_ERR_INVALID_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t v[8] = {s->submitted, s->completed, s->n_batches, s->n_single,
                         s->peak_reserved, s->max_inflight, s->rejected,
                         s->trims};
  for (int i = 0; i < n; ++i) out[i] = v[i];
  return QSV_OK;
}

qsv_status qsv_server_destroy(qsv_server s) {
  if (!s) return QSV_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->th.join();
  for (auto& kv : s->states)
    for (qsv_state st : kv.second) (void)qsv_free(st);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  for (auto& kv : s->all) {
    s->hpool.put(kv.second->host, std::max<size_t>(kv.second->host_bytes, 8));
    delete kv.second;
  }
  s->dpool.clear();
  s->hpool.clear();
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return QSV_OK;
}

}  // extern "C"
