// Gate-fusion and tiling planner.
//
// The planner is the single-GPU counterpart of the transpile-time cache
// blocking described in Section III.B: there, qubit reordering and inserted
// swaps gather runs of gates onto the qubits inside one 2^nc chunk so that
// they run without exchanging data.  Here a "chunk" is an LDS tile of 2^L
// amplitudes (the coset of L tile qubits), and the planner reorders gates
// that commute so that long runs of gates touch only the tile qubits; each
// run then costs one HBM read and one HBM write of the state.  Diagonal gates
// need no tile qubits at all: their factor depends only on the amplitude's
// index, which every tile knows, so they join any pass.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <array>
#include <functional>
#include <map>
#include <tuple>
#include <unordered_map>
#include <unordered_set>

namespace qsv {

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }

// Below this width a circuit's tile passes take microseconds, less than the
// ownership search would cost; the batch engine steers every variant (its
// plan serves thousands of runs).
constexpr int kSteerMinQubits = 16;

std::string resolve_options(int n, int bytes_per_amp, const int* v,
                            PlanOptions* o) {
  PlanOptions r;
  r.strategy = v ? v[0] : 0;
  r.tile_log2 = (v && v[1]) ? v[1] : 12;
  r.k_max = (v && v[2]) ? v[2] : 5;
  r.low_qubits = (v && v[3]) ? v[3] : 4;
  // A circuit that fits one tile runs on one work-group, bound by the
  // latency of its op chain: eight amplitudes per thread put twice the
  // waves on it (12 qubits: 158 against 188 us per circuit, complex64).
  r.reg_log2 = (v && v[4]) ? v[4]
                           : (n <= r.tile_log2 && r.tile_log2 <= 12 ? 3 : 4);
  if (r.strategy < 0 || r.strategy > 3) return "unknown strategy";
  if (r.tile_log2 < 8 || r.tile_log2 > 13) return "tile_log2 must be 8..13";
  if (r.k_max < 1 || r.k_max > kMaxK) return "k_max must be 1..5";
  if (r.low_qubits < 0 || r.low_qubits > r.tile_log2 - 1)
    return "low_qubits must be 0..tile_log2-1";
  if (r.reg_log2 < 3 || r.reg_log2 > 5) return "reg_log2 must be 3, 4 or 5";
  if (r.reg_log2 > r.tile_log2 - 2) return "reg_log2 too large for tile";
  if (r.tile_log2 - r.reg_log2 > 9)
    return "tile_log2 - reg_log2 must be <= 9 (512 threads per tile)";
  if (bytes_per_amp == 16 && r.reg_log2 > 4)
    return "reg_log2 must be 4 for complex128 (register budget)";
  r.steer = n >= kSteerMinQubits;
  *o = r;
  return "";
}

std::string make_gate(int n, int k, int c, const int32_t* qubits,
                      const double* matrix, HostGate* g) {
  if (k < 1 || k > kMaxK) return "k must be 1..5";
  if (c < 0 || k + c > n) return "too many targets + controls for n";
  if (!qubits) return "null qubit list";
  if (!matrix) return "null matrix";
  uint64_t seen = 0;
  for (int i = 0; i < k + c; ++i) {
    int q = qubits[i];
    if (q < 0 || q >= n) return "qubit index out of range";
    if (seen >> q & 1) return "duplicate qubit among targets and controls";
    seen |= 1ull << q;
  }
  HostGate h;
  h.k = k;
  h.c = c;
  for (int i = 0; i < k; ++i) {
    h.t[i] = qubits[i];
    h.tmask |= 1ull << qubits[i];
  }
  for (int i = 0; i < c; ++i) {
    h.ctl[i] = qubits[k + i];
    h.cmask |= 1ull << qubits[k + i];
  }
  const int d = 1 << k;
  h.m.assign(matrix, matrix + 2 * d * d);
  for (double x : h.m)
    if (!std::isfinite(x)) return "matrix has a non-finite entry";
  bool diag = true;
  for (int r = 0; r < d && diag; ++r)
    for (int s = 0; s < d; ++s)
      if (r != s && (h.m[2 * (r * d + s)] != 0.0 ||
                     h.m[2 * (r * d + s) + 1] != 0.0)) {
        diag = false;
        break;
      }
  h.diagonal = diag;
  bool mp = diag;
  for (int r = 0; r + 1 < d && mp; ++r)
    mp = h.m[2 * (r * d + r)] == 1.0 && h.m[2 * (r * d + r) + 1] == 0.0;
  h.masked_phase = mp;
  *g = std::move(h);
  return "";
}

uint64_t plain_gate_bytes(const HostGate& g, int n, int b) {
  int free_bits = n - g.c - (g.masked_phase ? g.k : 0);
  return 2ull * (uint64_t(1) << free_bits) * uint64_t(b);
}

// One greedy scan over `pending` in list order.  A gate is taken when it
// commutes with every gate skipped before it in this scan, `ok` accepts its
// index and the bits it requires fit into `set` (at most `capacity` bits).
// Taken gates keep their relative order; skipped gates stay pending in
// their order.  `took` hears of each gate taken, as it is taken.
template <class Need, class Ok, class Took>
static void greedy(const std::vector<HostGate>& G, std::vector<int>* pending,
                   uint64_t* set, int capacity, Need need, Ok ok,
                   std::vector<int>* taken, Took took) {
  std::vector<int> rest;
  rest.reserve(pending->size());
  uint64_t blk_touch = 0, blk_dense = 0;
  for (int gi : *pending) {
    const HostGate& g = G[gi];
    bool take = false;
    bool conflict = (g.dense() & blk_touch) || (g.touch() & blk_dense);
    if (!conflict && ok(gi)) {
      uint64_t want = need(g) & ~*set;
      if (popc(*set | want) <= capacity) {
        *set |= want;
        take = true;
      }
    }
    if (take) {
      taken->push_back(gi);
      took(gi);
    } else {
      rest.push_back(gi);
      blk_touch |= g.touch();
      blk_dense |= g.dense();
    }
  }
  pending->swap(rest);
}

static bool tileable(const HostGate& g) {
  return g.diagonal ? (g.masked_phase || g.k <= 2) : g.k == 1;
}

// Which op absorbs a two-qubit diagonal gate (a CZ, say) decides how many
// one-target gates merge: the gates on qubit a before and after a CZ(a, b)
// fuse into one op muxed by b, but only one of a and b can take the CZ (the
// other's op then reads a or b in the middle of its run).  The emitter
// below gives a pending diagonal gate to the first dense gate processed
// that touches it, so the processing order inside a segment is the lever.
//
// Model, per pass and per qubit q: the dense one-target gates on q in
// order; a diagonal gate on q and one other qubit b is "owned" by the side
// whose next gate absorbs it (forced when only one side has a later gate in
// the pass, or when the two next gates lie in different register segments:
// the earlier segment's takes it), and is then a read of b attached to q's
// next gate.  A diagonal
// gate owned by the other side, or a dense gate with q as a control,
// between two gates on q keeps them apart.  Gates on q join into one op
// when nothing keeps them apart and the reads attached to them are all of
// one qubit b, with no dense gate on b between the reads.  The most joins
// on a qubit under a given ownership is a small dynamic program over its
// gates; the ownership of each shared diagonal gate is improved by local
// search (flip while the two qubits' joins grow) from two starts, the
// lower qubit owning every shared gate and the higher one.  Each segment is
// then put in a commuting order (a topological order of its gates, earliest
// first) where the owner's next gate comes before the other qubit's.  The
// emitter still checks every merge itself: the order changes op counts,
// never results.  The segments themselves are built knowing the ownership
// the pass would have with no segment boundaries, so that an owner's next
// gate does not land in a later segment than the other side's (see
// plan_tiled).
// A pass's gates in processing order, with per-qubit rows (compressed) of
// the positions touching each qubit and of the dense gates on it.
struct PassOrder {
  const std::vector<HostGate>& G;
  std::vector<int> order, target, ev, tp;
  std::array<int, 65> eo, to;
  PassOrder(const std::vector<HostGate>& g, std::vector<int> ord)
      : G(g), order(std::move(ord)) {
    const int N = int(order.size());
    target.resize(N);
    eo.fill(0);
    to.fill(0);
    for (int i = 0; i < N; ++i) {
      const HostGate& h = G[order[i]];
      target[i] = (!h.diagonal && h.k == 1) ? h.t[0] : -1;
      for (uint64_t m = h.touch(); m; m &= m - 1) ++eo[__builtin_ctzll(m) + 1];
      if (target[i] >= 0) ++to[target[i] + 1];
    }
    for (int q = 0; q < 64; ++q) {
      eo[q + 1] += eo[q];
      to[q + 1] += to[q];
    }
    ev.resize(eo[64]);
    tp.resize(to[64]);
    std::array<int, 64> fe, ft;
    std::copy(eo.begin(), eo.begin() + 64, fe.begin());
    std::copy(to.begin(), to.begin() + 64, ft.begin());
    for (int i = 0; i < N; ++i) {
      for (uint64_t m = G[order[i]].touch(); m; m &= m - 1)
        ev[fe[__builtin_ctzll(m)]++] = i;
      if (target[i] >= 0) tp[ft[target[i]]++] = i;
    }
  }
  int size() const { return int(order.size()); }
  // dense gates on target b before position i
  int version(int b, int i) const {
    return int(std::lower_bound(tp.begin() + to[b], tp.begin() + to[b + 1], i) -
               (tp.begin() + to[b]));
  }
  // next position after i with a dense gate on target q (-1: none)
  int next_on(int q, int i) const {
    auto it = std::upper_bound(tp.begin() + to[q], tp.begin() + to[q + 1], i);
    return it == tp.begin() + to[q + 1] ? -1 : *it;
  }
  // the other qubit of the two-qubit gate at position d
  int other(int d, int q) const {
    return __builtin_ctzll(G[order[d]].touch() & ~(uint64_t(1) << q));
  }
};

// The owner qubit of each diagonal gate of `po` (-1: none), by the model
// above; `shared` receives the positions of the gates either side could
// take.  With `seg_of`, a gate whose two next gates lie in different
// segments goes to the earlier segment's side.
static std::vector<int> choose_owners(const PassOrder& po,
                                      const std::vector<int>* seg_of,
                                      std::vector<int>* shared,
                                      int* joined = nullptr) {
  const std::vector<HostGate>& G = po.G;
  const int N = po.size();
  std::vector<int> owner(N, -1);
  shared->clear();
  for (int d = 0; d < N; ++d) {
    const HostGate& g = G[po.order[d]];
    if (!g.diagonal) continue;
    const uint64_t tm = g.touch();
    if (popc(tm) == 1) {
      owner[d] = __builtin_ctzll(tm);
    } else if (popc(tm) == 2) {
      const int a = __builtin_ctzll(tm), b = 63 - __builtin_clzll(tm);
      const int na = po.next_on(a, d), nb = po.next_on(b, d);
      const bool apart = seg_of && na >= 0 && nb >= 0 &&
                         (*seg_of)[na] != (*seg_of)[nb];
      if (na >= 0 && nb >= 0 && !apart) shared->push_back(d);
      else if (na >= 0 && (nb < 0 || (*seg_of)[na] < (*seg_of)[nb])) owner[d] = a;
      else if (nb >= 0) owner[d] = b;
    }
  }
  // the most joins on qubit q under `owner`
  auto joins = [&](int q) -> int {
    int bn = -1, bm = -1, mq = -1, mv = -1;  // best per op state
    bool first = true, apart = false, prev_plain = false;
    int rq = -1, rv = -1;
    bool rbad = false;
    auto read = [&](int b, int v) {
      if (rq < 0) {
        rq = b;
        rv = v;
      } else if (rq != b || rv != v) {
        rbad = true;
      }
    };
    for (int e = po.eo[q]; e < po.eo[q + 1]; ++e) {
      const int i = po.ev[e];
      const HostGate& g = G[po.order[i]];
      if (po.target[i] != q) {
        if (!g.diagonal || owner[i] != q || popc(g.touch()) > 2) {
          apart = true;  // q is read by another op, or the gate stands apart
        } else if (popc(g.touch()) == 2) {
          const int b = po.other(i, q);
          read(b, po.version(b, i));
        }
        continue;
      }
      const bool plain = g.c > 1;
      if (g.c == 1) read(g.ctl[0], po.version(g.ctl[0], i));
      if (rbad || plain) {  // the reads are emitted apart from the gate
        apart = true;
        rq = rv = -1;
        if (g.c == 1) {
          rq = g.ctl[0];
          rv = po.version(rq, i);
        }
      }
      const bool join = !first && !apart && !plain && !prev_plain;
      const int top = std::max(bn, bm);
      if (first) {
        bn = rq < 0 ? 0 : -1;
        bm = rq < 0 ? -1 : 0;
        mq = rq;
        mv = rv;
      } else if (rq < 0) {
        const int nn = std::max(top, join && bn >= 0 ? bn + 1 : -1);
        bm = join && bm >= 0 ? bm + 1 : -1;
        bn = nn;
      } else {
        int nm = top;
        if (join && bn >= 0) nm = std::max(nm, bn + 1);
        if (join && bm >= 0 && mq == rq && mv == rv) nm = std::max(nm, bm + 1);
        bm = nm;
        bn = -1;
        mq = rq;
        mv = rv;
      }
      if (plain) {  // a controlled op stands alone
        bn = std::max(bn, bm);
        bm = -1;
      }
      first = false;
      apart = false;
      prev_plain = plain;
      rq = rv = -1;
      rbad = false;
    }
    return std::max(0, std::max(bn, bm));
  };
  if (shared->empty()) {
    if (joined) {
      *joined = 0;
      for (int q = 0; q < 64; ++q)
        if (po.eo[q + 1] > po.eo[q]) *joined += joins(q);
    }
    return owner;
  }
  std::vector<int> best_owner;
  int best_total = -1;
  for (int start = 0; start < 2; ++start) {
    for (int d : *shared) {
      const uint64_t tm = G[po.order[d]].touch();
      owner[d] = start == 0 ? __builtin_ctzll(tm) : 63 - __builtin_clzll(tm);
    }
    std::array<int, 64> jq;
    jq.fill(0);
    int total = 0;
    for (int q = 0; q < 64; ++q)
      if (po.eo[q + 1] > po.eo[q]) total += (jq[q] = joins(q));
    for (int round = 0; round < 8; ++round) {
      bool better = false;
      for (int d : *shared) {
        const int a = owner[d], b = po.other(d, a);
        owner[d] = b;
        const int ja = joins(a), jb = joins(b);
        if (ja + jb > jq[a] + jq[b]) {
          total += ja + jb - jq[a] - jq[b];
          jq[a] = ja;
          jq[b] = jb;
          better = true;
        } else {
          owner[d] = a;
        }
      }
      if (!better) break;
    }
    if (total > best_total) {
      best_total = total;
      best_owner = owner;
    }
  }
  if (joined) *joined = best_total;
  return best_owner;
}

// The processing order of each segment of a tile pass (see above).
static std::vector<std::vector<int>> merge_order(
    const Pass& p, const std::vector<HostGate>& G) {
  std::vector<int> order, seg_of;
  std::vector<std::vector<int>> out(p.segs.size());
  for (size_t si = 0; si < p.segs.size(); ++si) {
    out[si] = p.segs[si].gates;
    for (int gi : p.segs[si].gates) {
      order.push_back(gi);
      seg_of.push_back(int(si));
    }
  }
  const PassOrder po(G, std::move(order));
  std::vector<int> shared;
  const std::vector<int> owner = choose_owners(po, &seg_of, &shared);
  if (shared.empty()) return out;
  // per segment: dependency edges (gates that do not commute keep their
  // order: per qubit, a dense gate after everything since the previous
  // dense gate, anything else after the previous dense gate) plus "owner's
  // next gate first" edges; Kahn's algorithm taking the earliest ready
  // gate; a cycle keeps the segment's order
  const int N = po.size();
  std::vector<std::vector<int>> first_of(N);
  for (int d : shared) {
    const int ua = po.next_on(owner[d], d),
              ub = po.next_on(po.other(d, owner[d]), d);
    if (ua > ub && seg_of[ua] == seg_of[ub]) first_of[ua].push_back(ub);
  }
  int lo = 0;
  for (size_t si = 0; si < p.segs.size(); ++si) {
    const int m = int(p.segs[si].gates.size()), hi = lo + m;
    bool any = false;
    for (int i = lo; i < hi && !any; ++i) any = !first_of[i].empty();
    if (any) {
      std::vector<std::vector<int>> succ(m);
      std::vector<int> indeg(m, 0);
      auto edge = [&](int i, int j) {
        succ[i].push_back(j);
        ++indeg[j];
      };
      std::array<int, 64> last_dense;
      last_dense.fill(-1);
      std::array<std::vector<int>, 64> since;
      for (int j = 0; j < m; ++j) {
        const HostGate& g = G[po.order[lo + j]];
        for (uint64_t t = g.touch(); t; t &= t - 1) {
          const int q = __builtin_ctzll(t);
          if (last_dense[q] >= 0) edge(last_dense[q], j);
          if (g.dense() >> q & 1) {
            for (int i : since[q]) edge(i, j);
            since[q].clear();
            last_dense[q] = j;
          } else {
            since[q].push_back(j);
          }
        }
      }
      for (int i = lo; i < hi; ++i)
        for (int j : first_of[i]) edge(i - lo, j - lo);
      std::vector<int> res;
      std::vector<int> heap;  // min-heap of ready local indices
      for (int i = 0; i < m; ++i)
        if (indeg[i] == 0) heap.push_back(i);
      std::make_heap(heap.begin(), heap.end(), std::greater<int>());
      while (!heap.empty()) {
        std::pop_heap(heap.begin(), heap.end(), std::greater<int>());
        const int i = heap.back();
        heap.pop_back();
        res.push_back(po.order[lo + i]);
        for (int j : succ[i])
          if (--indeg[j] == 0) {
            heap.push_back(j);
            std::push_heap(heap.begin(), heap.end(), std::greater<int>());
          }
      }
      if (int(res.size()) == m) out[si] = std::move(res);
    }
    lo = hi;
  }
  return out;
}

static void add_plain(const std::vector<HostGate>& G, int gi, int n, int b,
                      Plan* plan) {
  Pass p;
  p.kind = kPassPlain;
  p.gates.push_back(gi);
  p.qubits = G[gi].touch();
  p.alg_bytes = plain_gate_bytes(G[gi], n, b);
  plan->alg_bytes += p.alg_bytes;
  plan->plain_passes++;
  plan->passes.push_back(std::move(p));
}

static void plan_tiled(const std::vector<HostGate>& G, int n, int b,
                       const PlanOptions& o, Plan* plan) {
  const int L = std::min(o.tile_log2, n);
  const int RB = o.reg_log2;
  const int m = std::min(o.low_qubits, L);
  std::vector<int> pending(G.size());
  for (size_t i = 0; i < G.size(); ++i) pending[i] = int(i);

  while (!pending.empty()) {
    if (!tileable(G[pending[0]])) {
      add_plain(G, pending[0], n, b, plan);
      pending.erase(pending.begin());
      continue;
    }
    // The tile's qubit set: the low qubits plus either the first qubits the
    // gates in order ask for (greedy) or a window of L - m consecutive
    // qubits, whichever takes the most dense gates.  A pass costs about as
    // much as several dense ops whatever it holds (one HBM round trip, the
    // re-layouts, the tile's load and store), so fewer, fuller passes win;
    // windows follow the light cone of nearest-neighbour circuits, where the
    // greedy choice takes one or two layers of a window's gates per pass.
    const uint64_t low = (m >= 64) ? ~0ull : ((1ull << m) - 1);
    auto tile_ok = [&](int gi) { return tileable(G[gi]); };
    auto no_took = [](int) {};
    auto dense_count = [&](const std::vector<int>& t) {
      int c = 0;
      for (int gi : t) c += !G[gi].diagonal;
      return c;
    };
    uint64_t Q = low;
    std::vector<int> taken, rest = pending;
    greedy(G, &rest, &Q, L, [](const HostGate& g) { return g.dense(); },
           tile_ok, &taken, no_took);
    int best = dense_count(taken), best_s0 = -1;
    for (int s0 = m; s0 + (L - m) <= n && L > m; ++s0) {
      // the dense gates a fixed window takes (the greedy scan, counting)
      uint64_t W = low;
      for (int q = s0; q < s0 + L - m; ++q) W |= uint64_t(1) << q;
      uint64_t blk_touch = 0, blk_dense = 0;
      int c = 0;
      for (int gi : pending) {
        const HostGate& g = G[gi];
        if (!(g.dense() & blk_touch) && !(g.touch() & blk_dense) &&
            tileable(g) && !(g.dense() & ~W)) {
          c += !g.diagonal;
        } else {
          blk_touch |= g.touch();
          blk_dense |= g.dense();
        }
      }
      if (c > best) {
        best = c;
        best_s0 = s0;
      }
    }
    if (best_s0 >= 0) {
      Q = low;
      for (int q = best_s0; q < best_s0 + L - m; ++q) Q |= uint64_t(1) << q;
      taken.clear();
      rest = pending;
      greedy(G, &rest, &Q, L, [](const HostGate& g) { return g.dense(); },
             tile_ok, &taken, no_took);
    }
    pending.swap(rest);
    // Fill the tile's qubit set up to exactly L qubits (lowest free first).
    for (int q = 0; q < n && popc(Q) < L; ++q) Q |= 1ull << q;

    Pass p;
    p.kind = kPassTile;
    p.L = L;
    p.qubits = Q;
    int local_of[64];
    for (int q = 0, j = 0; q < n; ++q)
      if (Q >> q & 1) {
        p.q[j] = q;
        local_of[q] = j++;
      }
    // Register segments: the same greedy scan over tile-local target bits
    // with capacity RB; diagonal gates need no register bit.  Unused
    // register bits are filled with the highest free tile-local bits, so
    // that the low bits index lanes (contiguous HBM runs across lanes) and a
    // segment that needs few bits tends to match the I/O layout (register
    // bits L-RB..L-1), which saves the re-layout on entry or exit.
    // Two-qubit diagonal gates whose owner (the side whose next gate takes
    // it, chosen as if there were no segments) should keep that gate no
    // later than the other side's: with `keep_owners`, a gate waits for the
    // owners' gates it must follow (`after`).
    std::unordered_map<int, std::vector<int>> after;  // gate -> owners' gates
    p.steer = o.steer;
    if (o.steer) {
      const PassOrder po(G, taken);
      std::vector<int> shared;
      const std::vector<int> owner = choose_owners(po, nullptr, &shared);
      for (int d : shared) {
        const int ua = po.next_on(owner[d], d),
                  ub = po.next_on(po.other(d, owner[d]), d);
        if (ua < 0 || ub < 0) continue;
        after[po.order[ub]].push_back(po.order[ua]);
      }
    }
    auto build_segs = [&](bool seed_io, bool keep_owners) {
      std::vector<Pass::Seg> segs;
      std::vector<int> seg_pending = taken;
      bool waits = keep_owners && !after.empty();
      std::unordered_set<int> placed;
      bool first = true;
      while (!seg_pending.empty()) {
        // seed_io: the first segment takes the I/O layout's register bits
        // and collects the gates that fit them
        uint64_t S = (first && seed_io) ? ((1ull << RB) - 1) << (L - RB) : 0;
        first = false;
        std::vector<int> seg_gates;
        auto need = [&](const HostGate& g) -> uint64_t {
          return g.diagonal ? 0 : (1ull << local_of[g.t[0]]);
        };
        if (!waits) {
          greedy(G, &seg_pending, &S, RB, need, [](int) { return true; },
                 &seg_gates, [](int) {});
        } else {
          greedy(G, &seg_pending, &S, RB, need,
                 [&](int gi) {
                   const auto it = after.find(gi);
                   if (it == after.end()) return true;
                   for (int ga : it->second)
                     if (!placed.count(ga)) return false;
                   return true;
                 },
                 &seg_gates, [&](int gi) { placed.insert(gi); });
          bool any_dense = false;
          for (int gi : seg_gates) any_dense |= !G[gi].diagonal;
          if (!any_dense && !seg_pending.empty()) {
            // waiting gates block every remaining one: drop the waits
            waits = false;
            seg_pending.insert(seg_pending.begin(), seg_gates.begin(),
                               seg_gates.end());
            std::vector<int> keep_order;
            for (int gi : taken)
              if (std::find(seg_pending.begin(), seg_pending.end(), gi) !=
                  seg_pending.end())
                keep_order.push_back(gi);
            seg_pending.swap(keep_order);
            first = segs.empty();
            continue;
          }
        }
        for (int lb = L - 1; lb >= 0 && popc(S) < RB; --lb) S |= 1ull << lb;
        Pass::Seg sg;
        for (int lb = 0, j = 0; lb < L; ++lb)
          if (S >> lb & 1) sg.reg_bits[j++] = lb;
        sg.gates = std::move(seg_gates);
        segs.push_back(std::move(sg));
      }
      return segs;
    };
    // re-layouts a segment list costs: entry, between segments, exit
    auto relayouts = [&](const std::vector<Pass::Seg>& segs) {
      auto same = [&](const Pass::Seg& x, const int* rb) {
        for (int i = 0; i < RB; ++i)
          if (x.reg_bits[i] != rb[i]) return false;
        return true;
      };
      int io[6];
      for (int i = 0; i < RB; ++i) io[i] = L - RB + i;
      int r = !same(segs.front(), io) + !same(segs.back(), io);
      for (size_t i = 1; i < segs.size(); ++i)
        r += !same(segs[i], segs[i - 1].reg_bits);
      return r;
    };
    // ops the emitted program would hold, as the ownership model counts
    // them: one-target gates less the joins it finds
    auto op_count = [&](const std::vector<Pass::Seg>& segs) -> double {
      std::vector<int> order, seg_of;
      for (size_t si = 0; si < segs.size(); ++si)
        for (int gi : segs[si].gates) {
          order.push_back(gi);
          seg_of.push_back(int(si));
        }
      const PassOrder po(G, std::move(order));
      int ones = 0, joined = 0;
      for (int t : po.target) ones += t >= 0;
      std::vector<int> shared;
      choose_owners(po, &seg_of, &shared, &joined);
      return double(ones - joined);
    };
    // Of the plain and the I/O-seeded scans, with and without the owners'
    // waits: the fewest ops plus, per re-layout, half an op for complex64
    // and a whole one for complex128 (a re-layout moves every amplitude's
    // bytes through LDS twice; the weights are the best of 0.5, 1 and 2
    // measured on the 30-, 33- and 34-qubit circuits).
    const double relayout_ops = 0.5 * double(b) / 8.0;
    p.segs = build_segs(false, false);
    if (!p.segs.empty() && !o.steer) {
      // the plain scan, or the seeded one where it needs fewer re-layouts
      std::vector<Pass::Seg> seeded = build_segs(true, false);
      if (relayouts(seeded) < relayouts(p.segs)) p.segs.swap(seeded);
    } else if (!p.segs.empty()) {
      double best = op_count(p.segs) + relayout_ops * relayouts(p.segs);
      for (int v = 1; v < 4; ++v) {
        if ((v & 2) && after.empty()) continue;
        std::vector<Pass::Seg> alt = build_segs(v & 1, (v & 2) != 0);
        const double c = op_count(alt) + relayout_ops * relayouts(alt);
        if (c < best) {
          best = c;
          p.segs.swap(alt);
        }
      }
    }
    for (const auto& sg : p.segs)
      p.gates.insert(p.gates.end(), sg.gates.begin(), sg.gates.end());
    p.alg_bytes = 2ull * (uint64_t(1) << n) * uint64_t(b);
    plan->alg_bytes += p.alg_bytes;
    plan->tile_passes++;
    plan->segments += int(p.segs.size());
    plan->passes.push_back(std::move(p));
  }
}

static void plan_fused(const std::vector<HostGate>& G, int n, int b,
                       const PlanOptions& o, Plan* plan) {
  const int K = std::min(o.k_max, n);
  std::vector<int> pending(G.size());
  for (size_t i = 0; i < G.size(); ++i) pending[i] = int(i);
  auto fits = [K](const HostGate& g) { return popc(g.touch()) <= K; };
  while (!pending.empty()) {
    if (!fits(G[pending[0]])) {
      add_plain(G, pending[0], n, b, plan);
      pending.erase(pending.begin());
      continue;
    }
    uint64_t S = 0;
    std::vector<int> taken;
    greedy(G, &pending, &S, K,
           [](const HostGate& g) { return g.touch(); },
           [&](int gi) { return fits(G[gi]); }, &taken, [](int) {});
    Pass p;
    p.kind = kPassFused;
    p.qubits = S;
    p.fk = popc(S);
    for (int q = 0, j = 0; q < n; ++q)
      if (S >> q & 1) p.fq[j++] = q;
    p.gates = std::move(taken);
    p.alg_bytes = 2ull * (uint64_t(1) << n) * uint64_t(b);
    plan->alg_bytes += p.alg_bytes;
    plan->fused_passes++;
    plan->passes.push_back(std::move(p));
  }
}

// Value of diagonal gate d on a basis state given by `bits` (only the
// qubits of d matter): its diagonal entry where all controls are 1, else 1.
static void diag_value(const HostGate& d, uint64_t bits, double* re,
                       double* im) {
  if ((bits & d.cmask) != d.cmask) {
    *re = 1;
    *im = 0;
    return;
  }
  int r = 0;
  for (int j = 0; j < d.k; ++j) r |= int(bits >> d.t[j] & 1) << j;
  const int dim = 1 << d.k;
  *re = d.m[2 * (r * dim + r)];
  *im = d.m[2 * (r * dim + r) + 1];
}

// Phase terms of a diagonal unitary gate.  Its phase function over the
// target bits, phi(r) = arg of diagonal entry r, has a unique multilinear
// expansion phi(r) = sum over target subsets S of c_S * [all bits of S set
// in r]; the coefficients are the Moebius inversion c_S = sum over T within
// S of (-1)^{|S|-|T|} phi(T).  Each nonzero c_S becomes a term whose mask is
// S's qubits plus the controls.  False when an entry is not of unit modulus
// (then the gate is not a phase and keeps its own op).
static bool phase_terms(const HostGate& g,
                        std::vector<std::pair<uint64_t, double>>* out) {
  const int d = 1 << g.k;
  double phi[1 << kMaxK];
  for (int r = 0; r < d; ++r) {
    const double re = g.m[2 * (r * d + r)], im = g.m[2 * (r * d + r) + 1];
    if (std::fabs(std::hypot(re, im) - 1.0) > 1e-12) return false;
    phi[r] = std::atan2(im, re);
  }
  for (int j = 0; j < g.k; ++j)
    for (int S = 0; S < d; ++S)
      if (S >> j & 1) phi[S] -= phi[S ^ (1 << j)];
  for (int S = 0; S < d; ++S) {
    if (std::fabs(phi[S]) < 1e-15) continue;
    uint64_t mask = g.cmask;
    for (int j = 0; j < g.k; ++j)
      if (S >> j & 1) mask |= uint64_t(1) << g.t[j];
    out->push_back({mask, phi[S]});
  }
  return true;
}

// An angle as a fixed-point fraction of a turn: round(angle / 2pi * 2^64)
// modulo 2^64.
static uint64_t angle_turns(double ang) {
  double f = ang / (2.0 * M_PI);
  f -= std::floor(f);  // [0, 1]
  const double x = std::ldexp(f, 32);
  const double hi = std::floor(x);
  const uint64_t lo = uint64_t(std::llround(std::ldexp(x - hi, 32)));
  return (uint64_t(hi) << 32) + lo;  // wraps modulo 2^64
}

// The kernels' dispatch code of a finished op (see kCode* in program.h).
// A dense op without a mux, or with one outside the tile, takes its matrix
// by one bit of the tile's base index: the outer mux qubit, or bit 63,
// which no index has (its second matrix is then a copy of the first).
std::string set_op_code(TileOp* op) {
  int32_t cls = 0;
  op->arg = 0;
  switch (op->kind) {
    case kOpDense1:
      if (op->mux == kMuxNone || op->mux < 0) {
        cls = op->lctrl ? kCodeCtrl : kCodeUniform;
        if (op->mux == kMuxNone) {
          op->arg = 63;
          std::memcpy(op->m2, op->m, sizeof op->m);
          std::memcpy(op->mf2, op->mf, sizeof op->mf);
        } else {
          op->arg = -1 - op->mux;
        }
      } else if (op->lctrl == 0 && op->mux_reg >= 0) {
        cls = kCodeRegMux;
        op->arg = op->mux_reg;
      } else {
        cls = op->lctrl == 0 ? kCodeThreadMux : kCodeCtrlMux;
        op->arg = op->mux;
      }
      if (op->reg < 0 || op->reg >= kMaxRegBits)
        return "internal planner error: bad register index";
      op->code = (cls << 3) | op->reg;
      return "";
    case kOpPhase:
      op->code = kCodePhase << 3;
      return "";
    case kOpDiag:
      op->code = kCodeDiag << 3;
      op->arg = op->dk;
      return "";
    case kOpPhaseBlock:
      op->code = kCodePhaseBlock << 3;
      return "";
    default:
      return "internal planner error: unknown op kind";
  }
}

// Exactly the 2x2 identity (interleaved complex, row-major).
static bool is_identity2(const double* m) {
  static const double id[8] = {1, 0, 0, 0, 0, 0, 1, 0};
  for (int i = 0; i < 8; ++i)
    if (m[i] != id[i]) return false;
  return true;
}

std::string emit_tile_pass(const Pass& p, const std::vector<HostGate>& G,
                           int RB, std::vector<TilePass>* tpasses,
                           std::vector<TileSeg>* tsegs,
                           std::vector<TileOp>* tops,
                           TileEmitStats* stats) {
  TilePass tp = {};
  tp.L = p.L;
  tp.nseg = int32_t(p.segs.size());
  tp.seg_begin = int32_t(tsegs->size());
  // Thread bits of the I/O layout are tile bits 0..L-RB-1; the lowest six
  // of them index the lanes of a wave, the rest are uniform over a wave.
  // The lane part of a byte offset is below 16 * 2^(q[lane bits - 1] + 1)
  // even for complex128; where that fits 32 bits each access is a
  // wave-uniform address plus a 32-bit lane offset.
  tp.flags = 0;
  {
    const int lane_bits = std::min(p.L - RB, 6);
    if (lane_bits <= 0 || p.q[lane_bits - 1] + 1 + 4 <= 32)
      tp.flags |= kPassLane32;
  }
  // the tile is 2^(L - m) contiguous runs, m = its lowest contiguous qubits
  int m = 0;
  while (m < p.L && p.q[m] == m) ++m;
  if (p.L - m >= 3) tp.flags |= kPassSpread;
  int local_of[64];
  for (int j = 0; j < p.L; ++j) {
    tp.q[j] = p.q[j];
    local_of[p.q[j]] = j;
  }
  auto place_ctrl = [&](TileOp* op, uint64_t mask) {
    for (int q = 0; q < 64; ++q)
      if (mask >> q & 1) {
        if (p.qubits >> q & 1)
          op->lctrl |= 1u << local_of[q];
        else
          op->gctrl |= uint64_t(1) << q;
      }
  };
  auto emit_diag = [&](const HostGate& g) {
    TileOp op = {};
    op.mux = kMuxNone;
    place_ctrl(&op, g.cmask);
    const int d = 1 << g.k;
    if (g.masked_phase) {
      op.kind = kOpPhase;
      place_ctrl(&op, g.tmask);
      op.m[0] = g.m[2 * ((d - 1) * d + (d - 1))];
      op.m[1] = g.m[2 * ((d - 1) * d + (d - 1)) + 1];
    } else {
      op.kind = kOpDiag;
      op.dk = g.k;
      int* db[2] = {&op.dbit0, &op.dbit1};
      for (int j = 0; j < g.k; ++j) {
        const int q = g.t[j];
        *db[j] = (p.qubits >> q & 1) ? local_of[q] : -1 - q;
      }
      for (int r = 0; r < d; ++r) {
        op.m[2 * r] = g.m[2 * (r * d + r)];
        op.m[2 * r + 1] = g.m[2 * (r * d + r) + 1];
      }
    }
    for (int e = 0; e < 8; ++e) op.mf[e] = float(op.m[e]);
    tops->push_back(op);
  };

  // Dense one-target gates are emitted as "mux" gates: matrix M(v) for each
  // value v of at most one other qubit (a single control c becomes
  // M(0) = I, M(1) = U).  Diagonal gates wait in `pend` until a dense gate
  // acts on one of their qubits (they commute with everything else) and
  // are folded into it when they involve at most that mux qubit:
  // M(v) <- M(v) diag(e_0(v), e_1(v)).  A new gate on t then merges into
  // the previous op on t when no op emitted since touches t and the mux
  // qubit's value cannot have changed in between (no dense op on it since):
  // M(v) <- M_new(v) M_prev(v).  The state after the pass is unchanged up
  // to rounding.
  const int n_q = 64;
  std::vector<int> last_touch(n_q, -1), last_dense(n_q, -1);
  const int op_base = int(tops->size());
  auto touch_op = [&](uint64_t mask, int idx) {
    for (int q = 0; q < n_q; ++q)
      if (mask >> q & 1) last_touch[q] = std::max(last_touch[q], idx);
  };
  auto mux_code = [&](int q) -> int32_t {
    return q < 0 ? kMuxNone
                 : ((p.qubits >> q & 1) ? local_of[q] : -1 - q);
  };
  // mux qubit and dense target of each op emitted in this pass (-1: none)
  std::vector<int> op_mux_q, op_target_q;
  // pending (deferred) one-target products per qubit, and the segment
  // (pass-local index) where each would be emitted
  std::vector<std::array<double, 8>> pp(n_q);
  std::vector<char> has_pp(n_q, 0);
  std::vector<int> pp_seg(n_q, -1);
  int cur_si = 0;          // the segment being emitted
  TileSeg* cur_ts = nullptr;
  auto emit_diag_tracked = [&](const HostGate& g) {
    emit_diag(g);
    op_mux_q.push_back(-1);
    op_target_q.push_back(-1);
    touch_op(g.touch(), int(tops->size()) - 1);
  };
  // Runs of diagonal gates: those whose phase terms all fit the segment's
  // layout (at most one register bit per term, or register bits only)
  // become one kOpPhaseBlock when there are at least kMinBlock of them; the
  // others keep an op each.  Diagonal gates commute, so the order of the
  // block and the single ops does not matter.
  constexpr size_t kMinBlock = 4;
  struct Blob {
    int op;
    std::vector<char> bytes;
  };
  std::vector<Blob> blobs;
  auto emit_diag_run = [&](const std::vector<int>& run, const Pass::Seg& sg) {
    std::vector<int> blocked, single;
    // per term: accumulator, thread mask, outer mask -> summed turns
    std::map<std::tuple<int, uint32_t, uint64_t>, uint64_t> acc;
    uint64_t table[1 << kMaxRegBits] = {0};
    std::vector<std::pair<uint64_t, double>> terms;
    struct Placed {
      int k;
      uint32_t tm;
      uint64_t gm;
      uint32_t regs;
      uint64_t turns;
    };
    std::vector<std::vector<Placed>> placed(run.size());
    for (size_t i = 0; i < run.size(); ++i) {
      const HostGate& g = G[run[i]];
      terms.clear();
      bool ok = phase_terms(g, &terms);
      for (size_t e = 0; ok && e < terms.size(); ++e) {
        Placed pl = {0, 0u, 0, 0u, angle_turns(terms[e].second)};
        int nreg = 0, rlast = -1;
        for (int q = 0; q < 64; ++q) {
          if (!(terms[e].first >> q & 1)) continue;
          if (!(p.qubits >> q & 1)) {
            pl.gm |= uint64_t(1) << q;
            continue;
          }
          const int lb = local_of[q];
          int r = -1;
          for (int b = 0; b < RB; ++b)
            if (sg.reg_bits[b] == lb) r = b;
          if (r >= 0) {
            pl.regs |= 1u << r;
            ++nreg;
            rlast = r;
          } else {
            pl.tm |= 1u << lb;
          }
        }
        if (nreg <= 1) pl.k = nreg ? 1 + rlast : 0;
        else if (pl.tm == 0 && pl.gm == 0) pl.k = -1;  // register table
        else ok = false;
        placed[i].push_back(pl);
      }
      (ok ? blocked : single).push_back(int(i));
    }
    if (blocked.size() < kMinBlock) {
      for (int d : run) emit_diag_tracked(G[d]);
      return;
    }
    for (int i : single) emit_diag_tracked(G[run[i]]);
    if (stats) {
      stats->blocks++;
      stats->block_gates += blocked.size();
    }
    uint64_t touched = 0;
    for (int i : blocked) {
      touched |= G[run[i]].touch();
      for (const Placed& pl : placed[i]) {
        if (pl.k >= 0) {
          acc[std::make_tuple(pl.k, pl.tm, pl.gm)] += pl.turns;
        } else {
          for (uint32_t j = 0; j < (1u << RB); ++j)
            if ((j & pl.regs) == pl.regs) table[j] += pl.turns;
        }
      }
    }
    PhaseBlock hdr = {};
    std::vector<PhaseTerm> out;
    for (const auto& kv : acc) {  // ordered by accumulator, then tmask
      if (kv.second == 0) continue;
      const int k = std::get<0>(kv.first);
      PhaseTerm t = {};
      t.tmask = std::get<1>(kv.first);
      t.gmask = std::get<2>(kv.first);
      t.turns = kv.second;
      t.turns32 = uint32_t((kv.second + (uint64_t(1) << 31)) >> 32);
      (t.tmask ? hdr.n_thr : hdr.n_uni)[k]++;
      out.push_back(t);
    }
    for (uint32_t j = 0; j < (1u << RB); ++j) {
      if (table[j]) hdr.has_table = 1;
      const double a = std::ldexp(double(table[j]), -64) * 2.0 * M_PI;
      hdr.td[2 * j] = std::cos(a);
      hdr.td[2 * j + 1] = std::sin(a);
      hdr.tf[2 * j] = float(hdr.td[2 * j]);
      hdr.tf[2 * j + 1] = float(hdr.td[2 * j + 1]);
    }
    hdr.n_terms = int32_t(out.size());
    Blob bl;
    bl.bytes.resize(sizeof hdr + out.size() * sizeof(PhaseTerm));
    std::memcpy(bl.bytes.data(), &hdr, sizeof hdr);
    if (!out.empty())
      std::memcpy(bl.bytes.data() + sizeof hdr, out.data(),
                  out.size() * sizeof(PhaseTerm));
    TileOp op = {};
    op.kind = kOpPhaseBlock;
    op.mux = kMuxNone;
    tops->push_back(op);
    bl.op = int(tops->size()) - 1;
    blobs.push_back(std::move(bl));
    op_mux_q.push_back(-1);
    op_target_q.push_back(-1);
    touch_op(touched, int(tops->size()) - 1);
  };
  // Emit (or merge) a dense one-target op with mux matrices M on target t:
  // merged into the previous op on t when no op emitted since touches t
  // and the mux qubit cannot have changed in between, else appended.
  // With `defer`, an op without a mux that cannot merge is kept pending on
  // t instead (see below).  Returns an error text or "".
  auto put_dense = [&](int t, int mux_q, double (*M)[8], int seg_idx,
                       bool defer) -> std::string {
    const int lb = local_of[t];
    int reg = -1;
    for (int i = 0; i < RB; ++i)
      if (p.segs[seg_idx].reg_bits[i] == lb) reg = i;
    if (reg < 0) return "internal planner error: target not in a register bit";
    const int prev = last_touch[t];
    if (prev >= op_base) {
      TileOp& po = (*tops)[prev];
      const int pq = op_mux_q[prev - op_base];
      if (po.kind == kOpDense1 && op_target_q[prev - op_base] == t &&
          po.lctrl == 0 && po.gctrl == 0 &&
          (pq < 0 || mux_q < 0 || pq == mux_q) &&
          (mux_q < 0 || last_dense[mux_q] < prev)) {
        const int mq = pq >= 0 ? pq : mux_q;
        double out[2][8];
        for (int v = 0; v < 2; ++v) {
          const double* A = M[v];
          const double* B = (pq >= 0 && v) ? po.m2 : po.m;
          for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
              double cr = 0, ci = 0;
              for (int k = 0; k < 2; ++k) {
                const double ar = A[2 * (2 * r + k)], ai = A[2 * (2 * r + k) + 1];
                const double br = B[2 * (2 * k + c)], bi = B[2 * (2 * k + c) + 1];
                cr += ar * br - ai * bi;
                ci += ar * bi + ai * br;
              }
              out[v][2 * (2 * r + c)] = cr;
              out[v][2 * (2 * r + c) + 1] = ci;
            }
        }
        std::memcpy(po.m, out[0], sizeof out[0]);
        std::memcpy(po.m2, out[1], sizeof out[1]);
        po.mux = mux_code(mq);
        op_mux_q[prev - op_base] = mq;
        for (int e = 0; e < 8; ++e) {
          po.mf[e] = float(po.m[e]);
          po.mf2[e] = float(po.m2[e]);
        }
        if (mq >= 0) touch_op(uint64_t(1) << mq, prev);
        last_dense[t] = std::max(last_dense[t], prev);
        return "";
      }
    }
    if (defer && mux_q < 0) {
      std::memcpy(pp[t].data(), M[0], sizeof M[0]);
      has_pp[t] = 1;
      pp_seg[t] = seg_idx;
      return "";
    }
    TileOp op = {};
    op.kind = kOpDense1;
    op.reg = reg;
    std::memcpy(op.m, M[0], sizeof op.m);
    std::memcpy(op.m2, M[1], sizeof op.m2);
    op.mux = mux_code(mux_q);
    for (int e = 0; e < 8; ++e) {
      op.mf[e] = float(op.m[e]);
      op.mf2[e] = float(op.m2[e]);
    }
    if (seg_idx == cur_si) {
      tops->push_back(op);
      op_mux_q.push_back(mux_q);
      op_target_q.push_back(t);
      const int idx = int(tops->size()) - 1;
      touch_op((uint64_t(1) << t) | (mux_q >= 0 ? uint64_t(1) << mux_q : 0), idx);
      last_dense[t] = idx;
      return "";
    }
    // An earlier, closed segment (a pending product whose qubit is not a
    // register bit of the current segment; mux_q < 0): the op goes at that
    // segment's end.  Nothing emitted since touches t, so the op commutes
    // with everything after it; every later index moves up by one.
    const int pos = (*tsegs)[size_t(tp.seg_begin) + size_t(seg_idx)].op_end;
    tops->insert(tops->begin() + pos, op);
    op_mux_q.insert(op_mux_q.begin() + (pos - op_base), -1);
    op_target_q.insert(op_target_q.begin() + (pos - op_base), t);
    for (int& v : last_touch)
      if (v >= pos) ++v;
    for (int& v : last_dense)
      if (v >= pos) ++v;
    for (Blob& bl : blobs)
      if (bl.op >= pos) ++bl.op;
    for (int k = seg_idx; k < cur_si; ++k) {
      TileSeg& T = (*tsegs)[size_t(tp.seg_begin) + size_t(k)];
      if (k > seg_idx) ++T.op_begin;
      ++T.op_end;
    }
    ++cur_ts->op_begin;
    last_touch[t] = pos;
    last_dense[t] = pos;
    return "";
  };
  // Deferred one-target gates.  A dense gate without controls whose op would
  // have no mux, and that cannot merge into the previous op on its target,
  // is kept as a pending 2x2 product on the target instead of being
  // emitted: the next dense gate on that target absorbs it (M <- M P), so a
  // gate between two controlled-phase folds joins one op.  A pending product
  // is emitted first wherever its qubit must be settled: before an op that
  // uses the qubit as its mux or a control, before a diagonal run touching
  // it, and by the pass's end.  It may wait across segments; when settled it
  // goes into the latest segment so far that holds its qubit in a register
  // bit (at that segment's end when the segment is already closed).
  auto flush = [&](int q) -> std::string {
    if (!has_pp[q]) return "";
    has_pp[q] = 0;
    double M[2][8];
    std::memcpy(M[0], pp[q].data(), sizeof M[0]);
    std::memcpy(M[1], pp[q].data(), sizeof M[1]);
    return put_dense(q, -1, M, pp_seg[q], false);
  };
  auto flush_mask = [&](uint64_t mask) -> std::string {
    for (int q = 0; q < n_q; ++q)
      if (mask >> q & 1) {
        std::string e = flush(q);
        if (!e.empty()) return e;
      }
    return "";
  };
  auto touched_by = [&](const std::vector<int>& ds) {
    uint64_t m = 0;
    for (int d : ds) m |= G[d].touch();
    return m;
  };
  std::vector<int> pend;
  std::vector<std::vector<int>> seg_order;
  if (p.steer) {
    seg_order = merge_order(p, G);
  } else {
    for (const auto& sg : p.segs) seg_order.push_back(sg.gates);
  }
  for (size_t si = 0; si < p.segs.size(); ++si) {
    const auto& sg = p.segs[si];
    TileSeg ts = {};
    for (int i = 0; i < RB; ++i) ts.reg_bits[i] = sg.reg_bits[i];
    ts.op_begin = int32_t(tops->size());
    cur_si = int(si);
    cur_ts = &ts;
    // a pending product is emitted as late as possible: in the latest
    // segment so far that holds its qubit in a register bit
    for (int i = 0; i < RB; ++i) {
      const int q = p.q[sg.reg_bits[i]];
      if (has_pp[q]) pp_seg[q] = int(si);
    }
    for (int gi : seg_order[si]) {
      const HostGate& g = G[gi];
      if (g.diagonal) {
        pend.push_back(gi);
        continue;
      }
      const int t = g.t[0];
      std::vector<int> hit, keep;
      for (int d : pend)
        (G[d].touch() >> t & 1 ? hit : keep).push_back(d);
      pend.swap(keep);
      // the gate as mux matrices
      int mux_q = -1;
      const bool plain = g.c > 1;  // more than one control: a controlled op
      double M[2][8];
      if (g.c == 1) {
        mux_q = g.ctl[0];
        const double id[8] = {1, 0, 0, 0, 0, 0, 1, 0};
        std::memcpy(M[0], id, sizeof id);
        std::memcpy(M[1], g.m.data(), sizeof M[1]);
      } else {
        std::memcpy(M[0], g.m.data(), sizeof M[0]);
        std::memcpy(M[1], g.m.data(), sizeof M[1]);
      }
      bool fold = !plain;
      for (int d : hit) {
        const uint64_t others = G[d].touch() & ~(uint64_t(1) << t);
        if (__builtin_popcountll(others) > 1) fold = false;
        if (others) {
          const int q = __builtin_ctzll(others);
          if (mux_q < 0 && fold) mux_q = q;
          else if (mux_q != q) fold = false;
        }
      }
      std::string err;
      if (!fold) {
        // the pending products of the run's qubits precede it
        if (!(err = flush_mask(touched_by(hit))).empty()) return err;
        emit_diag_run(hit, sg);
        if (!plain && g.c == 0) mux_q = -1;
        if (!plain && g.c == 1) mux_q = g.ctl[0];
      } else {
        for (int v = 0; v < 2; ++v)
          for (int sc = 0; sc < 2; ++sc) {  // column sc scaled by e_sc(v)
            double er = 1, ei = 0;
            const uint64_t bits = (uint64_t(sc) << t) |
                                  (mux_q >= 0 ? uint64_t(v) << mux_q : 0);
            for (int d : hit) {
              double vr, vi;
              diag_value(G[d], bits, &vr, &vi);
              const double nr = er * vr - ei * vi, ni = er * vi + ei * vr;
              er = nr;
              ei = ni;
            }
            for (int r = 0; r < 2; ++r) {
              double* x = &M[v][2 * (2 * r + sc)];
              const double xr = x[0], xi = x[1];
              x[0] = xr * er - xi * ei;
              x[1] = xr * ei + xi * er;
            }
          }
      }
      if (plain) {
        // a controlled op: its target and controls are settled first
        if (!(err = flush_mask(g.touch())).empty()) return err;
        const int lb = local_of[t];
        int reg = -1;
        for (int i = 0; i < RB; ++i)
          if (sg.reg_bits[i] == lb) reg = i;
        if (reg < 0) return "internal planner error: target not in a register bit";
        TileOp op = {};
        op.kind = kOpDense1;
        op.reg = reg;
        op.mux = kMuxNone;
        place_ctrl(&op, g.cmask);
        for (int e = 0; e < 8; ++e) {
          op.m[e] = g.m[e];
          op.mf[e] = float(op.m[e]);
        }
        tops->push_back(op);
        op_mux_q.push_back(-1);
        op_target_q.push_back(t);
        const int idx = int(tops->size()) - 1;
        touch_op(g.touch(), idx);
        last_dense[t] = idx;
        continue;
      }
      // absorb the target's pending product (applied before this gate)
      if (has_pp[t]) {
        has_pp[t] = 0;
        for (int v = 0; v < 2; ++v) {
          double out[8];
          const double* A = M[v];
          const double* B = pp[t].data();
          for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
              double cr = 0, ci = 0;
              for (int k = 0; k < 2; ++k) {
                const double ar = A[2 * (2 * r + k)], ai = A[2 * (2 * r + k) + 1];
                const double br = B[2 * (2 * k + c)], bi = B[2 * (2 * k + c) + 1];
                cr += ar * br - ai * bi;
                ci += ar * bi + ai * br;
              }
              out[2 * (2 * r + c)] = cr;
              out[2 * (2 * r + c) + 1] = ci;
            }
          std::memcpy(M[v], out, sizeof out);
        }
      }
      // the mux qubit is settled before an op that reads it
      if (mux_q >= 0 && !(err = flush(mux_q)).empty()) return err;
      if (!(err = put_dense(t, mux_q, M, int(si), true)).empty()) return err;
    }
    // pending products wait across segments (the next dense gate on the
    // qubit may absorb them); the pass's end settles every one of them
    if (si + 1 == p.segs.size()) {
      if (std::string err = flush_mask(~uint64_t(0)); !err.empty()) return err;
      emit_diag_run(pend, sg);
      pend.clear();
    }
    ts.op_end = int32_t(tops->size());
    tsegs->push_back(ts);
  }
  // Locate each op's tile-local mux bit in its own segment's register bits
  // (merges above may have changed an op's mux after its segment closed),
  // then give every op its dispatch code.
  for (size_t si = 0; si < p.segs.size(); ++si) {
    const TileSeg& ts = (*tsegs)[tp.seg_begin + si];
    for (int oi = ts.op_begin; oi < ts.op_end; ++oi) {
      TileOp& op = (*tops)[oi];
      op.mux_reg = -1;
      if (op.kind == kOpDense1 && op.mux != kMuxNone && op.mux >= 0) {
        for (int i = 0; i < RB; ++i)
          if (ts.reg_bits[i] == op.mux) op.mux_reg = i;
        if (op.mux_reg == op.reg)
          return "internal planner error: mux bit equals the target bit";
      }
      std::string err = set_op_code(&op);
      if (!err.empty()) return err;
    }
  }
  if (stats) {
    stats->ops += tops->size() - size_t(op_base);
    for (size_t i = size_t(op_base); i < tops->size(); ++i) {
      const TileOp& o = (*tops)[i];
      // fraction of the amplitudes the op touches: its controls must be 1
      // (a phase op's masks hold its targets too)
      double frac = std::ldexp(
          1.0, -(__builtin_popcount(o.lctrl) + __builtin_popcountll(o.gctrl)));
      if (o.kind == kOpDense1 && o.mux != kMuxNone) {
        // a mux op applies m on half of those amplitudes and m2 on the
        // other half; an identity half changes nothing
        frac *= 0.5 * ((is_identity2(o.m) ? 0 : 1) +
                       (is_identity2(o.m2) ? 0 : 1));
      } else if (o.kind == kOpDense1 && is_identity2(o.m)) {
        frac = 0;
      }
      stats->flops_per_amp += (o.kind == kOpDense1 ? 14.0 : 6.0) *
                              (o.kind == kOpPhaseBlock ? 1.0 : frac);
    }
  }
  // Phase-block records follow the pass's ops, in whole TileOp slots.
  for (const Blob& bl : blobs) {
    const size_t at = tops->size();
    const size_t nrec = (bl.bytes.size() + sizeof(TileOp) - 1) / sizeof(TileOp);
    tops->resize(at + nrec);
    std::memcpy(static_cast<void*>(&(*tops)[at]), bl.bytes.data(), bl.bytes.size());
    (*tops)[bl.op].blob = int32_t((at - size_t(bl.op)) * sizeof(TileOp));
  }
  tpasses->push_back(tp);
  return "";
}

void make_plan(const std::vector<HostGate>& G, int n, int b,
               const PlanOptions& o, Plan* plan) {
  *plan = Plan();
  int strategy = o.strategy;
  if (strategy == 0) strategy = (n >= o.reg_log2 + 2) ? 2 : 1;
  if (strategy == 2 && n < o.reg_log2 + 2) strategy = 1;
  if (strategy == 1) {
    for (size_t i = 0; i < G.size(); ++i) add_plain(G, int(i), n, b, plan);
  } else if (strategy == 2) {
    plan_tiled(G, n, b, o, plan);
  } else {
    plan_fused(G, n, b, o, plan);
  }
}

}  // namespace qsv
