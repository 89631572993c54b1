/*
 * qsv -- dense quantum state-vector engine for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libqsv.so.  Plain pointers and sizes only.
 *
 * The operation every call serves is the evaluation step of both simulation
 * methods compared in the paper: apply a circuit's gates to a 2^n complex
 * amplitude vector, then reduce it to the output probability vector
 * (Section IV.A, Evaluator: the state-vector run followed by the conversion
 * of the state to probabilities).  Full-circuit execution runs it once on the
 * whole vector; circuit cutting runs it on every subcircuit variant.
 *
 * Conventions shared by all calls
 * -------------------------------
 * - State layout: one contiguous device array a[0 .. 2^n - 1] of interleaved
 *   (re, im) pairs, float for QSV_C64 (8 B per amplitude) and double for
 *   QSV_C128 (16 B per amplitude); Table III sizes the complex128 case as
 *   16 * 2^n bytes.
 * - Index convention: little-endian.  Bit q of an index is the value of
 *   qubit q.
 * - Gate matrices: 2^k x 2^k complex, row-major, interleaved (re, im) doubles
 *   in host memory.  Row/column index r = sum_j bit(q = targets[j]) * 2^j,
 *   i.e. targets[0] is the least significant bit of r.  A gate with controls
 *   acts only on amplitudes whose control bits are all 1.
 * - Errors: every call returns a qsv_status; the library never aborts.
 *   Argument validation is synchronous, on the host, before any device work,
 *   and leaves the state unchanged on error.  qsv_last_error() returns a
 *   thread-local message for the last failing call on the calling thread.
 * - Device faults surface as QSV_ERR_DEVICE at the next call that
 *   synchronises; the state is then marked failed and later calls on it
 *   return QSV_ERR_DEVICE.  Other states are unaffected.
 * - Ownership: input arrays (qubit lists, matrices, circuits) are copied or
 *   consumed before the call returns; the caller may free them at once.
 *   Output buffers belong to the caller.
 * - Streams: each state is bound to one HIP stream (hipStream_t passed as
 *   void*, NULL = the default stream).  Apply calls only enqueue work and
 *   return; calls that return host data (norm, marginal, sample, get) wait
 *   for the state's stream.  One state must not be used from two threads at
 *   once; different states are independent.
 */
#ifndef QSV_H
#define QSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QSV_OK = 0,
  QSV_ERR_INVALID_ARG = 1,   /* bad pointer, qubit, size or option value */
  QSV_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
  QSV_ERR_DEVICE = 3,        /* a HIP call or kernel failed */
  QSV_ERR_UNSUPPORTED = 4,   /* unknown precision, gate or strategy */
  QSV_ERR_BUDGET = 5,        /* request larger than an admission budget */
  QSV_ERR_CANCELLED = 6,     /* a queued request was cancelled */
  QSV_ERR_TIMEOUT = 7        /* a wait ended before the request finished */
} qsv_status;

typedef enum { QSV_C64 = 1, QSV_C128 = 2 } qsv_precision;

#define QSV_MAX_QUBITS 34  /* 2^34 c64 amplitudes = 128 GiB fit in 288 GB */
#define QSV_MAX_TARGETS 5  /* largest k of a dense gate or fused block */

typedef struct qsv_state_s* qsv_state;

/* ---------------------------------------------------------------- states */

/* Allocate a 2^n_qubits state of precision prec on the current HIP device,
 * bound to hip_stream.  The library owns the 2^n * (8|16) bytes and frees
 * them in qsv_free.  The contents are undefined until initialised.
 * 1 <= n_qubits <= QSV_MAX_QUBITS.  The state vector of full-circuit
 * simulation in single or double precision (Section III.B), sized as in
 * Table III (16 * 2^n bytes for complex128, half that for complex64); one
 * GPU's HBM holds 34 complex64 or 33 complex128 qubits.  Errors:
 * QSV_ERR_INVALID_ARG for n_qubits out of range or a NULL out,
 * QSV_ERR_UNSUPPORTED for an unknown precision, QSV_ERR_OUT_OF_MEMORY when
 * the device allocation fails (*out is then untouched). */
qsv_status qsv_alloc(int32_t n_qubits, int32_t prec, void* hip_stream,
                     qsv_state* out);

/* Bind a state to caller-owned device memory (e.g. a torch tensor's
 * storage) of at least 2^n * (8|16) bytes, 16-byte aligned.  The caller
 * keeps the memory alive until qsv_free; qsv_free does not release it.  The
 * same state vector as qsv_alloc (Section III.B, Table III sizes) in memory
 * the caller already holds.  Errors: QSV_ERR_INVALID_ARG for a NULL or
 * misaligned pointer, too few bytes or n_qubits out of range,
 * QSV_ERR_UNSUPPORTED for an unknown precision. */
qsv_status qsv_wrap(int32_t n_qubits, int32_t prec, void* device_ptr,
                    size_t bytes, void* hip_stream, qsv_state* out);

/* Release a state (and, for qsv_alloc states, its memory).  NULL is a
 * no-op.  Waits for the state's pending work first.  (Control call.) */
qsv_status qsv_free(qsv_state s);

/* Set the state to the computational basis state |index>: a[index] = 1,
 * every other amplitude 0.  index < 2^n.  (Each subcircuit variant starts
 * from such a state before its cut-input preparation, Section III.A.) */
qsv_status qsv_init_basis(qsv_state s, uint64_t index);

/* ----------------------------------------------------------------- gates */

/* Apply one gate: the 2^k x 2^k matrix on targets[0..k-1], controlled on
 * controls[0..c-1] (all must be 1).  1 <= k <= QSV_MAX_TARGETS; targets and
 * controls are distinct qubits < n.  The update is, for every base index i
 * with all target bits 0 and all control bits 1,
 *   a'[i_r] = sum_s U[r][s] a[i_s],  i_r = i | sum_j bit_j(r) << targets[j].
 * This is the per-gate kernel of full-circuit execution (Section III.B,
 * gates u1/u3/CNOT of the cache-blocking example).  Gates on 4 or 5 targets
 * without controls run on the matrix cores (the matrix rounded once to FP32
 * for complex64 states); all others on the vector units.  Amplitudes
 * outside the update keep their values, but a pass may store some of them
 * back unchanged (controls on the lowest qubits), so no other stream may
 * write the state's memory meanwhile.  Enqueued on the state's stream; the
 * matrix is copied before return. */
qsv_status qsv_apply_gate(qsv_state s, const int32_t* targets, int32_t k,
                          const int32_t* controls, int32_t c,
                          const double* matrix);

/* A gate list, all arrays host-resident, consumed before return.
 *   k[g], c[g]  : number of targets / controls of gate g
 *   qubits      : concatenated per gate: k[g] targets then c[g] controls
 *   matrices    : concatenated per gate: 2^k[g] x 2^k[g] complex matrices
 *                 (interleaved re/im doubles, row-major) */
typedef struct {
  size_t n_gates;
  const int32_t* k;
  const int32_t* c;
  const int32_t* qubits;
  const double* matrices;
} qsv_circuit;

typedef enum {
  QSV_PLAN_AUTO = 0,   /* tiled runs, plain kernels where a tile cannot go */
  QSV_PLAN_PLAIN = 1,  /* one kernel per gate */
  QSV_PLAN_TILED = 2,  /* LDS-staged tiles applying runs of gates per pass */
  QSV_PLAN_FUSED = 3   /* fused k-qubit unitaries (built in FP64 on device) */
} qsv_strategy;

/* Options of qsv_apply_fused; all-zero (or NULL) selects defaults.
 *   tile_log2  : tile size L (amplitudes per tile = 2^L), 8..13, with
 *                L - reg_log2 <= 9 (default 12)
 *   k_max      : widest fused block, 1..5 (default 5)
 *   low_qubits : qubits 0..low_qubits-1 belong to every tile so that HBM
 *                accesses are contiguous runs (default 4)
 *   reg_log2   : amplitudes per thread inside a tile, as log2: 3, 4 or 5
 *                (5 for c64 only; default 4)
 * This is the single-GPU form of the chunking and cache blocking of
 * Section III.B: a tile of 2^L amplitudes plays the role of a 2^nc chunk
 * (blocking_qubits), and the planner reorders commuting gates so that runs
 * of gates touch only the tile's qubits. */
typedef struct {
  int32_t strategy;
  int32_t tile_log2;
  int32_t k_max;
  int32_t low_qubits;
  int32_t reg_log2;
} qsv_fuse_opts;

/* Plan and apply a whole gate list: the transpile-time cache blocking of
 * Section III.B (qubit and gate reordering onto the qubits of one chunk,
 * here an LDS/register tile) followed by the passes it produces.  The
 * result equals applying the gates one by one in list order (up to
 * rounding): passes only regroup gates that commute (disjoint qubits, or
 * both diagonal).  Enqueued on the state's stream.  Errors (nothing is
 * enqueued): QSV_ERR_INVALID_ARG for a bad gate (qubit out of range,
 * duplicate qubit, k outside 1..5, non-finite matrix) or option,
 * QSV_ERR_OUT_OF_MEMORY when the program buffer cannot grow. */
qsv_status qsv_apply_fused(qsv_state s, const qsv_circuit* circ,
                           const qsv_fuse_opts* opts);

/* Outputs computed with a circuit (qsv_apply_fused_outputs).  Each is
 * optional:
 *   probs_dev  : device, 2^n probabilities p_i = |a_i|^2 as float
 *                (probs_fp64 = 0) or double, as qsv_probabilities writes
 *   marg_m     : 0, or the marginal of marg_qubits[0..marg_m-1] (host,
 *                distinct, 1 <= marg_m <= 20) into marg_out (host, 2^marg_m
 *                doubles), as qsv_marginal
 *   n_shots    : 0, or n_shots draws (<= 2^32) with shot_seed into
 *                shots_out (host), as qsv_sample */
typedef struct {
  void* probs_dev;
  int32_t probs_fp64;
  int32_t marg_m;
  const int32_t* marg_qubits;
  double* marg_out;
  uint64_t n_shots;
  uint64_t shot_seed;
  uint64_t* shots_out;
} qsv_outputs;

/* qsv_apply_fused followed by the requested outputs, with the reductions
 * folded into the circuit's last pass when it is a tile pass: that pass
 * writes the probabilities and, per tile, FP64 sums of p over the tile's
 * amplitudes grouped by the marginal's qubits and by the sampler's
 * 1024-amplitude blocks, and two small kernels add those partial sums over
 * the tiles in increasing tile order, so no output reads the state again
 * (the distribution of specified qubits of the Builder, Section IV.A, and
 * the shots of Section III.A, streamed out of the last gate pass).  The
 * results equal qsv_apply_fused + qsv_probabilities + qsv_marginal +
 * qsv_sample up to the order of the FP64 sums (so a draw may differ only
 * where its uniform falls within rounding of a CDF step); a given state
 * and request always give the same bits.  Outputs the last pass cannot
 * fold (a plain or fused last pass, a marginal spanning more than
 * tile_log2 - reg_log2 tile qubits, n <= 10 for shots) run as the separate
 * kernels.  The state keeps its final amplitudes.  Waits for the stream
 * when a host output is requested.  Errors: those of qsv_apply_fused, and
 * QSV_ERR_INVALID_ARG for a bad output request (nothing is enqueued). */
qsv_status qsv_apply_fused_outputs(qsv_state s, const qsv_circuit* circ,
                                   const qsv_fuse_opts* opts,
                                   const qsv_outputs* outs);

/* Statistics of the last qsv_apply_fused on this state (the passes of the
 * cache-blocked plan, Section III.B):
 *   out[0] passes launched, out[1] gates, out[2] algorithmic HBM bytes
 *   (sum over passes of bytes read + written), out[3] tile passes,
 *   out[4] plain passes, out[5] fused passes, out[6] tile segments,
 *   out[7] host planning time in nanoseconds, out[8] tile ops,
 *   out[9] phase blocks (runs of diagonal gates applied as one phase
 *   polynomial), out[10] diagonal gates inside phase blocks, out[11] the
 *   outputs the last pass folded (qsv_apply_fused_outputs: bit 0
 *   probabilities, bit 1 marginal, bit 2 shots), out[12] real flops the
 *   tile ops define (14 per amplitude a dense 2x2 op changes, 6 per
 *   amplitude a diagonal op, phase op or phase block multiplies).
 *   n_out <= 13 entries. */
qsv_status qsv_last_plan_stats(qsv_state s, uint64_t* out, int32_t n_out);

/* Per-pass timing of the passes of Section III.B's cache-blocked plan.
 * While enabled (enable != 0), qsv_apply_fused records a HIP event pair
 * around every pass it launches, on the state's stream.
 * qsv_pass_times waits for the last qsv_apply_fused to finish and writes,
 * for its first min(cap, passes) passes, the kernel time in milliseconds
 * (ms_out) and the pass kind (kinds_out: 1 plain, 2 tile, 3 fused; may be
 * NULL); *count receives the number of passes recorded. */
qsv_status qsv_set_profiling(qsv_state s, int32_t enable);
qsv_status qsv_pass_times(qsv_state s, float* ms_out, int32_t* kinds_out,
                          int32_t cap, int32_t* count);

/* Autotuning of the chunk parameters of Section III.B's cache blocking
 * (the evaluator of Section IV.A fixes its blocking qubits per machine;
 * here the tile size, the low qubits of every tile and the amplitudes per
 * thread are chosen per state width, precision and circuit structure).
 * Plans the circuit under the defaults and under every valid (tile_log2,
 * low_qubits, reg_log2), ranks the latter by a cost model, and times the
 * defaults and the best-ranked candidates, max_timed in all (0: 6; at most
 * 64), one run each after one untimed run: the kernel time of the passes,
 * by HIP events.  The fastest wins if it beats the defaults by 2 % or more,
 * else the defaults stay.  Runs the circuit on the state, so the state's
 * contents are overwritten (initialise it again afterwards); blocks until
 * the runs finish.  base: strategy and k_max (NULL: defaults; other fields
 * ignored).  The result is cached per (device, n, precision, strategy,
 * k_max, circuit structure: gate shapes, qubits and diagonal form, not the
 * matrix values); a cached call runs nothing and sets *from_cache = 1.
 * Outputs: *best (filled options for qsv_apply_fused), *best_ms and
 * *default_ms (may be NULL), *from_cache (may be NULL).  Errors:
 * QSV_ERR_INVALID_ARG for a NULL best, max_timed outside 0..64 or a bad
 * circuit, QSV_ERR_UNSUPPORTED for an unknown strategy, QSV_ERR_DEVICE if a
 * run fails. */
qsv_status qsv_autotune_fused(qsv_state s, const qsv_circuit* circ,
                              const qsv_fuse_opts* base, int32_t max_timed,
                              qsv_fuse_opts* best, float* best_ms,
                              float* default_ms, int32_t* from_cache);

/* Host-only planner dry run of the cache blocking of Section III.B (no
 * device work; usable without a GPU).
 * For n_qubits and precision prec, writes for each gate g:
 *   gate_pass[g]  : index of the pass that applies g
 *   gate_order[j] : the j-th gate applied (a permutation of 0..n_gates-1)
 * and for each pass p (< *n_passes, at most n_gates):
 *   pass_kind[p]  : 1 plain, 2 tile, 3 fused
 *   pass_qubits[p]: bit mask of the pass's qubit set (tile: its 2^L qubit
 *                   set; fused: the block's qubits; plain: the gate's) */
qsv_status qsv_plan_describe(const qsv_circuit* circ, int32_t n_qubits,
                             int32_t prec, const qsv_fuse_opts* opts,
                             int32_t* gate_pass, int32_t* gate_order,
                             int32_t* pass_kind, uint64_t* pass_qubits,
                             int32_t* n_passes);

/* Host-only dry run of the device program (no device work): plans the
 * circuit as qsv_apply_fused would (the cache-blocking transpilation of
 * Section III.B) and builds its tile programs, then writes out[0] passes,
 * out[1] tile passes, out[2] tile segments, out[3] tile ops, out[4] phase
 * blocks, out[5] diagonal gates inside phase blocks, out[6] real flops the
 * tile ops define (as out[12] of qsv_last_plan_stats) (host array;
 * n_out <= 7 entries).  QSV_ERR_UNSUPPORTED for an unknown precision,
 * QSV_ERR_INVALID_ARG for a bad circuit, option, n_qubits or buffer. */
qsv_status qsv_plan_program_stats(const qsv_circuit* circ, int32_t n_qubits,
                                  int32_t prec, const qsv_fuse_opts* opts,
                                  uint64_t* out, int32_t n_out);

/* Testing aid for the failure paths (Control call.): kind 1 makes the
 * next `count` device allocations of the library (states, program
 * buffers, scratch) fail as out of memory, without allocating; kind 2 makes
 * the next `count` device calls made for a state fail as device errors,
 * without making them, so that the state turns failed (every later call on
 * it returns QSV_ERR_DEVICE) while other states are unaffected.  count 0
 * clears the kind.  Process-wide.  QSV_ERR_INVALID_ARG for another kind or
 * a negative count. */
qsv_status qsv_debug_inject(int32_t kind, int32_t count);

/* Testing aid (host only, no device work): plan the circuit with the
 * tiled strategy (Section III.B's cache blocking) for n_qubits <= 16,
 * build the exact device program the
 * tile kernel would run (passes, register segments, folded and merged
 * ops) and execute it on the host in complex128 on `state` (2^n
 * interleaved re/im doubles, updated in place).  Lets the planner's
 * reordering and gate merging be checked on a machine without a GPU. */
qsv_status qsv_debug_emulate_tiled(const qsv_circuit* circ, int32_t n_qubits,
                                   const qsv_fuse_opts* opts, double* state);

/* Standard gate matrix by name into out (2^k x 2^k complex, interleaved),
 * with *k_out its target count.  Names: "h","x","y","z","s","sdg","p"(1),
 * "u3"(3: theta, phi, lambda; the OpenQASM 2 U3, used as u3 in the
 * cache-blocking example of Section III.B), "id".  out holds >= 8 doubles. */
qsv_status qsv_gate_matrix(const char* name, const double* params,
                           int32_t n_params, double* out, int32_t* k_out);

/* qsv_gate_matrix for `count` gates of one name (the u1/u3 gates of
 * Section III.B's example, in bulk): params holds count x n_params values
 * (gate i uses params[i*n_params ...]); out receives count consecutive 2x2
 * matrices (8 doubles each). */
qsv_status qsv_gate_matrices(const char* name, const double* params,
                             int32_t n_params, size_t count, double* out);

/* ------------------------------------------------------------ reductions */

/* p_i = |a_i|^2 for all 2^n amplitudes into out_dev (caller-owned device
 * memory), as double if out_fp64 != 0 else float.  c64 states compute p in
 * FP64 from the FP32 amplitudes before rounding.  (The probability vector
 * the evaluator returns, Section IV.A.)  Enqueued on the state's stream. */
qsv_status qsv_probabilities(qsv_state s, void* out_dev, int32_t out_fp64);

/* Sum of p_i in FP64 with Neumaier compensation in a fixed-order tree
 * (bitwise reproducible for a given state).  The total of the probability
 * vector the evaluator returns (Section IV.A), which the Verifier's error
 * margin presupposes to be one; reported rather than assumed, since
 * rounding moves it.  Waits for the stream; errors: QSV_ERR_INVALID_ARG for
 * a NULL state or out, QSV_ERR_DEVICE for a failed state. */
qsv_status qsv_norm(qsv_state s, double* out);

/* Divide every amplitude by sqrt(norm); returns the norm before scaling in
 * *norm_out (may be NULL).  Restores a probability vector summing to one
 * (Section IV.A) after rounding drift; optional, never implicit.  Waits
 * for the stream; errors: QSV_ERR_INVALID_ARG for a NULL state or a zero
 * norm, QSV_ERR_DEVICE for a failed state. */
qsv_status qsv_renormalize(qsv_state s, double* norm_out);

/* (For callers that cannot allocate.)  qsv_renormalize for callers that
 * may not allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid allocation): the same kernels and
 * the same result bit for bit, with the norm's partial sums in a fixed
 * scratch array of 4 MiB + 256 B that the library holds on each device
 * until the process ends, so no call allocates or frees memory.  That bounds the
 * state to 30 qubits (2^18 partial pairs); wider states return
 * QSV_ERR_INVALID_ARG and nothing runs.  All calls on one device share the
 * array: calls that overlap on one device (states on different streams or
 * host threads) race and must be serialised by the caller.  Other errors
 * as qsv_renormalize. */
qsv_status qsv_renormalize_noalloc(qsv_state s, double* norm_out);

/* Marginal distribution of the specified qubits (the Builder's
 * distribution of specified qubits, Section IV.A):
 *   out[j] = sum of p_i over i with bit qubits[l] of i == bit l of j,
 * qubits[0] the least significant bit of j; 1 <= m <= 20, distinct qubits.
 * out_host holds 2^m doubles.  FP64 with Neumaier compensation in a fixed
 * order.  Waits for the stream. */
qsv_status qsv_marginal(qsv_state s, const int32_t* qubits, int32_t m,
                        double* out_host);

/* n_shots basis indices drawn from p (shots, Section III.A).  Draw j uses
 * u_j = (SplitMix64(seed, j) >> 11) * 2^-53, SplitMix64(seed, j) being
 * output j of the SplitMix64 generator (Steele, Lea & Flood 2014) seeded
 * with seed, and returns the least i with C(i) > u_j * C(2^n - 1), C the
 * inclusive FP64 cumulative sum of p (accumulated per 1024-amplitude block,
 * then within the block).  out_host receives n_shots indices in draw
 * order.  n_shots <= 2^32.  Waits for the stream. */
qsv_status qsv_sample(qsv_state s, uint64_t n_shots, uint64_t seed,
                      uint64_t* out_host);

/* Relabel qubits: qubit q becomes qubit perm[q] (perm: host, a
 * permutation of 0..n-1), i.e. the amplitude of index i moves to the index
 * whose bit perm[q] is bit q of i.  This is the data movement of the
 * paper's swap insertion (Section III.B): one pass that brings busy high
 * qubits to low positions.  Out of place into a second state-sized buffer
 * that the state allocates on first use and keeps until qsv_free; for a
 * state from qsv_alloc the two buffers then trade places (the device
 * pointer reported by qsv_info changes), for a wrapped state the result is
 * copied back.  Pure data movement: bit-exact.  Asynchronous. */
qsv_status qsv_permute_qubits(qsv_state s, const int32_t* perm);

/* The k most probable outcomes (1 <= k <= min(65536, 2^n)): idx_out[k]
 * and p_out[k] (host), ordered by probability, largest first, and by index
 * among equal probabilities.  The probability of outcome i is decided as
 * p = re*re + im*im in FP64 with each product and the sum rounded
 * separately (for c64 the amplitudes are widened to FP64 first), so the
 * selection equals that of any plain FP64 evaluation.  This is the literal
 * top-k alternative to the marginal over specified qubits (Section IV.A).
 * Reads the state about seven times (radix select on 12-bit digits), waits. */
qsv_status qsv_top_k(qsv_state s, uint32_t k, uint64_t* idx_out,
                     double* p_out);

/* Expectation values <psi|P_t|psi> of n_terms Pauli strings, the X/Y/Z
 * observables whose eigenbases the cut identity uses (Section III.A,
 * eq 3.1), as an output beside the probability vector (host arrays):
 * x_masks[t] has bit q set where P_t acts on qubit q with X or Y, z_masks[t]
 * where it acts with Z or Y (Y = i X Z).  out[t] (host) is the real value
 * for the state as it is (not renormalised); sums are FP64 with Neumaier
 * compensation in a fixed order.  Masks naming a qubit >= n are rejected.
 * One read of the state (plus its partner amplitudes) per term; waits. */
qsv_status qsv_expectation_pauli(qsv_state s, int32_t n_terms,
                                 const uint64_t* x_masks,
                                 const uint64_t* z_masks, double* out);

/* ------------------------------------------------- batched cut variants */

/* One subcircuit variant (Section III.A): a width-qubit circuit started in
 * |0...0>, whose cut-input qubits are first prepared in |0>, |1>, |+> or
 * |+i> (labels 0..3; the eigenstates of eqs 3.3-3.6, |+i> = S H |0>) and
 * whose cut-output qubits are finally rotated so that a computational-basis
 * readout measures I (basis 0: nothing), X (basis 1: H) or Y (basis 2:
 * S-dagger then H).  The body gates must be one-target dense gates (any
 * controls) or diagonal gates on at most two targets (or masked phases).
 * reg_log2 + 2 <= width <= QSV_BATCH_MAX_WIDTH (so width >= 6 at the
 * default reg_log2 = 4).  All arrays are host memory. */
#define QSV_BATCH_MAX_WIDTH 24
typedef struct {
  int32_t width;
  qsv_circuit body;
  int32_t n_inputs;
  const int32_t* input_qubits;
  const int32_t* input_labels;
  int32_t n_outputs;
  const int32_t* output_qubits;
  const int32_t* output_bases;
} qsv_variant;

/* Options of a batch; all-zero (or NULL) selects defaults.
 *   tile_log2 : tile size for every variant wider than it (default 12 c64,
 *               11 c128); variants at most this wide run in one tile
 *   reg_log2  : amplitudes per thread, as log2 (4, or 5 for c64)
 *   grid      : work-groups of each phase launch (default: as many as
 *               stay resident, from the kernel's occupancy)
 *   autotune  : time (tile_log2, reg_log2) candidates at creation and keep
 *               the fastest
 *   use_graph : capture the phase launches in a hipGraph and replay it
 *   out_fp64  : probabilities as double (else float) */
typedef struct {
  int32_t tile_log2;
  int32_t reg_log2;
  int32_t grid;
  int32_t autotune;
  int32_t use_graph;
  int32_t out_fp64;
} qsv_batch_opts;

typedef struct qsv_batch_s* qsv_batch;

/* Plan count variants of precision prec (the subcircuit variants of
 * Section III.A, which the evaluator runs independently, Section IV.A) for
 * phase launches on hip_stream.  Every variant is planned into tile passes
 * and the programs are uploaded once.  Phase p applies pass p of every
 * variant that has one: the phase's tiles, over all those variants, are
 * divided among the work-groups by their estimated cost (ops per tile), and
 * a kernel boundary separates the phases.  A variant that fits one tile
 * starts from |0...0> in registers and is done in phase 0; a wider one keeps
 * its state in the batch's scratch buffer between phases.  Each tile is
 * computed the same way wherever it runs, so a variant's probabilities do
 * not depend on the rest of the batch.  Allocates the program and the
 * scratch buffer.  Errors: QSV_ERR_INVALID_ARG for a bad variant (width,
 * labels, gates a tile cannot hold) or option, QSV_ERR_UNSUPPORTED for an
 * unknown precision, QSV_ERR_OUT_OF_MEMORY when an allocation fails. */
qsv_status qsv_batch_create(const qsv_variant* vars, size_t count,
                            int32_t prec, const qsv_batch_opts* opts,
                            void* hip_stream, qsv_batch* out);

/* Ragged output layout: variant i's 2^width probabilities occupy elements
 * [offsets[i], offsets[i+1]) of the output; offsets holds count + 1.  The
 * per-variant probability vectors the reconstruction consumes
 * (Section III.A). */
qsv_status qsv_batch_out_offsets(qsv_batch b, uint64_t* offsets);

/* Enqueue the batch writing all probability vectors into out_dev
 * (caller-owned device memory of offsets[count] floats or doubles): one
 * kernel launch per phase, or, with use_graph, one replay of a hipGraph
 * holding those launches (captured at the first call for this out_dev, and
 * captured again when out_dev changes).  Asynchronous on the batch's
 * stream; the evaluation of every variant of Section III.A / IV.A.
 * Errors: QSV_ERR_INVALID_ARG for a NULL batch or buffer, QSV_ERR_DEVICE
 * when a launch fails. */
qsv_status qsv_batch_launch(qsv_batch b, void* out_dev);

/* out[0] variants, out[1] tile passes, out[2] tiles processed, out[3] ops,
 * out[4] scratch bytes, out[5] tile_log2, out[6] reg_log2, out[7] grid,
 * out[8] variants run in one tile, out[9] amplitude updates (sum over
 * variants of 2^width x ops).  n_out <= 10.  (Control call.) */
qsv_status qsv_batch_stats(qsv_batch b, uint64_t* out, int32_t n_out);

/* Release a batch (waits for its stream).  NULL is a no-op.  (Control
 * call.) */
qsv_status qsv_batch_free(qsv_batch b);

/* --------------------------------------------------------------- serving */

/* A request server: requests (circuits of different widths, depths and
 * precisions) are submitted as they arrive; a scheduler thread admits them
 * first-come first-served while the device memory they need fits the
 * budget, the way the evaluator sizes its worker pool by the memory each
 * worker needs (Section IV.A).  A request's need counts device bytes only
 * (pinned host result buffers are not HBM): its state (2^w x 8 or 16
 * bytes), its output on the device, sampling scratch and an allowance for
 * its program, plus 1/8 for pooled block rounding.  Device blocks and
 * states the server keeps for reuse count against the budget too: before
 * an admission that would not fit beside them they are freed.  Admitted
 * requests of width <= small_width whose gates fit tiles are packed into
 * batch slots (one group of phase launches per precision); wider ones run
 * on their own state.  Groups run on up to n_streams streams at once, so work
 * admitted while other work is on the GPU overlaps it (continuous
 * batching).  The path and kernels a request takes depend only on the
 * request, so its result is the same alone or in any mix.
 *   budget_bytes : admission budget (0 = 256e9)
 *   max_batch    : most requests per batch launch (0 = 256)
 *   small_width  : widest request packed into batch slots (0 = 20)
 *   n_streams    : concurrent streams (0 = 4)
 *   serial       : 1 = one request at a time, nothing overlaps (baseline) */
typedef struct {
  uint64_t budget_bytes;
  int32_t max_batch;
  int32_t small_width;
  int32_t n_streams;
  int32_t serial;
} qsv_server_opts;

/* One request: the circuit runs on |0...0> of `width` qubits; the output
 * is the probability vector (float for c64, double for c128) or `shots`
 * samples drawn as in qsv_sample with `seed`. */
typedef struct {
  int32_t width;
  int32_t prec;
  qsv_circuit body;
  int32_t want_samples;
  uint64_t shots;
  uint64_t seed;
} qsv_request;

/* A finished request.  data points to host memory owned by the server
 * until qsv_server_release: n_out floats/doubles (probabilities) or n_out
 * uint64 samples.  Times are seconds on qsv_clock(). */
typedef struct {
  int32_t status;
  int32_t width;
  int32_t prec;
  int32_t is_samples;
  int32_t batched;
  int32_t pad;
  uint64_t n_out;
  const void* data;
  double t_submit, t_admit, t_start, t_done;
} qsv_result;

typedef struct qsv_server_s* qsv_server;

/* Create a server (no device work until the first request runs): the
 * evaluator's memory-sized worker pool of Section IV.A as one scheduler.
 * Errors: QSV_ERR_INVALID_ARG for bad options or a NULL out. */
qsv_status qsv_server_create(const qsv_server_opts* opts, qsv_server* out);

/* Validate and enqueue a request (a circuit for the evaluator, Section IV.A;
 * inputs are copied); returns its ticket.
 * QSV_ERR_BUDGET if the request alone exceeds the budget.  The pinned host
 * buffer for its result is taken when the request is admitted to the
 * device; if that allocation fails the request completes with
 * QSV_ERR_OUT_OF_MEMORY (reported by qsv_server_wait). */
qsv_status qsv_server_submit(qsv_server s, const qsv_request* req,
                             uint64_t* ticket);

/* Block until the ticket's request has finished and describe its result
 * (the probability vector or shots of Sections III.A / IV.A).  Errors:
 * QSV_ERR_INVALID_ARG for an unknown ticket; the request's own status is
 * in out->status. */
qsv_status qsv_server_wait(qsv_server s, uint64_t ticket, qsv_result* out);

/* qsv_server_wait with a time limit: returns QSV_ERR_TIMEOUT if the
 * request has not finished within timeout_s seconds (it stays queued or
 * running and can be waited for again), else as qsv_server_wait (the
 * probability vector or shots of Sections III.A / IV.A).  Errors:
 * QSV_ERR_INVALID_ARG for an unknown ticket or a negative or non-finite
 * timeout. */
qsv_status qsv_server_wait_timeout(qsv_server s, uint64_t ticket,
                                   double timeout_s, qsv_result* out);

/* Withdraw a request that is still queued (not yet admitted to the
 * device): it finishes with status QSV_ERR_CANCELLED (qsv_server_wait
 * reports it) and nothing of it runs.  QSV_ERR_INVALID_ARG for an unknown
 * ticket or a request already admitted or finished.  (Control call.) */
qsv_status qsv_server_cancel(qsv_server s, uint64_t ticket);

/* Free the ticket's result buffers.  (Control call.) */
qsv_status qsv_server_release(qsv_server s, uint64_t ticket);

/* out[0] submitted, out[1] completed, out[2] batch launches, out[3] single
 * launches, out[4] peak reserved bytes, out[5] most groups in flight at
 * once, out[6] rejected, out[7] times the idle blocks and cached states
 * were freed to admit a request.  n_out <= 8.  (Control call.) */
qsv_status qsv_server_stats(qsv_server s, uint64_t* out, int32_t n_out);

/* Finish queued work, stop the scheduler and free everything.  (Control
 * call.) */
qsv_status qsv_server_destroy(qsv_server s);

/* The library's steady clock, in seconds.  (Control call.) */
double qsv_clock(void);

/* ---------------------------------------------------- cut reconstruction */

/* A wire-cut problem (Section III.A): n_sub subcircuits joined by n_cuts
 * cut wires.  Subcircuit s has widths[s] local qubits; for each local qubit
 * (arrays concatenated over s, sum of widths entries each):
 *   out_qubit : the uncut qubit whose final value is measured there, or -1
 *   cut_in    : the cut whose downstream end initialises it, or -1
 *   cut_out   : the cut whose upstream end is measured there, or -1
 * Every local qubit is measured exactly once (out_qubit >= 0 or
 * cut_out >= 0, not both); every cut has one upstream and one downstream end
 * in two different subcircuits; every uncut qubit 0..n_qubits-1 is the
 * out_qubit of exactly one local qubit.
 *
 * Variants of subcircuit s are numbered by its cut ends taken in increasing
 * local-qubit order (a downstream end before an upstream end on the same
 * qubit), the first end least significant: a downstream end is a digit in
 * 0..3 (initial state |0>, |1>, |+>, |+i>), an upstream end a digit in 0..2
 * (readout basis I, X, Y; X is read after H, Y after S-dagger then H).
 * This is the order of the prologue / epilogue labels of qsv_variant.
 *
 * Limits: 1 <= n_sub <= 16, 0 <= n_cuts <= 8, widths 1..24, at most 6 cut
 * ends per subcircuit, 1 <= n_qubits <= 30. */
typedef struct {
  int32_t n_sub;
  int32_t n_cuts;
  int32_t n_qubits;
  const int32_t* widths;
  const int32_t* out_qubit;
  const int32_t* cut_in;
  const int32_t* cut_out;
} qsv_cut_spec;

/* Device workspace that qsv_cut_reconstruct needs for this problem (the
 * reconstruction of Section III.A).
 * Validates the specification (QSV_ERR_INVALID_ARG with a message). */
qsv_status qsv_cut_workspace_bytes(const qsv_cut_spec* spec, uint64_t* bytes);

/* Probability vector of the uncut circuit from its subcircuits' variant
 * probability vectors (Section III.A: per subcircuit, the four terms of
 * every cut end, by shot attribution (eq 3.7) for upstream ends and by the
 * initial-state combinations of eqs 3.3-3.6 for downstream ends; then
 * p(x) = (1/2)^K times the sum over all 4^K term choices of the product over
 * subcircuits of their term vectors at x's bits).
 *   probs_dev  : device buffer of probs_elems FP32 (probs_fp64 = 0) or FP64
 *                entries holding every variant's 2^w vector (little-endian
 *                index, as written by qsv_batch_launch or qsv_probabilities)
 *   offsets    : host, for s = 0..n_sub-1 and each variant v of s in the
 *                order above: the element offset of its vector in probs_dev;
 *                each vector must lie inside probs_elems
 *   workspace  : device, at least qsv_cut_workspace_bytes; owned by the
 *                caller and not used by anything else until the work is done
 *   out_dev    : device, 2^n_qubits FP64, written (bit q of the index =
 *                uncut qubit q)
 * All arithmetic is FP64.  The call validates everything on the host first
 * (nothing is launched on an error), copies its tables into the workspace on
 * the stream, waits for that copy, then enqueues two kernels and returns. */
qsv_status qsv_cut_reconstruct(const qsv_cut_spec* spec, const void* probs_dev,
                               int32_t probs_fp64, uint64_t probs_elems,
                               const uint64_t* offsets, void* workspace,
                               uint64_t workspace_bytes, double* out_dev,
                               void* hip_stream);

/* ---------------------------------------------------- copies and control */

/* Copy all amplitudes to / from host memory (2^n interleaved pairs of the
 * state's precision): the state-vector copy between device and host that
 * the evaluator makes before converting to probabilities (Section IV.A);
 * here for tests and checkpoints, since every output is computed on the
 * device.  Waits.  Errors: QSV_ERR_INVALID_ARG for a NULL state or buffer,
 * QSV_ERR_DEVICE for a failed copy or state. */
qsv_status qsv_get_amplitudes(qsv_state s, void* host_out);
qsv_status qsv_set_amplitudes(qsv_state s, const void* host_in);

/* Device pointer, qubit count and precision of a state.  (Control call.) */
qsv_status qsv_info(qsv_state s, void** device_ptr, int32_t* n_qubits,
                    int32_t* prec);

/* Wait for the state's stream; reports deferred device errors.  (Control
 * call.) */
qsv_status qsv_sync(qsv_state s);

/* Thread-local message of the last failing call ("" if none).  (Control
 * call.) */
const char* qsv_last_error(void);

/* Library version string.  (Control call.) */
const char* qsv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QSV_H */
