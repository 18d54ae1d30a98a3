/*
 * qgm.h -- C ABI of the MI355X amplitude engine for random grid circuits
 * viewed as complex undirected graphical models (arXiv:1712.05384).
 *
 * The library computes output amplitudes <x|U|0...0> of a circuit built from
 * single-qubit gates and CZ gates (Sec. III.A, Eq. (fpath)), for a batch of
 * output bitstrings x, by variable elimination on the graphical model of
 * Sec. III.B (Eq. (psi_x)): one Boolean variable per qubit per non-diagonal
 * gate, complex factors per gate, eliminated either in the vertical (worldline
 * by worldline) order of Sec. IV.A (ordering 0) or by bucket elimination
 * (App. A) along greedy treewidth orders (Sec. IV.B; ordering 1, the faster).
 * Leaving some output deltas out of Eq. (psi_x) gives sets of amplitudes at
 * once (the "open" qubits below, Sec. III.A); fixing some variables and
 * summing over their values ("slicing", the space-time tradeoff of Sec. V)
 * bounds the memory of the largest intermediate results (Sec. II).
 *
 * Conventions (all entry points)
 *  - Qubit (r, c) of a rows x cols lattice has index q = r*cols + c; n <= 64.
 *  - A bitstring is a uint64_t whose bit q is the output bit of qubit q.  Bits
 *    at positions >= n and bits on open qubits are ignored.
 *  - Entry points that implement a passage of the paper name it; the
 *    multi-circuit entry is qgm_graph_create (there is no separate
 *    plan-for-many-circuits call: each circuit gets its own plan, order and
 *    slicing from qgm_plan, and one graph runs them together).
 *  - Complex numbers are interleaved (re, im): complex64 = 2 floats,
 *    complex128 = 2 doubles.  A 2x2 gate matrix is stored row-major with
 *    element [row][col] = <row|U|col> (row = the state after the gate).
 *  - Every entry point returns a qgm_status; on failure qgm_last_error()
 *    returns a message (thread-local, valid until the next call on the same
 *    thread).  Arguments are validated before anything is launched.
 *  - Device pointers are HIP device pointers on the current device; `stream`
 *    is a hipStream_t passed as void* (NULL = the default stream).  All device
 *    work is enqueued asynchronously on that stream; HIP errors raised by the
 *    kernels surface as QGM_E_HIP at the next call or at qgm_sync_check().
 *  - The caller owns every buffer passed in; the library never frees them and
 *    never allocates device memory on the amplitude path except the one-time
 *    per-device upload of a plan's constant tables (see qgm_amplitudes).
 */
#ifndef QGM_API_H_
#define QGM_API_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QGM_OK = 0,
    QGM_E_INVALID = -1,      /* malformed circuit, options or arguments */
    QGM_E_UNSUPPORTED = -2,  /* valid input outside what the kernels handle */
    QGM_E_OOM = -3,          /* plan cannot fit the memory budget / workspace too small */
    QGM_E_HIP = -4,          /* a HIP runtime call failed */
    QGM_E_INTERNAL = -5
} qgm_status;

/* Gate kinds (Sec. II: H, X^1/2, Y^1/2, T, CZ; plus value-slot gates).
 *  QGM_H  = (1/sqrt2)[[1,1],[1,-1]]              (table of App. D)
 *  QGM_T  = diag(1, e^{i pi/4})                   (Sec. II)
 *  QGM_XH = RX(pi/2) = (1/sqrt2)[[1,-i],[-i,1]]   (Sec. II; phases of App. F Eq. (phX))
 *  QGM_YH = RY(pi/2) = (1/sqrt2)[[1,-1],[1,1]]    (Sec. II; phases of App. F Eq. (phX))
 *  QGM_CZ = diag(1,1,1,-1) on (q0, q1)            (Sec. III.B)
 *  QGM_U  = general 2x2 read from gate_vals[slot]; non-diagonal, so it opens a
 *           new worldline variable (Sec. III.A)
 *  QGM_UD = diagonal 2x2 read from the diagonal of gate_vals[slot]; like T it
 *           adds no variable (Sec. III.A)
 * Inverses and Pauli operators (for expectation values <0|U^dag O U|0>, which
 * the same graphical model computes, Sec. III.B; see qgm_expectation_circuit):
 *  QGM_TDG = diag(1, e^{-i pi/4}), QGM_XHDG = RX(-pi/2) = (1/sqrt2)[[1,i],[i,1]],
 *  QGM_YHDG = RY(-pi/2) = (1/sqrt2)[[1,1],[-1,1]], QGM_X = [[0,1],[1,0]],
 *  QGM_Y = [[0,-i],[i,0]], QGM_Z = diag(1,-1) (TDG and Z diagonal) */
typedef enum { QGM_H = 0, QGM_T = 1, QGM_XH = 2, QGM_YH = 3, QGM_CZ = 4, QGM_U = 5, QGM_UD = 6, QGM_TDG = 7,
               QGM_XHDG = 8, QGM_YHDG = 9, QGM_X = 10, QGM_Y = 11, QGM_Z = 12, QGM_U2 = 13 } qgm_kind;
/* QGM_U2 = general two-qubit gate on (q0, q1), non-diagonal: it opens a new
 *           variable on both qubits and its factor couples the four (the
 *           4-clique of Sec. III.B).  Its 4x4 matrix M[r][c], r = 2 a0 + a1 the
 *           values after the gate and c = 2 c0 + c1 before (a0, c0 on q0), is
 *           read from four value slots: M[r][c] = gate_vals[slot + r][c >> 1][c & 1].
 *           Bucket elimination (ordering 1) only; no qgm_backward. */

typedef struct {
    int32_t kind;    /* qgm_kind */
    int32_t cycle;   /* clock cycle >= 0; gates apply in (cycle, list index) order */
    int32_t q0;      /* qubit */
    int32_t q1;      /* second qubit of a CZ, -1 otherwise */
    int32_t slot;    /* index into gate_vals for QGM_U / QGM_UD, -1 otherwise */
} qgm_gate;

typedef struct {
    int32_t rows, cols;      /* lattice; n = rows*cols qubits, 1 <= n <= 64 */
    int32_t n_gates;
    int32_t n_slots;         /* number of 2x2 values gate_vals must hold */
    const qgm_gate* gates;   /* host array [n_gates]; a qubit is used at most once per cycle */
} qgm_circuit;

typedef struct {
    int32_t ordering;          /* 0 = vertical order of Sec. IV.A (qubits along the shorter side first);
                                  1 = bucket elimination (App. A) along a greedy treewidth order (min-degree /
                                      min-fill with randomised tie breaks, the cheapest of several; Sec. IV.B);
                                      open qubits (their last variables are never summed: one more bucket
                                      multiplies every result left on them), slicing, qgm_backward without open
                                      qubits or slicing */
    int32_t precision;         /* qgm_precision: QGM_PREC_C64 = complex64 values, FP32 arithmetic in every
                                  step; QGM_PREC_BF16X3 = ordering 0 only: every worldline step that the
                                  matrix-core kernel supports (K and N of 2^3..2^5) runs in BF16x3 (as
                                  kernel_policy 4; kernel_policy must then be 0 or 4), the others in FP32;
                                  QGM_E_UNSUPPORTED for ordering 1 or when no step supports it */
    int32_t kernel_policy;     /* 0 = auto (the vector-ALU kernel, one row per thread); 1 = the same;
                                  2 = FP32 matrix-core kernel for every step it supports (K and N of
                                      2^3..2^5), the vector-ALU kernel elsewhere;
                                  3 = vector-ALU kernel with two rows per thread on dense steps
                                      (|K|+|N| >= 8 bits);
                                  4 = as 2 with BF16x3 split-precision matrix cores (bf16 hi+lo
                                      operands, three products, FP32 accumulation) */
    int32_t min_sliced_vars;   /* slice at least this many variables (Sec. V outlook: space-time tradeoffs):
                                  each sliced variable is fixed to 0 and to 1 in turn and the amplitudes of
                                  the slices are summed in FP64.  Ordering 0: at most 12, slices run as
                                  batch columns.  Ordering 1: at most 24 and n + slices <= 64 (slice j is
                                  carried by bit n + j of a batch column's 64-bit word); the slices run in
                                  chunks of batch columns (see mem_budget) */
    int32_t out_c128;          /* 1: amplitudes are written as complex128, 0: complex64 */
    int32_t max_rank;          /* 0 = no limit; else slice until every frontier tensor (ordering 0) or
                                  bucket result (ordering 1) has rank <= max_rank; QGM_E_OOM if slicing
                                  cannot reach it */
    int32_t checkpoint_every;  /* qgm_backward keeps every c-th frontier (0 = ceil(sqrt(steps))) */
    int32_t no_chain_merge;    /* ordering 1 only: 1 = one variable per bucket step; 0 = a bucket whose only
                                  input is an earlier bucket's result absorbs that bucket when the merged
                                  index space grows by at most one bit (up to 3 summed variables) */
    int32_t tree_exec;         /* ordering 1 only: how qgm_amplitudes runs the buckets.
                                  0 = auto: the LDS-resident launch (3) when the plan fits it, else one
                                      launch per level (1);
                                  1 = one launch per level of the elimination tree (the last small levels
                                      and the amplitude product in one more launch), results in a
                                      batch-minor workspace arena in HBM;
                                  2 = one persistent launch for all levels and the amplitude product: each
                                      64-bitstring group runs on one accelerator complex and each bucket task
                                      starts when the tasks making its inputs have signalled completion; the
                                      workspace then keeps every result at its own rows.  Calls in this mode
                                      must not run concurrently on one device (each needs the whole GPU at
                                      once); a launch that cannot proceed gives up after a bounded wait,
                                      writes NaN amplitudes and records the failure in the plan
                                      (qgm_plan_check returns QGM_E_INTERNAL);
                                  3 = one launch of one work-group per bitstring that keeps every result of
                                      the elimination and the factor-table entries at the bitstring's output
                                      bits in LDS (at most 7936 complex64 values, i.e. 62 KiB, per
                                      work-group): no workspace unless the circuit reads gate values (then
                                      the factor tables of the call).  Needs no open qubits, buckets of at
                                      most 4 inputs and 3 summed variables; qgm_plan returns
                                      QGM_E_UNSUPPORTED when the plan does not fit (qgm_plan_info gives the
                                      reason as lds_why). */
    int32_t no_tile;           /* ordering 1 only: 1 = every bucket uses the general wave unit; 0 = a
                                  two-input bucket summing two or more variables whose result has two bits
                                  carried by one input only and one carried by the other only (neither in
                                  its factor table) computes 8 result rows per wave unit from 4 + 2 input
                                  rows per summed value */
    int32_t order_finalists;   /* ordering 1 only: the candidate elimination orders (greedy min-degree and
                                  min-fill with randomised tie breaks, ranked by their symbolic traffic
                                  before chains are merged) of which this many first ones are built in full
                                  and scored by the bytes the kernels issue per bitstring plus 8 KiB per
                                  launch; the lowest score is kept.  0 = 64 (2 beyond 600 free variables);
                                  1 = the first order as ranked; at most 64 */
    int32_t order_restarts;    /* ordering 1 only: randomised tie-break restarts of each greedy criterion
                                  (candidates = 2 x (restarts + 1)).  0 = 64 up to 600 free variables, 4 up
                                  to 1500, 1 beyond; at most 1024.  More restarts find plans with fewer
                                  bytes on larger circuits at a plan time of up to about 0.2 s at 64 */
    int32_t order_pick;        /* ordering 1 only: keep the finalist of this rank by score (0 = the lowest
                                  score); for callers that time several finalists on their own batch.
                                  QGM_E_INVALID if fewer finalists build; at most 63 */
    int32_t persist_spin;      /* tree_exec 2 only: polls after which a wait of the persistent launch gives up
                                  (0 = 2^20).  A launch that gives up writes NaN for the amplitudes it could
                                  not finish and records the failure in the plan, which qgm_plan_check reports;
                                  a small value forces that path (for tests of the error report) */
    uint64_t mem_budget;       /* 0 = no limit; else a bound on qgm_workspace_bytes(plan, 64), the workspace
                                  of a call over 64 bitstrings (a call over B needs about B / 64 times
                                  that).  Ordering 1 slices further until one slice at a time fits, then
                                  runs as many slices per chunk as fit (Sec. II memory wall, Sec. V
                                  space-time tradeoff); QGM_E_OOM when 24 sliced variables do not fit.
                                  Ordering 0 runs its slices as batch columns, which does not shrink the
                                  frontier, so there the budget is a check: QGM_E_OOM when it is exceeded */
    uint64_t checkpoint_budget;/* 0 = no limit; else a bound on the forward frames qgm_backward keeps for 64
                                  bitstrings.  Ordering 0 with checkpoint_every = 0: the interval c with the
                                  least recomputation whose (steps - 1) / c checkpoints plus c - 1 segment
                                  frames fit, at most ceil(sqrt(steps)); QGM_E_OOM when even that does not
                                  fit.  Ordering 1 keeps every result for its adjoint: QGM_E_OOM when those
                                  exceed the budget */
    int32_t no_compose;        /* ordering 1 only: 1 = only buckets without inputs become leaf tables; 0 = a
                                  bucket whose inputs are all leaf tables, whose result bits plus the output
                                  bits of its subtree are at most 18 (those output bits at most 10), becomes
                                  a leaf table too: its result depends on the bitstring only through those
                                  bits, so it is built once with the plan for all their values (Sec. V:
                                  reuse across bitstrings) and read at each bitstring's bits.  Circuits
                                  with gate values have no leaf tables */
    int32_t reserved0;         /* 0 */
} qgm_plan_opts;

typedef enum { QGM_PREC_C64 = 0, QGM_PREC_BF16X3 = 1 } qgm_precision;

typedef struct qgm_plan_s qgm_plan_t;

/* Fills *opts with the defaults (all zero: vertical order, complex64 out). */
void qgm_default_opts(qgm_plan_opts* opts);

/* Builds a contraction plan on the host (no device call): the graphical model
 * of Sec. III.B (a variable per qubit at the start and after every
 * non-diagonal gate; one factor per gate, CZ as the pairwise factor
 * (-1)^(a b)), the elimination order (the vertical order of Sec. IV.A, or the
 * cheapest of several greedy min-degree / min-fill orders, Sec. IV.B, run as
 * the bucket elimination of App. A), the sliced variables (Sec. V) and the
 * device program of every step.  The plan depends on which gates are diagonal
 * and on the open qubits, not on gate values or bitstrings, so one plan serves
 * any batch of bitstrings and any gate_vals.
 *  open_qubits: host array [n_open] of distinct qubits whose output bit is left
 *               free (the delta of Eq. (psi_x) omitted); output index bit i
 *               corresponds to open_qubits[i].  May be NULL when n_open = 0.
 *  opts:        may be NULL for the defaults.
 *  *out:        receives the plan; free it with qgm_plan_destroy.
 * Errors: QGM_E_INVALID for a malformed circuit (qubit out of range, CZ with
 * q0 == q1, a qubit used twice in one cycle, unknown kind, slot out of range),
 * duplicate or out-of-range open qubits, out-of-range options;
 * QGM_E_UNSUPPORTED when a step would exceed the kernels' limits (ordering 1
 * first slices to meet them); QGM_E_OOM when max_rank, mem_budget or
 * checkpoint_budget cannot be met. */
qgm_status qgm_plan(const qgm_circuit* circuit, const int32_t* open_qubits, int32_t n_open,
                    const qgm_plan_opts* opts, qgm_plan_t** out);

/* Writes a JSON description of the plan into json[0..cap) (NUL-terminated) and
 * the size it needs (including the NUL) into *needed (may be NULL).  detail 0:
 * summary and per-step sizes (rank, sliced variables, bytes and flops per
 * amplitude); detail 1: also the axis layouts and the factor programs of every
 * step; detail 2 (ordering 1): also the LDS-resident program (its jobs and
 * table copies).  Returns QGM_E_INVALID if cap is too small (json may
 * be NULL to query the size). */
qgm_status qgm_plan_info(const qgm_plan_t* plan, int32_t detail, char* json, size_t cap, size_t* needed);

/* Device workspace (bytes) that qgm_amplitudes needs for a batch of B
 * bitstrings: the live intermediate results of the elimination, whose size is
 * the memory wall of Sec. II (ordering 0: two frontier tensors and the variant
 * ids; ordering 1: the arena of bucket results, none for the LDS-resident
 * launch), the factor tables of the call when the circuit reads gate values,
 * and for a sliced bucket plan the words and amplitudes of one chunk's batch
 * columns and the FP64 slice sums.  For ordering 1 the arena's rows hold the
 * chunk's columns (B << slice_chunk_bits) rounded up to a power of two (at
 * least 64), so the kernels scale rows by a shift: a batch just above a power
 * of two takes up to twice the memory of one just below it (the work covers
 * only the batch's own 64-column groups). */
qgm_status qgm_workspace_bytes(const qgm_plan_t* plan, int64_t B, uint64_t* bytes);

/* Computes out[b][o] = <x_b with the open bits set to o | U | 0...0> for
 * b < B and o < 2^n_open (the path sum of Eq. (fpath) written as the
 * graphical model of Eq. (psi_x), with the deltas of the open qubits left out:
 * the sets of amplitudes of Sec. III.A), by the plan's elimination steps on
 * the device.
 *  gate_vals: device complex64 [n_slots][2][2]; may be NULL when n_slots = 0.
 *  bits:      device uint64 [B].
 *  out:       device complex64 or complex128 (opts.out_c128) [B][2^n_open].
 *  workspace: device buffer of at least qgm_workspace_bytes(plan, B) bytes,
 *             256-byte aligned; its contents are scratch.  May be NULL when
 *             that size is 0 (the LDS-resident launch of a circuit that reads
 *             no gate values).
 * The first call of a plan on a device uploads the plan's constant tables
 * (a synchronous hipMalloc + hipMemcpy, kept until qgm_plan_destroy).
 * Sums over sliced variables are done in FP64.  Calls that share a workspace
 * must be ordered on one stream. */
qgm_status qgm_amplitudes(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B,
                          void* out, void* workspace, uint64_t ws_bytes, void* stream);

/* qgm_amplitudes without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc.  It computes exactly what
 * qgm_amplitudes computes, with the same kernels, using as its workspace a
 * file-scope device array of the library (64 MiB; one copy per device, held
 * until the process ends).  It calls no hipMalloc, hipFree or other allocating
 * routine, so the plan's constant tables must already be on the current device:
 * run qgm_amplitudes (or qgm_graph_create) with the plan once on the device
 * first, else QGM_E_INVALID.  QGM_E_OOM when qgm_workspace_bytes(plan, B)
 * exceeds 64 MiB; QGM_E_INVALID when per-phase timing is on.  Every call on a
 * device shares that device's array: calls that overlap on one device (on
 * different streams, or from several threads) race and must be ordered by the
 * caller; the array keeps the last call's contents, which no call relies on.
 * Other arguments, layouts and errors as qgm_amplitudes. */
qgm_status qgm_amplitudes_static(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B,
                                 void* out, void* stream);

/* Device workspace (bytes) that qgm_backward needs for a batch of B bitstrings
 * (for ordering 1 sized by the same power-of-two row pitch): the forward
 * frames it keeps (checkpoints, or every bucket result), their adjoints and
 * the factor-adjoint partial sums. */
qgm_status qgm_backward_workspace_bytes(const qgm_plan_t* plan, int64_t B, uint64_t* bytes);

/* Gradient of a real loss with respect to the gate values (the gate
 * environments), by the adjoint of the elimination steps.  Runs the forward
 * pass itself, keeping every c-th frontier (opts.checkpoint_every, default
 * ceil(sqrt(steps))) and recomputing each segment during the reverse sweep.
 *  grad_amps:  device complex64 [B][2^n_open], dL/dRe A + i dL/dIm A for each
 *              amplitude (the torch convention).
 *  amps_out:   device [B][2^n_open] (complex64 or complex128 per opts.out_c128),
 *              receives the amplitudes of the forward pass; may be NULL.
 *  gate_grads: device complex64 [n_slots][2][2], receives
 *              dL/dRe U + i dL/dIm U summed over the gates that read each slot
 *              (for QGM_UD slots only the diagonal is written non-zero).  May be
 *              NULL when n_slots = 0.
 *  workspace:  at least qgm_backward_workspace_bytes(plan, B) bytes, 256-byte aligned.
 * With L = sum_x log |A_x|^2 (grad_amps = 2 / conj(A)) this is the gradient of
 * m times the cross-entropy estimator of App. B, Eq. (cee).  Ordering 1 keeps
 * every bucket result instead of checkpoints and supports no open qubits, no
 * slicing and no QGM_U2 gates (QGM_E_UNSUPPORTED). */
qgm_status qgm_backward(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B,
                        const void* grad_amps, void* amps_out, void* gate_grads, void* workspace, uint64_t ws_bytes,
                        void* stream);

/* Chooses the kernel of every elimination step by measurement on the current
 * device (the cGEMM-shape autotuner): for each step it times the vector-ALU
 * kernel with one and with two rows per thread, the FP32 matrix-core kernel
 * and, if allow_bf16x3, the BF16x3 matrix-core kernel (each where the step's
 * shape allows it) on the given batch, and keeps the fastest.  Timings are
 * cached in a text file keyed by (arch, K, V, N, sigma bits, rank, batch,
 * kernel): cache_path, or $QGM_TUNE_CACHE when cache_path is NULL, or no cache.
 * Runs one qgm_amplitudes call first (out may be NULL only here: the call's
 * output is not written), uses `workspace` as scratch and synchronises
 * `stream`.  The choice is stored in the plan (see qgm_plan_info). */
qgm_status qgm_autotune(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B, void* workspace,
                        uint64_t ws_bytes, void* stream, int32_t allow_bf16x3, const char* cache_path);

/* Per-phase timing of qgm_amplitudes (hipEvents recorded on the call's
 * stream; instrumentation for the benchmark, off by default).  enable = 1
 * starts recording and clears the totals; 0 stops.  While enabled each call
 * records 5 events: before the boundary kernel, after it, after the G
 * builder, after the last elimination step, after the output stage. */
qgm_status qgm_plan_set_timing(qgm_plan_t* plan, int32_t enable);

/* Synchronises the recorded events and returns the accumulated times (ms) of
 * the phases [0] boundary, [1] G build, [2] elimination steps, [3] output
 * stage into ms[4], and the number of timed calls into *n_calls.  The step
 * phase holds n_steps kernel launches per call. */
qgm_status qgm_plan_timings(qgm_plan_t* plan, double* ms, int64_t* n_calls);

/* ---- Multi-circuit batches: one HIP graph for several plans ---------------
 * qgm_graph_create records the complete qgm_amplitudes launch sequence of
 * n_circ independent (plan, batch) pairs into one HIP graph, one branch per
 * circuit (the branches fork from and join back to a common node, so the
 * device may run small circuits beside large ones), and instantiates it.
 * The buffers are fixed at creation: every later qgm_graph_launch recomputes
 * out[i] from the current contents of bits[i] and gate_vals[i].  All arrays
 * are host arrays of length n_circ; the pointers they hold follow the rules of
 * qgm_amplitudes (workspaces must not be shared between circuits).  Creation
 * uploads missing plan tables first and captures on private streams; it does
 * not launch anything.  When a branch runs as one persistent launch (tree_exec
 * 2), which needs the whole GPU at once, every branch runs after the previous
 * one; otherwise the branches are concurrent.  A graph
 * must not outlive its plans or buffers. */
typedef struct qgm_graph_s qgm_graph_t;
qgm_status qgm_graph_create(int32_t n_circ, qgm_plan_t* const* plans, const void* const* gate_vals,
                            const uint64_t* const* bits, const int64_t* B, void* const* out,
                            void* const* workspace, const uint64_t* ws_bytes, qgm_graph_t** graph);
/* Enqueues one replay of the graph on `stream`. */
qgm_status qgm_graph_launch(qgm_graph_t* graph, void* stream);
/* Destroys the graph (NULL is ignored). */
void qgm_graph_destroy(qgm_graph_t* graph);

/* ---- Expectation values of Pauli strings ------------------------------------
 * qgm_expectation_circuit (host only): writes to gates[0, *n_gates) a circuit
 * whose amplitude at the all-zero bitstring is <0|U^dag O U|0> for the Pauli
 * string O = prod_i paulis[i] on qubits[i] (kinds QGM_X, QGM_Y, QGM_Z, distinct
 * qubits; Sec. III.B: the operator enters the same graphical model as factors).
 * It is U restricted to the backward light cone of O's qubits (gates outside
 * it cancel against their inverses), then O at cycle d (one past U's last
 * cycle), then the inverses of the kept gates in reverse order at cycle 2d - t;
 * same lattice as circuit.  Plan it with qgm_plan and evaluate it with
 * qgm_amplitudes at bitstring 0 (real up to rounding for Hermitian O).  U must
 * use fixed gate kinds (QGM_E_UNSUPPORTED for value slots).  If cap is below
 * the gate count, *n_gates receives the count and QGM_E_OOM is returned (call
 * with cap = 0 to size the array).  Other errors: QGM_E_INVALID as qgm_plan's
 * circuit checks, plus bad operator qubits or kinds. */
qgm_status qgm_expectation_circuit(const qgm_circuit* circuit, int32_t n_ops, const int32_t* qubits,
                                   const int32_t* paulis, qgm_gate* gates, int32_t cap, int32_t* n_gates);

/* ---- Cross-entropy benchmarking and sampling on top of the amplitudes ------
 * Both take a device array of B amplitudes (complex64 when c128 = 0, else
 * complex128), e.g. the out array of qgm_amplitudes, and a caller-allocated,
 * 256-byte aligned device workspace of at least qgm_xeb_workspace_bytes(B)
 * bytes; they only enqueue kernels on `stream` (NULL: the null stream).
 *
 * qgm_xeb (App. B): with p_j = |amp_j|^2 in FP64, writes 8 doubles to the
 * device array out: [0] sum_j log p_j, [1] sum_j p_j, [2] sum_j p_j log p_j (the
 * three over the nonzero p_j), [3] the number of zero p_j, [4] the cross entropy
 * of the batch taken as a sample of a device's output, -mean log p_j over the
 * nonzero p_j (Eq. (cee)), [5] the fidelity estimate of Eq. (ae),
 * (H_0 - [4]) / (H_0 - H(p_U)) with the Porter-Thomas values H_0 = n log 2 +
 * gamma and H(p_U) = n log 2 - 1 + gamma (gamma: Euler's constant), [6] the
 * entropy of the output distribution estimated from the batch taken as a
 * uniformly chosen set, -(2^n / B) sum_j p_j log p_j (App. C), [7] (2^n / B)
 * sum_j p_j (1 + O(1/sqrt B) for such a set).  Sums run in a fixed order: the
 * same input gives the same bits.  Errors: QGM_E_INVALID for B < 1, n_qubits
 * outside 1..64, a NULL pointer or an unaligned workspace; QGM_E_OOM when
 * ws_bytes is too small.
 *
 * qgm_sample_set (App. C): draws m indices j of the batch, each with
 * probability p_j / sum_k p_k: draw i uses the caller's uniform u[i] in [0, 1)
 * (device doubles; the random numbers are the caller's) and writes to idx[i]
 * (device int64) the first j whose FP64 inclusive cumulative sum of p exceeds
 * u[i] times the total (B - 1 if none).  Errors as for qgm_xeb (m < 0 is
 * QGM_E_INVALID; m = 0 only scans). */
/* qgm_prob_sums (Sec. III.A, sets of amplitudes): for each of the B
 * bitstrings of an amplitude array laid out as qgm_amplitudes writes it,
 * amps[b][o] for o < 2^n_open (complex64 when c128 = 0, else complex128),
 * writes out[b] = sum_o |amps[b][o]|^2 computed in FP64, summed in a fixed
 * order (the same input gives the same bits).  It is the normalisation check
 * of a set: the sum is at most 1 (the probability that the fixed qubits read
 * x_b), and exactly 1 with every qubit open.  out: device doubles [B].  No
 * workspace; one launch on `stream`.  Errors: QGM_E_INVALID for B < 0, n_open
 * outside 0..40 or a NULL pointer (B = 0 does nothing); QGM_E_UNSUPPORTED for
 * B >= 2^31. */
qgm_status qgm_prob_sums(const void* amps, int32_t c128, int64_t B, int32_t n_open, double* out, void* stream);

qgm_status qgm_xeb_workspace_bytes(int64_t B, uint64_t* bytes);
qgm_status qgm_xeb(const void* amps, int32_t c128, int64_t B, int32_t n_qubits, double* out, void* workspace,
                   uint64_t ws_bytes, void* stream);
qgm_status qgm_sample_set(const void* amps, int32_t c128, int64_t B, const double* u, int64_t m, int64_t* idx,
                          void* workspace, uint64_t ws_bytes, void* stream);

/* Synchronises `stream`, then reports whether a persistent launch of this
 * plan (tree_exec 2) on the current device gave up since the last check: its
 * bounded wait for another wave ran out (the GPU was shared, or the grid could
 * not be resident at once) and it wrote NaN for the amplitudes it could not
 * finish.  The record is cleared by the check.  Returns QGM_E_HIP for a pending
 * HIP error, QGM_E_INTERNAL for a launch that gave up, QGM_E_INVALID for a
 * NULL plan, else QGM_OK (also for plans never run on this device).  Call it
 * after qgm_amplitudes or qgm_graph_launch when the plan runs persistently. */
qgm_status qgm_plan_check(qgm_plan_t* plan, void* stream);

/* Destroys a plan and frees its device tables (NULL is ignored). */
void qgm_plan_destroy(qgm_plan_t* plan);

/* Last error message of the calling thread ("" if none). */
const char* qgm_last_error(void);

/* Synchronises `stream` and reports any pending HIP error as QGM_E_HIP. */
qgm_status qgm_sync_check(void* stream);

#ifdef __cplusplus
}
#endif

#endif /* QGM_API_H_ */
