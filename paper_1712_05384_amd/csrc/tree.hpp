// Bucket-elimination plans with greedy treewidth orders (ordering 1).
//
// App. A processes one bucket per variable: the tensors whose earliest
// variable is v are multiplied with broadcasting and v is summed out; the
// result goes to the bucket of its earliest remaining variable.  Sec. IV.B
// reports that orders found by treewidth heuristics are far cheaper than the
// vertical order; here the order is the cheapest of several greedy
// min-degree / min-fill orders (randomised tie breaks) on the graph of the
// variables that the deltas of Eq. (psi_x) leave free.
//
// Every bucket becomes one device step over batch-minor tensors
//   R[o][b] = sum_w G_sigma(b)[g(o), w] * prod_t T_t[idx_t(o, w)][b],
// where the T_t are earlier results, G is the product of the bucket's own gate
// factors (Sec. III.B) with the output bits of bitstring b substituted, and
// o runs over the remaining variables of the bucket and w over the summed
// one (or the two or three of a merged chain, see merge_chains in the
// planner).  Factors without any free
// variable form a per-bitstring phase, evaluated in FP64 with the final
// product of the rank-0 results.  Buckets whose inputs are ready run in the
// same launch (one launch per level of the elimination tree); a bucket
// without inputs is folded into the factor table of the bucket that reads its
// result, and the last levels, whose buckets have few rows, run in one tail
// launch with the final product.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "qgm.h"

namespace qgm {

struct Plan;

constexpr int kTreeMaxRank = 28;    // rank of a bucket result
constexpr int kTreeMaxSliced = 24;  // sliced variables of a bucket plan (also n + sliced <= 64)
// Persistent launch (qgm_amplitudes, tree_exec): the flags area holds the
// abort word at [0], one word per (complex, rank) of its work-groups from
// kPersistSeen0, and the completion flags from kPersistFlags0.
constexpr int kPersistXcds = 8;                 // accelerator complexes (each with its own L2) of one MI355X
constexpr int kPersistMaxRanks = 256;           // work-groups per complex in one launch, at most
constexpr int kPersistSeen0 = 64;
constexpr int kPersistFlags0 = kPersistSeen0 + kPersistXcds * kPersistMaxRanks;
constexpr int kTreeLeafTableBits = 14;   // a leaf table has at most 2^14 entries (result bits + output bits)
// A bucket whose inputs are all leaf tables becomes a leaf table too (built once for every value of the output
// bits its subtree reads, instead of per bitstring) when its result bits plus those output bits are at most
// this many and the output bits at most kTreeComposeSig.
constexpr int kTreeComposeBits = 18;
constexpr int kTreeComposeSig = 10;
constexpr int kTreeMaxIn = 8;       // earlier results multiplied in one bucket
constexpr int kTreeMaxSig = 12;     // output bits read by one bucket's factors
constexpr int kTreeMaxGBits = 10;   // variables of a bucket's factor table besides v
constexpr int kTreeMaxGIndex = 20;  // gb + k + sb
constexpr int kTreeMaxSum = 3;      // variables summed by one (merged) bucket: beyond 3 the
                                    // serial load batches of a wave outweigh the saved launch
constexpr int kTreeTailTasks = 8;   // tail levels: at most this many wave tasks per bitstring group
constexpr int kTreeTailInputs = 4;  // ... and at most this many inputs per bucket
constexpr int kTreeTailMaxTasks = 32;    // task records of all tail levels (staged in LDS)
constexpr int kTreeTailLdsRows = 64;     // result rows made in the tail, kept in LDS (64 bitstrings each)
constexpr int kTreeTailMaxLevels = 16;
constexpr int kTreeTailMaxFinal = 64;    // rank-0 results the tail multiplies
constexpr int kTreeTailGEntries = 2048;  // factor-table entries of the tail's buckets (copied to LDS)
constexpr int kTreeOcBits = 3;      // a wave unit covers up to 2^kTreeOcBits consecutive result rows
constexpr int kTreeOrderFinalists = 64;        // candidate orders built in full and scored by issued bytes
constexpr int kTreeMaxFinalists = 64;          //   (plan option order_finalists: 0 = the default, at most this)
constexpr int kTreeOrderRestarts = 64;         // randomised restarts per greedy criterion up to 600 free variables
constexpr int kTreeMaxRestarts = 1024;         //   (plan option order_restarts: 0 = the default, at most this)
constexpr double kTreeLaunchBytes = 8192.0;    // ... a launch weighed as this many bytes per bitstring
constexpr int64_t kTreeMaxTasks = int64_t(1) << 22;   // (bucket, row chunk) records of a plan

// Result rows of one wave unit of a bucket with k summed variables in a
// launch whose buckets have at most nin inputs: the loads of those rows are
// issued together (about 64 at most).
constexpr int tree_unit_rows(int nin, int k) {
    const int lpb = (nin + 1) * ((1 << k) < 8 ? (1 << k) : 8);   // loads per row and batch of summed values
    return lpb <= 8 ? 8 : (lpb <= 16 ? 4 : (lpb <= 32 ? 2 : 1));
}
static_assert(tree_unit_rows(1, 1) == (1 << kTreeOcBits), "a unit never exceeds the rows reserved per result");

// Inputs of the bucket-kernel variant that runs a level whose buckets have at
// most n inputs (variants exist for 1, 2, 3, 4 and kTreeMaxIn inputs).
constexpr int launch_inputs(int n) { return n <= 1 ? 1 : (n <= 4 ? n : 8); }

// Sources of a variable inside a factor of the tree plan.
enum : int32_t {
    TS_ZERO = 0,   // fixed to 0 (input delta)
    TS_G = 1,      // bit `bit` of the factor-table index c = (g << kg) | w (w: the summed variables)
    TS_SIG = 2,    // output bit: bit `bit` of sigma (bucket factors) or qubit `bit` of x (phase)
    TS_INT = 3     // bit `bit` of a factor group's own summed value (an absorbed bucket's variables)
};

// Factor types of the tree plan.
enum : int32_t {
    TF_MAT = 0,     // non-diagonal 2x2 gate: M[new][old], (src0, bit0) = new, (src1, bit1) = old
    TF_DIAG = 1,    // diagonal gate: M[c][c] on (src0, bit0)
    TF_CZ = 2,      // (-1)^(a b)
    TF_DELTA0 = 3,  // phase only: the amplitude is 0 unless (src0, bit0) is 0
    TF_MAT4 = 4     // non-diagonal two-qubit gate: M[2 a0 + a1][2 c0 + c1], sources 0, 1 = a0, a1 (after),
                    //   2, 3 = c0, c1 (before); the value slots mat - kFixedMats .. + 3 hold the rows
};

struct TFactor {
    int32_t type, mat;
    int32_t src0, bit0;
    int32_t src1, bit1;
    int32_t src2, bit2;                 // TF_MAT4 only: the variables before the gate
    int32_t src3, bit3;
};

// A group of factors of a bucket's factor table: the table entry is the
// product over groups of (prod_f f) for k_int = 0, or of
// (sum over the 2^k_int values of the group's own variables of prod_f f) --
// a bucket without inputs whose result only one later bucket reads is folded
// into that bucket's table this way.
struct TGroup {
    int k_int = 0;
    std::vector<int> vars;              // the group's own summed variables (ids), k_int of them
    std::vector<TFactor> factors;
};

struct TreeStep {
    std::vector<int> vars;              // variables summed out (a merged chain sums up to kTreeMaxSum)
    int kg = 1;                         // summed-variable bits of the table index (= vars.size())
    int level = 0;                      // level in the elimination tree (0: no earlier result)
    int out_tensor = -1;                // id of the result
    std::vector<int> out_axes;          // result axes (variables); the first kTreeOcBits chosen for wave-unit
                                        //   reuse (unit_axis_order), the rest in elimination order
    std::vector<int> in_tensors;        // earlier results multiplied in
    std::vector<int> gvars;             // factor-table variables besides the summed ones (index bits kg..)
    std::vector<int> sig_q;             // sigma bit i = output bit of qubit sig_q[i]
    std::vector<TGroup> groups;         // factor groups: [0] the bucket's own gate factors, then absorbed buckets
    int n_factors() const {
        int n = 0;
        for (auto& g : groups) n += int(g.factors.size());
        return n;
    }
    int64_t g_off = 0;                  // complex offset in the factor-table area
    // a bucket without inputs in a plan without gate values: its result is a table over (result index,
    // its output bits) built once with the plan, read per lane by its reader; no level, rows or tasks
    bool table_leaf = false;
    int64_t leaf_off = 0;               // complex offset of that table (entry (o << sb) | sigma)
    int64_t task_off = 0;               // first wave task of this bucket
    int unit_rows = 1;                  // result rows per wave task (tree_unit_rows of its launch, or 8 for a
                                        //   tile)
    int tile = 0;                       // 1 (two inputs) or 2 (three): a tile unit, whose unit bits 0 and 1
                                        //   vary only input 0, bit 2 only input 1 and none input 2 or the
                                        //   factor table; its 8 rows from 4 + 2 (+ 1) input rows and 1
                                        //   table row per summed value (0: the general unit); 3 or 4: the
                                        //   32-row tile, unit bits 0, 1, 3 varying input 0 only and 2, 4
                                        //   input 1 only, from 8 + 4 (+ 1) rows and 1 entry per value
    bool composed = false;              // a leaf table built from its inputs, which are leaf tables; its
                                        //   sig_q lists its own output bits first, then its inputs' others
    int leaf_depth = 0;                 // leaf tables: 0 without inputs, else 1 + the deepest input's
    bool quad = false;                  // a two-input 32-row tile whose result bits 5 and 6 vary input 1
                                        //   only: tasks 4m .. 4m + 3 read the same rows of input 0 and of
                                        //   the factor table, and run as one work-group that loads those
                                        //   once into LDS (level_quad)
    int64_t n_tasks() const {
        const int64_t rows = int64_t(1) << out_axes.size();
        return rows <= unit_rows ? 1 : rows / unit_rows;
    }
    int gb() const { return int(gvars.size()); }
    int sb() const { return int(sig_q.size()); }
    int64_t g_entries() const { return int64_t(1) << (gb() + kg + sb()); }
};

// ---- LDS-resident execution (qgm_amplitudes, tree_exec 3) -------------------
// One work-group per bitstring runs every level of the plan with its results
// in LDS: the factor tables and leaf tables are first copied to LDS at the
// bitstring's output bits, then each level's jobs (64, 128 or 256 result rows
// of one bucket, 1, 2 or 4 per lane) read inputs and table entries from LDS, with a
// block barrier between levels, and thread 0 writes phase x the rank-0 results.
// In LDS every tensor keeps its variables in decreasing order of elimination
// (the last eliminated lowest) and a factor table is indexed (w << gb) | g, so
// the lowest result axes of a bucket are the lowest axes of each input and of
// its table: the lanes of a job read consecutive entries (or the same entry),
// never two entries of one LDS bank.
constexpr int kLdsMaxComplex = 7936;   // complex64 entries of LDS data per work-group (62 KiB)
constexpr int kLdsMaxIn = 4;           // inputs of a bucket the LDS jobs handle
constexpr int kLdsMaxStages = 256;     // tables copied to LDS (each with its own output bits)
constexpr int kLdsHeader = 4 * kLdsMaxStages + 16;   // LDS bytes before the data: each table's output bits,
                                                     //   the FP64 phase
constexpr int kLdsSmallThreads = 256, kLdsLargeThreads = 512;   // work-group sizes (4 or 8 waves)

// A factor-table or leaf-table slice: the table entries src + sigma of its
// LdsEntry records, sigma bit i = bit sig_q[i] of the bitstring.  Its n
// entries are entries [e0, e0 + n) (n a power of two); the staged copy of the
// table area holds, for every sigma, the slice contiguously:
// staged[zoff + sigma * n + i] = area[entries[e0 + i].src + sigma].
struct LdsStage {
    int32_t n_sig, n, zoff, e0;
    int32_t sig_q[kTreeMaxSig];
};
// lds[tables0 + e] = table area[src + sigma of stage `stage`]
struct LdsEntry {
    uint32_t src;
    uint32_t stage;
};
// Rows o0 + l of one bucket's result, l < 64 (fewer for a small result: lanes
// beyond `lanes` compute a copy of a valid row and store nothing), and with
// rl > 0 also rows o0 + 64 m + l for m < 2^rl.  Lane l computes
//   R[o0 + l] = sum_w T[off_T(l) + tw[w]] * prod_t I_t[off_t(l) + in_w[t][w]]
// with off_s(l) = base[s] + sum_{i < 6} (bit i of l) * str[s][i] for each input
// s < nin and the table s = kLdsMaxIn, and row o0 + 64 m + l the same with
// off_s(l) + (bit 0 of m) * strx[0][s] + (bit 1 of m) * strx[1][s] (the
// strides of result bits 6 and 7).  Offsets are LDS bytes (< 64 KiB).
struct LdsJob {
    int32_t nin, k, lanes, out_row;
    int32_t base[kLdsMaxIn + 1];
    int32_t tw[8];
    int32_t in_w[kLdsMaxIn][8];
    int32_t str[kLdsMaxIn + 1][6];
    int32_t rl;                          // log2 of the rows per lane (0, 1 or 2)
    int32_t strx[2][kLdsMaxIn + 1];
};
// The device form of a job: kLdsRecordHalves 16-bit fields, 16-byte aligned:
// [0] nin | k << 3 | (lanes - 1) << 5 | rl << 11, [1] out_row, [2..6] base,
// [8..15] tw, [16..47] in_w[t][w] at 16 + 8 t + w, then for each slot s the
// lane offsets by three-bit groups: [48 + 16 s + c] = base[s] + the strides of
// the set bits of c (lane bits 0-2), [56 + 16 s + c] = the strides of the set
// bits of c as lane bits 3-5, so off_s(l) is one entry of each; [128..132]
// strx[0][s], [136..140] strx[1][s].
constexpr int kLdsRecordHalves = 144;
// A job with at most this many loads per row issues them all before its first product; a larger one
// interleaves loads and products to bound its registers.
constexpr int kLdsBatchLoads = 12;
// A job of 2^rl rows per lane batches its loads when (nin + 1) 2^k <= kLdsBatchLoads (rl <= 1) or
// <= kLdsBatchLoads / 2 (rl = 2).  The largest rl a job may take: 2 when its four rows batch, 1 when one
// row has at most two batches of loads, else 0.
constexpr bool lds_batched(int nin, int k, int rl) {
    return (nin + 1) * (1 << k) <= (rl >= 2 ? kLdsBatchLoads / 2 : kLdsBatchLoads);
}
constexpr int lds_max_rl(int nin, int k) {
    return lds_batched(nin, k, 2) ? 2 : (nin + 1) * (1 << k) <= 2 * kLdsBatchLoads ? 1 : 0;
}
constexpr int kLdsRecordBytes = 2 * kLdsRecordHalves;
struct LdsProgram {
    bool ok = false;
    std::string why;                     // reason when not ok
    int32_t lds_size = 0;                // complex64 entries of LDS data (results, tables, job records)
    int32_t tables0 = 0;                 // first entry of the copied tables
    int32_t recs0 = -1;                  // first entry of the job records in LDS (-1: read from memory)
    int32_t threads = 0;                 // work-group size
    std::vector<LdsStage> stages;
    std::vector<int32_t> stage_bucket;   // bucket of each stage
    std::vector<LdsEntry> entries;
    std::vector<uint32_t> zent;          // per entry: its staged index zoff + i, and its stage << 24
    std::vector<uint32_t> gent;          // per entry: its table-area index src, and its stage << 24 (for a
                                         //   circuit with gate values, whose tables change per call)
    int64_t z_entries = 0;               // size of the staged copy
    std::vector<LdsJob> jobs;
    std::vector<int32_t> job_bucket;
    std::vector<uint16_t> recs;          // [job][kLdsRecordHalves]
    std::vector<int32_t> level_job_off;  // jobs of level L: [off[L], off[L + 1])
    std::vector<int32_t> finals;         // LDS byte offsets of the rank-0 results
    std::vector<int32_t> tensor_lds;     // LDS data entry of each result's row 0 (-1: none)
};

struct TreePlan {
    std::vector<int> order;                      // elimination order (variable ids)
    std::vector<TreeStep> steps;                 // in elimination order
    std::vector<std::vector<int>> tensor_axes;   // axes of every result
    std::vector<int> tensor_made, tensor_used;   // level that writes / last reads each result
    std::vector<int64_t> tensor_row;             // arena row of each result
    std::vector<int> finals;                     // rank-0 results multiplied into the amplitude
    // open qubits (sets of amplitudes): the result over their variables, the output bit of each of its
    // axes, and the output bits of open qubits without non-diagonal gates (amplitude 0 when set)
    int n_open = 0;
    int open_tensor = -1;
    int n_table_leaves = 0;
    std::vector<int> open_axis_bit;
    int zero_mask = 0;
    std::vector<TFactor> phase;                  // factors without free variables
    std::vector<std::vector<int>> levels;        // step ids per level
    std::vector<int64_t> level_task_off;         // wave tasks of level L: [off[L], off[L + 1])
    std::vector<int> level_max_in;               // most inputs of a bucket in level L
    std::vector<int64_t> level_quad;             // the first level_quad[L] tasks of level L are quad tiles
                                                 //   (a multiple of 4, bucket by bucket)
    std::vector<char> level_quad_arena;          // every quad bucket of level L reads two arena results
    int64_t n_tasks = 0;
    // adjoint (qgm_backward): every result at its own rows, and per level the
    // scratch rows of the expansion (H and one Q per input for each bucket)
    std::vector<int64_t> tensor_row_all;
    int64_t arena_rows_all = 0;
    std::vector<int64_t> scratch_row;            // per step, within its level's scratch
    int64_t scratch_rows = 0;                    // the largest level's scratch
    std::vector<int64_t> hsum_row;               // per step: its table rows of H summed within the class
    int64_t hsum_rows = 0;
    int64_t ones_g = 0;                          // factor-table entry holding the constant 1 that a wave reads
                                                 //   (lane stride 0) for inputs its bucket does not have
    int n_absorbed = 0;                          // buckets without inputs folded into a later bucket's table
    int first_level = 1;                         // first level with buckets (0 unless every level-0 bucket
                                                 //   was absorbed)
    int tail_start = 0;                          // levels [tail_start, n_levels) run in the tail kernel
    std::vector<int32_t> tail_lds_row;           // per result made in the tail: its first row in the tail
                                                 //   kernel's LDS (-1: an arena result)
    int tail_lds_rows = 0;
    int64_t tail_g0 = 0, tail_g_entries = 0;     // factor tables of the tail's buckets: one range
    int64_t phase_g = 0;                         // FP64 values of the factors without free variables
                                                 //   (double2 [n_phase][4] from this float2 entry)
    int64_t arena_rows = 0;
    int64_t g_total = 0;
    int max_rank = 0;
    int max_in = 0;
    int n_free = 0;
    int n_candidates = 0;                        // orders tried
    int n_built = 0;                             // ... of which built in full and scored
    double order_score = 0;                      // the kept plan's score (issued bytes + launches)
    double bytes_per_b = 0;                      // algorithmic HBM bytes per bitstring
    double flops_per_b = 0;
    LdsProgram lds;                              // the LDS-resident program (lds.ok when the plan fits)
    // slicing (Sec. V outlook): sliced variable j is fixed by bit n + j of a batch column's word; a call runs
    // the 2^sliced slices of every bitstring in chunks of 2^chunk_bits as batch columns (column
    // b * 2^chunk_bits + j) and sums them in FP64 in slice order
    std::vector<int> sliced;
    int chunk_bits = 0;
};

// Builds t.lds from a finished bucket plan (sets t.lds.ok = false with a reason
// when the plan does not fit: open qubits, more than kLdsMaxIn inputs, LDS size).
void build_lds_program(TreePlan& t);
// LDS bytes one bitstring's program moves, counting only the rows a job keeps:
// per result row 2^k (inputs + table) complex64 reads and one write, plus one
// write per factor-table entry copied in (0 when the program does not fit).
int64_t lds_bytes_per_amp(const LdsProgram& P);

// Builds the bucket plan from the variables and gate records in `p`
// (ordering 1) with the variables in `sliced` fixed: slice j's value is bit
// n + j of a batch column's word (n + sliced.size() <= 64).
qgm_status build_tree_plan(const Plan& p, const std::vector<int>& sliced, TreePlan& t, std::string* err);
// The next variable to slice: the one in the most of the largest bucket index
// spaces (summed and result variables) of `t` (or, when no order fits the
// kernels, of the min-fill order's buckets without the limits); -1 when none
// is left.
int tree_pick_slice_var(const Plan& p, const std::vector<int>& sliced, const TreePlan* t);

// Row accesses (loads and stores of 64 lanes x 8 bytes) of one wave unit of a bucket.
int64_t tree_unit_accesses(const TreePlan& t, const TreeStep& st);
// Bytes the bucket kernels issue per bitstring (cache-served repeats included).
double tree_issued_bytes_per_b(const TreePlan& t);
// Kernel launches of one call: one per level before the tail, and the tail.
int tree_launches(const TreePlan& t);          // levels before the tail, plus the tail (the order score)
int tree_kernel_launches(const TreePlan& t);   // the same, a level with quad tiles and other tasks counted twice

// Per-bucket algorithmic bytes per batch entry: inputs read once, result written once.
double tree_step_bytes(const TreePlan& t, const TreeStep& st);

}  // namespace qgm
