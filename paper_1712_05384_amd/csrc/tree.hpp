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
// same launch (one launch per level of the elimination tree).
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "qgm.h"

namespace qgm {

struct Plan;

constexpr int kTreeMaxRank = 28;    // rank of a bucket result
constexpr int kTreeMaxIn = 8;       // earlier results multiplied in one bucket
constexpr int kTreeMaxSig = 12;     // output bits read by one bucket's factors
constexpr int kTreeMaxGBits = 10;   // variables of a bucket's factor table besides v
constexpr int kTreeMaxGIndex = 20;  // gb + kg + sb
constexpr int kTreeMaxSum = 3;      // variables summed by one (merged) bucket: beyond 3 the
                                    // serial load batches of a wave outweigh the saved launch
constexpr int kTreeOcBits = 3;      // a wave unit covers up to 2^kTreeOcBits consecutive result rows
constexpr int64_t kTreeMaxTasks = int64_t(1) << 22;   // (bucket, row chunk) records of a plan

// Sources of a variable inside a factor of the tree plan.
enum : int32_t {
    TS_ZERO = 0,   // fixed to 0 (input delta)
    TS_G = 1,      // bit `bit` of the factor-table index c = (g << kg) | w (w: the summed variables)
    TS_SIG = 2     // output bit: bit `bit` of sigma (bucket factors) or qubit `bit` of x (phase)
};

// Factor types of the tree plan.
enum : int32_t {
    TF_MAT = 0,     // non-diagonal 2x2 gate: M[new][old], (src0, bit0) = new, (src1, bit1) = old
    TF_DIAG = 1,    // diagonal gate: M[c][c] on (src0, bit0)
    TF_CZ = 2,      // (-1)^(a b)
    TF_DELTA0 = 3   // phase only: the amplitude is 0 unless (src0, bit0) is 0
};

struct TFactor {
    int32_t type, mat;
    int32_t src0, bit0;
    int32_t src1, bit1;
};

struct TreeStep {
    std::vector<int> vars;              // variables summed out (a merged chain sums up to kTreeMaxSum)
    int kg = 1;                         // summed-variable bits of the table index: the level's most
    int level = 0;                      // level in the elimination tree (0: no earlier result)
    int out_tensor = -1;                // id of the result
    std::vector<int> out_axes;          // result axes (variables), elimination position ascending
    std::vector<int> in_tensors;        // earlier results multiplied in
    std::vector<int> gvars;             // factor-table variables besides the summed ones (index bits kg..)
    std::vector<int> sig_q;             // sigma bit i = output bit of qubit sig_q[i]
    std::vector<TFactor> factors;       // gate factors of the bucket (none: G = 1)
    int64_t g_off = 0;                  // complex offset in the factor-table area
    int sig_row = -1;                   // row of the per-call sigma table (-1: reads no output bit)
    int64_t task_off = 0;               // first wave task (row chunk) of this bucket
    int oc_bits() const { return std::min(int(out_axes.size()), kTreeOcBits); }
    int64_t n_tasks() const { return int64_t(1) << (int(out_axes.size()) - oc_bits()); }
    int gb() const { return int(gvars.size()); }
    int sb() const { return int(sig_q.size()); }
    int64_t g_entries() const { return int64_t(1) << (gb() + kg + sb()); }
};

struct TreePlan {
    std::vector<int> order;                      // elimination order (variable ids)
    std::vector<TreeStep> steps;                 // in elimination order
    std::vector<std::vector<int>> tensor_axes;   // axes of every result
    std::vector<int> tensor_made, tensor_used;   // level that writes / last reads each result
    std::vector<int64_t> tensor_row;             // arena row of each result
    std::vector<int> finals;                     // rank-0 results multiplied into the amplitude
    std::vector<TFactor> phase;                  // factors without free variables
    std::vector<std::vector<int>> levels;        // step ids per level
    std::vector<int64_t> level_task_off;         // wave tasks of level L: [off[L], off[L + 1])
    std::vector<int> level_max_in;               // most inputs of a bucket in level L
    int64_t n_tasks = 0;
    int n_sig_rows = 0;                          // sigma rows, the last one all zero (buckets without output bits)
    int64_t ones_row = 0;                        // arena row of constant 1 (inputs a bucket does not have)
    std::vector<int> level_k;                    // most summed variables of a bucket in level L
    int64_t arena_rows = 0;
    int64_t g_total = 0;
    int max_rank = 0;
    int max_in = 0;
    int n_free = 0;
    int n_candidates = 0;                        // orders tried
    double bytes_per_b = 0;                      // algorithmic HBM bytes per bitstring
    double flops_per_b = 0;
};

// Builds the bucket plan from the variables and gate records in `p`
// (ordering 1; no open qubits, no slicing).
qgm_status build_tree_plan(const Plan& p, TreePlan& t, std::string* err);

// Per-bucket algorithmic bytes per batch entry: inputs read once, result written once.
double tree_step_bytes(const TreePlan& t, const TreeStep& st);

}  // namespace qgm
