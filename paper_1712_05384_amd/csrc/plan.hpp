// Host-side contraction planner: circuit -> graphical model -> elimination
// steps (Sec. III.B, Sec. IV.A, App. A).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "qgm.h"
#include "program.hpp"
#include "tree.hpp"

namespace qgm {

// One worldline variable b_q^k (Sec. III.A).
struct VarInfo {
    int qubit = -1;
    int k = 0;               // index along the worldline: 0 = input, d_q = output
    bool is_c0 = false;      // b_q^0, fixed to 0 by the input delta
    bool is_final = false;   // b_q^{d_q}, fixed to x_q unless the qubit is open
    int open_idx = -1;       // output-index bit when the qubit is open
    int slice_idx = -1;      // >= 0 when the variable is sliced
};

// A gate in time order, with the variables its factor touches.
struct GateRec {
    int type = 0;            // 0 = non-diagonal 1q, 1 = diagonal 1q, 2 = CZ, 3 = non-diagonal 2q (QGM_U2)
    int q0 = -1, q1 = -1;
    int var0 = -1, var1 = -1;   // NONDIAG: (new, old); DIAG: (cur, -1); CZ: (cur q0, cur q1);
                                // 2q: (new q0, new q1), with var2, var3 = (old q0, old q1)
    int var2 = -1, var3 = -1;
    int mat = -1;            // matrix index: 0..3 fixed kinds, 4 + slot for U/UD
    int gate_index = -1;     // row in the input gate list
};

// One elimination step: every variable of one qubit's worldline is summed
// out at once (the buckets of that worldline processed together).  With F
// the frontier tensor (product of all earlier bucket results) and G the
// product of the qubit's own factors summed over its internal variables:
//   F'[M, V, N] = sum_K F[M, V, K] * G_sigma[V, K, N].
struct Step {
    int qubit = -1;
    int r_in = 0, r_out = 0;
    int kb = 0, vb = 0, nb = 0, sb = 0;
    bool input_is_one = false;          // frontier is the constant 1 (first step)
    std::vector<int> in_axes, out_axes; // variable at each bit position
    std::vector<int> k_vars, v_vars, n_vars;
    std::vector<int> kpos;              // input position of K bit i (ascending)
    std::vector<int> vpos;              // output (row) position of V bit i
    std::vector<int> sig_src;           // variant bit i: qubit q (>= 0) or -(1 + slice index)
    std::vector<GOp> ops;               // factor program evaluated by the G builder
    int64_t g_off = 0;                  // complex offset of this step's G in the G table
    int kclass = 0;                     // 0 = vector-ALU kernel, 1 = FP32 MFMA kernel, 2 = BF16x3 MFMA kernel
    int pair_bit = -1;                  // vector-ALU kernel: rows paired on this row bit (-1: no pairing)
    int pair_in = 0;                    // input-tensor offset of the paired bit
    std::vector<int> inner_pos;         // MFMA tile: the 4 row positions inside a tile (no V axes)
    std::vector<int> outer_pos;         // MFMA tile: the other row positions
    int64_t g_entries() const { return int64_t(1) << (vb + kb + nb + sb); }
    double bytes_per_b() const;         // algorithmic HBM bytes per batch entry
    double flops_per_b() const;
};

struct Plan {
    int rows = 0, cols = 0, n = 0, n_slots = 0;
    int n_2q = 0;            // non-diagonal two-qubit gates (QGM_U2)
    int n_open = 0;
    std::vector<int> open_qubits;
    qgm_plan_opts opts{};
    std::vector<VarInfo> vars;
    std::vector<std::vector<int>> chain;     // chain[q] = worldline variables of qubit q
    std::vector<GateRec> recs;               // time-ordered gates
    std::vector<int> order;                  // elimination order of qubits (ordering 0)
    std::vector<Step> steps;
    std::vector<int> sliced;                 // sliced variable ids
    std::vector<int> final_pos;              // output bit i -> position in the last frontier
    int r_max = 0;
    int64_t g_total = 0;
    int64_t n_ops_total = 0;
    int n_diag_gates = 0, n_nondiag_gates = 0, n_cz = 0;
    int ckpt_every = 0;                      // qgm_backward checkpoint interval chosen for checkpoint_budget (0: none)
    bool is_tree = false;                    // ordering 1: bucket elimination with a greedy order
    TreePlan tree;
    // Device copies of the constant tables, one per device ordinal.
    struct DevTables { int device = -1; void* base = nullptr; };
    std::vector<DevTables> dev;
};

// Kernel candidates of an elimination step.
enum { KC_VALU = 0, KC_VALU_PAIR = 1, KC_MFMA_F32 = 2, KC_MFMA_BF16X3 = 3 };
bool step_supports(const Step& st, int cand);
void configure_step(Step& st, int cand);

// Builds the plan; returns QGM_OK or an error code with a message in *err.
qgm_status build_plan(const qgm_circuit* c, const int32_t* open, int32_t n_open,
                      const qgm_plan_opts& opts, Plan& p, std::string* err);

std::string plan_json(const Plan& p, int detail);

// Slices (bitstring copies per call) and padded batch.
int64_t padded_batch(int64_t B);
// Row pitch of the bucket path's arena: the padded batch rounded up to a power
// of two, so that the kernels scale rows by a shift.
int64_t tree_pitch(int64_t B);
inline int64_t batch_eff(const Plan& p, int64_t B) {
    return p.is_tree ? tree_pitch(B << p.tree.chunk_bits) : padded_batch(B) << p.sliced.size();
}

// Workspace of a call.  Ordering 0: two frontier buffers, the variant ids
// and the G table.  Ordering 1: the arena of bucket results (f0) and, when
// the circuit reads gate values, the factor tables (g).
struct WsLayout {
    uint64_t f0 = 0, f1 = 0, var_ids = 0, g = 0, flags = 0, total = 0;
    uint64_t ext = 0, part = 0, acc = 0;   // ordering 1 with slicing: column words, column amplitudes, sums
};
WsLayout workspace_layout(const Plan& p, int64_t B);
// ... of a bucket plan run with 2^chunk_bits slices per chunk (the plan's own chunk in workspace_layout).
WsLayout workspace_layout_chunk(const Plan& p, int64_t B, int chunk_bits);
// The gates of U, O, U^dag restricted to O's backward light cone (qgm_expectation_circuit).
qgm_status expectation_circuit(const qgm_circuit* c, int32_t n_ops, const int32_t* qubits, const int32_t* paulis,
                               std::vector<qgm_gate>& out, std::string* err);
// Bucket plans: whether qgm_amplitudes runs a batch of B in one persistent launch,
// and the words of one bitstring group's completion flags in that launch.
bool tree_persistent(const Plan& p, int64_t B);
// ... or in the LDS-resident launch (one work-group per bitstring, tree_exec 3, the default when it fits)
bool tree_lds(const Plan& p, int64_t B);
int64_t tree_flag_stride(const Plan& p);
int64_t tree_flag_words(const Plan& p, int64_t B);   // the whole flags area (header, ranks, flags)

}  // namespace qgm
