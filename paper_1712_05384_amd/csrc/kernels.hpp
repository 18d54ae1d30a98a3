// Launch interface of the device kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "program.hpp"
#include "tree.hpp"

namespace qgm {

// Per-step record of the device tables (boundary and G builder).
struct StepTab {
    int32_t vb, kb, nb, sb;
    int32_t ops_off, n_ops;
    int32_t sig_off, pad;
    int64_t g_off;
};

// Launch parameters of the matrix-core step kernel.
struct DenseParams {
    StepParams sp;
    int32_t inner_pos[4];
    int32_t outer_pos[kMaxRank];
    int32_t n_outer;
    int32_t bf16x3;           // 1: BF16x3 split-precision matrix cores, 0: FP32 matrix cores
};

// Launch parameters of the Gbar partial-product kernel.
struct GbarParams {
    StepParams sp;
    int32_t kw, nw;             // widths of the k and n slices (<= 8)
    int32_t n_kc, n_nc, n_rc;   // number of k slices, n slices, row chunks
    int32_t rc_rows;            // rows per chunk
    int32_t n_free;             // row bits that are not V bits
    int32_t free_pos[kMaxRank];
};

// Records of a tree plan's device tables (read with scalar loads: every
// field is 32- or 64-bit at its natural alignment).

// One wave task of a bucket with inputs: tree_unit_rows(launch inputs, k)
// consecutive result rows (times the 64-bitstring groups of the batch), with
// everything the unit needs about its bucket, so a wave reads one record.  A
// result with fewer rows has one task whose rows wrap around its index space;
// the arena reserves 2^kTreeOcBits rows for every result, so all rows of the
// task are stored and only the first 2^rank are read.
struct TreeTask {
    int32_t k;                                  // summed variables (1 .. kTreeMaxSum)
    int32_t n_sig, sb, gshift;                  // output bits read by the factors; gshift = k + sb
    int32_t out_row;                            // arena row of the task's first result row
    int32_t g_ent;                              // factor-table entry of (g(o0), w = 0, sigma = 0)
    int32_t n_in;                               // inputs of the bucket
    int32_t nin_class;                          // input variant of its level's launch (launch_inputs), which
                                                //   fixes the result rows a unit computes
    int32_t in_row[kTreeMaxIn];                 // arena row of input t at (o0, w = 0); -1 for t beyond the
                                                //   bucket's inputs (the wave reads the constant 1 instead)
    int32_t sig_q[kTreeMaxSig];                 // sigma bit i = bit sig_q[i] of the bitstring
    int32_t in_vs[kTreeMaxIn][kTreeMaxSum];     // row stride of summed variable i in input t (0: not an axis)
    int32_t in_inc[kTreeMaxIn][kTreeOcBits];    // row change of input t when o -> o + 1 with ctz(o + 1) = j
    int32_t g_inc[kTreeOcBits];                 // factor-table g change for the same steps
    int32_t tile;                               // 0: the general unit; 1 (two inputs), 2 (three): a tile unit
                                                //   whose input 0 varies along unit bits 0, 1, input 1 along
                                                //   bit 2, input 2 and the factor table along none: 8 rows
    int32_t dep_off[kTreeMaxIn];                // tasks of the bucket that makes input t: [dep_off, dep_off + dep_n)
    int32_t dep_n[kTreeMaxIn];
    int32_t in_omask[kTreeMaxIn];               // bit j: input t's row changes along the unit's result row bit j
    int32_t g_omask;                            // the same for the factor-table entry
    int32_t pad3;                               // (in the tail's copies of its tasks, out_row and g_ent count
                                                //   rows and entries of the tail kernel's LDS)
    // an input that is a leaf table (a bucket without inputs, built with the plan): its entry offset in the
    // factor-table area (-1: an arena result; -2, in the tail's copies: a result in the tail kernel's LDS,
    // in_row counting rows there), its output bits and their qubits (6 bits each); row r, bits s of the
    // lane's bitstring -> entry offset + (r << sb) + s
    int32_t in_tab[kTreeMaxIn];
    int32_t in_tsb[kTreeMaxIn];
    uint64_t in_tsig[kTreeMaxIn];
    int32_t pad4[2];                            // a whole number of 16-byte words (the tail copies records)
};
static_assert(sizeof(TreeTask) % 16 == 0, "task records are copied in 16-byte words");

// The leaf tables of a plan (built once): R[o][s] = sum_w G[((o << k) | w) << sb | s].
// A leaf table built with the plan: entry (o << sb) | sigma = sum over the k summed values w of the factor
// table's entry (((g << k) | w) << sb) | sigma, times, for a composed leaf (n_in > 0), each input leaf table t
// at (o_t << in_sb[t]) | sigma_t: g bit j = o bit gpos[j]; input axis a = o bit in_src[t][a], or summed bit
// in_src[t][a] - 16 when >= 16; sigma_t bit b = sigma bit in_spos[t][b].  A leaf without inputs has g = o.
// Leaves of depth d read only leaves of smaller depth (one launch per depth).
struct TreeLeaf {
    int64_t g_off, leaf_off;
    int32_t r, k, sb, n_in;
    int32_t gb, depth;
    int32_t gpos[16];
    int64_t in_off[kTreeMaxIn];
    int32_t in_sb[kTreeMaxIn], in_na[kTreeMaxIn];
    int8_t in_src[kTreeMaxIn][16];
    int8_t in_spos[kTreeMaxIn][16];
};

// One persistent launch of the bucket elimination (k_tree_persist): every
// task of every level and the amplitude product.  The flags area holds the
// abort word at [0], one word per (complex, rank) of the launch's work-groups
// from kPersistSeen0, and from kPersistFlags0 one completion flag per
// (bitstring group, task), the group's flags contiguous at a stride of
// flag_stride words.
struct TreePersist {
    const TreeTask* tasks;                      // tasks [task0, task0 + n_tasks) in level order (keep-all rows)
    int32_t task0, n_tasks;
    const int32_t* final_dep;                   // (first task, count) of each bucket making a rank-0 result
    int32_t n_final_dep;
    int32_t n_final;
    const int64_t* final_rows;
    const TFactor* phase;
    int32_t n_phase;
    int32_t c128;
    const double2* fixed;
    const float2* slots;
    float2* arena;
    const float2* gtab;
    int64_t ones_g;
    const uint64_t* bits;
    int64_t B;
    uint32_t B_eff;
    int32_t flag_stride;
    int32_t max_class;                          // largest input variant among the tasks (launch_inputs)
    int32_t* flags;
    void* out;
    int32_t* status;                            // the plan's failure record on this device (set, never cleared)
    int32_t spin_limit;                         // polls after which a wait gives up
    int32_t pad;
};

// Factor table of a bucket (prologue kernel): entry e = (((g << k) | w) << sb)
// | sigma is the product over the bucket's factor groups of (prod_f f), or of
// (sum over the group's own 2^k_int values of prod_f f).
struct TreeGTab {
    int32_t gb, sb, k, n_groups;
    int32_t group_off, n_fac;                   // first group record; factors of all groups
    int64_t g_off;
};

struct TreeGroup {
    int32_t fac_off, n_fac, k_int, pad;
};

// One block of the prologue: what it computes.
struct TreeProBlock {
    int32_t idx;       // factor table (-1: the FP64 values of the factors without free variables)
    int32_t sub;       // block within the table (256 entries)
};

// A level run by the tail kernel (one work-group per 64-bitstring group); its
// tasks are [task_off, task_off + n_tasks) of the tail's task copies.
struct TreeTailLevel {
    int32_t task_off, n_tasks, nin, pad;
};

// ---- adjoint of a bucket plan (qgm_backward with ordering 1) ----
// The adjoint keeps every forward result (each result at its own rows of a
// "keep-all" arena) and writes each result's adjoint at the same rows of an
// adjoint arena.  A bucket's index space is a = (o << k) | w: its result bits o
// and its summed bits w.
constexpr int kTreeMaxABits = 31;

struct TreeBwd {
    int32_t n_in, k, r, sb;
    int32_t a_bits, pad0;
    int32_t out_row;                            // keep-all row of the result and of its adjoint
    int32_t pad1;
    int64_t scratch_row;                        // H at [row, row + 2^a_bits), then Q_t for each input t
    int64_t g_off;                              // factor table base entry
    int32_t sig_q[kTreeMaxSig];
    int32_t in_row[kTreeMaxIn];                 // keep-all rows of the inputs
    int32_t in_str[kTreeMaxIn][32];             // row stride of a-bit i in input t
    int32_t g_str[32];                          // factor-table index stride of a-bit i (c units)
};

// One stage of a sum over a-bits: output row j of the record (an input's
// adjoint, H summed within a factor-table row, or a partial sum) is the sum of
// 2^n_sum source rows q_row + a0(j) + foff[f], where a0(j) places bit p of j at
// source-row bit pos[p].
constexpr int kTbSumBits = 5;
// Factor adjoints are summed without atomics: every table block (and each of
// the kTbPhaseBlocks blocks of the phase factors) writes its partial sums per
// factor, then one pass adds them in order.
constexpr uint32_t kTbGadjParts = 32;     // blocks per table-entry block of the factor adjoints (slot factors split)
constexpr uint32_t kTbPhaseBlocks = 64;  // blocks summing the phase factors' adjoints over the bitstrings
struct TreeBwdIn {
    int32_t r_t, n_sum;                         // output index bits; summed bits (at most kTbSumBits)
    int32_t dst_row;                            // first output row in the destination area
    int32_t dst_sel;                            // 0: adjoint arena, 1: row-sum area, 2: partial area
    int64_t q_row;                              // first source row (scratch, or the other partial area)
    int32_t pos[32];                            // source-row bit of output index bit p
    int32_t foff[1 << kTbSumBits];              // source-row offset of summed combination f
};

// Adjoint of a bucket's factor table, one table row c per block.
struct TreeBwdG {
    int32_t c_bits, sb;                         // c_bits = gb + k
    int64_t h_row;                              // row of H summed within table row c = 0 (row-sum area)
    int64_t g_off;                              // table base entry (the table adjoint has the same layout)
    int32_t sig_q[kTreeMaxSig];
};

// A list entry of one adjoint launch: descriptor index and its first row.
struct TreeBwdItem {
    int32_t idx;
    int32_t row0;
};

constexpr uint32_t kStepMaxGrid = 8192;           // work-groups of the step kernel (grid-stride beyond)
constexpr uint32_t kDenseMaxGrid = 4096;          // work-groups of the matrix-core step kernel
constexpr size_t kStepLdsBytes = 48 * 1024;       // G up to this size is staged in LDS

void launch_boundary(const uint64_t* bits, int64_t B, uint32_t B_pad, uint32_t B_eff, int n_steps,
                     const StepTab* steps, const int32_t* sig_src, uint16_t* vids, hipStream_t stream);
void launch_build_g(const StepTab* steps, int n_steps, uint32_t max_entries, const GOp* ops, const double2* fixed,
                    const float2* slots, float2* gtab, hipStream_t stream);
void launch_step(const StepParams& sp, const float2* fin, float2* fout, const uint16_t* vids, const float2* gtab,
                 uint32_t B_eff, hipStream_t stream);
void launch_dense(const DenseParams& dp, const float2* fin, float2* fout, const uint16_t* vids, const float2* gtab,
                  uint32_t B_eff, hipStream_t stream);
void launch_step_t(const StepParams& sp, const float2* cbar, float2* abar, const uint16_t* vids, const float2* gtab,
                   uint32_t B_eff, hipStream_t stream);
void launch_gbar(const GbarParams& gp, const float2* a, const float2* cbar, float2* part, const uint16_t* vids,
                 uint32_t B_eff, double2* gbar, hipStream_t stream);
void launch_gadj(const StepTab* steps, int n_steps, uint32_t max_entries, const GOp* ops, const double2* fixed,
                 const float2* slots, const double2* gbar, const int64_t* wave_base, double2* wpart, int max_ops,
                 hipStream_t stream);
void launch_slot_grads(const int32_t* slot_ops_off, const int32_t* slot_ops, const int64_t* wave_base,
                       const int32_t* step_waves, const double2* wpart, int max_ops, int n_slots, float2* grads,
                       hipStream_t stream);
void launch_seed(const float2* g, uint32_t B_eff, uint32_t B_pad, int64_t B, int n_open, const int32_t* final_pos,
                 float2* fbar, hipStream_t stream);
void launch_finalize(const float2* f, uint32_t B_eff, uint32_t B_pad, int64_t B, int n_slices, int n_open,
                     const int32_t* final_pos, void* out, bool c128, hipStream_t stream);

void launch_tree_prologue(const TreeProBlock* blocks, int n_blocks, const TreeGTab* gtabs, const TreeGroup* groups,
                          const TFactor* facs, const double2* fixed, const float2* slots, float2* gtab,
                          int64_t ones_g, const TFactor* phase, int n_phase, int64_t phase_g, hipStream_t stream);
// One level of a bucket plan for the first n_groups groups of 64 bitstrings;
// B_eff is the arena's row pitch and must be a power of two.
// n_quad: the first n_quad tasks (a multiple of 4) are quad tiles, run four to a work-group; quad_arena: both
// inputs of each of those buckets are arena results (not leaf tables)
void launch_tree_level(int nin, const TreeTask* tasks, int32_t n_tasks, const float2* ain, float2* aout,
                       const float2* gtab, int64_t ones_g, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       uint32_t n_groups, hipStream_t stream, int32_t n_quad = 0, bool quad_arena = false);
void launch_tree_final_open(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase,
                            const double2* fixed, const float2* slots, const float2* arena, int64_t open_row,
                            int n_open, uint32_t zero_mask, const uint64_t* bits, int64_t B, uint32_t B_eff,
                            void* out, bool c128, hipStream_t stream);
hipError_t launch_tree_persist(const TreePersist& a, hipStream_t stream);
void launch_tree_leaf_tables(const TreeLeaf* leaves, int n_leaves, int64_t max_entries, int max_depth, float2* gtab,
                             hipStream_t stream);
// Cross-entropy statistics and sampling from a set of amplitudes (xeb.hip).
uint64_t xeb_workspace_bytes(int64_t B);
void launch_xeb(const void* amps, bool c128, int64_t B, int n_qubits, double* out, double* ws, hipStream_t stream);
void launch_prob_sums(const void* amps, int c128, int64_t B, int64_t n_out, double* out, hipStream_t stream);
void launch_sample_set(const void* amps, bool c128, int64_t B, const double* u, int64_t m, int64_t* idx, double* ws,
                       hipStream_t stream);
void launch_persist_init(int32_t* flags, int64_t n_flags, void* out, int64_t B, bool c128, hipStream_t stream);
// The tail: levels, copies of their task records (results made in the tail
// and the tail's factor tables addressed in LDS), the rank-0 results (arena
// row, or -1 - LDS row), the phase factors with their FP64 values at float2
// entry phase_g of gtab and the bits they read (2 per factor, as staged by the
// tail: -1 none, -2 a two-qubit factor evaluated from its record).
struct TreeTailArgs {
    const TreeTailLevel* levels;
    const TreeTask* tasks;
    const int32_t* final_lds;
    const TFactor* phase;
    const int32_t* phase_q;
    const double2* fixed;
    const float2* slots;
    float2* arena;
    const float2* gtab;
    const uint64_t* bits;
    void* out;
    int64_t ones_g, tail_g0, phase_g, B;
    int32_t n_levels, n_tasks, n_final, n_phase, tail_g_entries, c128;
    uint32_t B_eff, pad;
};
void launch_tree_tail(const TreeTailArgs& a, hipStream_t stream);

// The LDS-resident launch of a bucket plan (tree_exec 3): one work-group of
// a.threads threads per bitstring, kLdsHeader bytes + a.lds_size complex64
// entries of dynamic LDS.
struct LdsArgs {
    const LdsStage* stages;
    const uint32_t* zent;                       // per table entry: its index in ztab | stage << 24
    const float2* ztab;                         // the staged copy of the tables (LdsStage), or (staged = 0)
                                                //   the table area itself
    const uint16_t* recs;                       // [job][kLdsRecordHalves]
    const int32_t* level_job_off;               // n_levels + 1
    const int32_t* finals;                      // LDS byte offsets of the rank-0 results
    const TFactor* phase;
    const int32_t* phq;                         // per phase factor: the bits its two variables read (-1: 0;
                                                //   -2: a two-qubit gate, evaluated from its record)
    const double2* pv;                          // per phase factor: its 4 FP64 values (the prologue's)
    const double2* fixed;
    const float2* slots;
    const float2* gtab;                         // factor tables (and leaf tables) of the call
    const uint64_t* bits;
    void* out;
    int64_t B;
    int32_t n_stages, n_entries, tables0, lds_size;
    int32_t n_levels, n_final, n_phase, c128;
    int32_t threads, n_jobs, recs0, staged;
};
void launch_tree_lds(const LdsArgs& a, hipStream_t stream);
// The staged copy of the tables for the LDS launch: for every stage, every sigma and every entry i of the
// stage, z[zoff + sigma * n + i] = gtab[entries[e0 + i].src + sigma]; max_m = the largest n << n_sig.
void launch_lds_stage(const LdsStage* stages, int n_stages, const LdsEntry* entries, const float2* gtab, float2* z,
                      int64_t max_m, hipStream_t stream);
void launch_tb_seed(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                    const float2* slots, const float2* arena, float2* adj, const uint64_t* bits, int64_t B,
                    uint32_t B_eff, const float2* grad_amps, void* amps_out, bool c128, double2* phibar,
                    hipStream_t stream);
void launch_tb_phase_adj(const TFactor* phase, int n_phase, const double2* fixed, const float2* slots,
                         const uint64_t* bits, int64_t B, const double2* phibar, const int64_t* part_off, int64_t f0,
                         double2* fpart, hipStream_t stream);
void launch_tb_fsum(const int64_t* part_off, int64_t n_fbar, const double2* fpart, double2* fbar,
                    hipStream_t stream);
void launch_tb_expand(const TreeBwdItem* items, int n_items, int64_t total_rows, const TreeBwd* bwd,
                      const float2* arena, const float2* adj, const float2* gtab, float2* scratch,
                      const uint64_t* bits, int64_t B, uint32_t B_eff, bool write_h, hipStream_t stream);
void launch_tb_reduce(const TreeBwdItem* items, int n_items, int64_t total_rows, const TreeBwdIn* bin,
                      const float2* src, float2* dst_adj, float2* dst_hsum, float2* dst_part, uint32_t B_eff,
                      hipStream_t stream);
void launch_tb_gbin(const TreeBwdItem* items, int n_items, int64_t total_rows, const TreeBwdG* bg, const float2* hsum,
                    const uint64_t* bits, int64_t B, uint32_t B_eff, double2* gbar, hipStream_t stream);
void launch_tb_gadj(const TreeProBlock* blocks, int n_blocks, const TreeGTab* gtabs, const TreeGroup* groups,
                    const TFactor* facs, const double2* fixed, const float2* slots, const double2* gbar,
                    const int64_t* part_off, double2* fpart, hipStream_t stream);
void launch_tb_slots(const int32_t* slot_off, const int32_t* slot_occ, int n_slots, const double2* fbar,
                     float2* grads, hipStream_t stream);
void launch_tree_final(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                       const float2* slots, const float2* arena, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       void* out, bool c128, hipStream_t stream);
// Slicing of bucket plans: the words of a chunk's batch columns (bitstring b, slice slice0 + j at column
// b * 2^chunk_bits + j, slice bits above bit n), and the FP64 sum of a chunk's column amplitudes
// (complex128 [B << chunk_bits][2^n_open]) into acc or, for the last chunk, into out.
void launch_slice_cols(const uint64_t* bits, int64_t B, int n, int chunk_bits, uint64_t slice0, uint64_t* cols,
                       hipStream_t stream);
void launch_slice_sum(const double2* part, int64_t B, int chunk_bits, int n_open, double2* acc, bool first, bool last,
                      void* out, bool c128, hipStream_t stream);

}  // namespace qgm
