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

// Device record of one bucket of a tree plan (read with scalar loads: every
// field is 32-bit).
struct TreeStepDev {
    int32_t n_in, sb, sig_row, gshift;          // inputs, output bits, row of the sigma table, kg + sb
    int32_t in_vs[kTreeMaxIn][kTreeMaxSum];     // row stride of summed variable i in input t (0: not an axis
                                                //   of t, or t is a constant-1 pad beyond the bucket's inputs)
    int32_t in_inc[kTreeMaxIn][kTreeOcBits];    // row change of input t when o -> o + 1 with ctz(o + 1) = j
    int32_t g_inc[kTreeOcBits];                 // factor-table g change for the same steps
    int32_t pad;
};

// One wave task: a chunk of 2^kTreeOcBits consecutive result rows of a
// bucket (times the 64-bitstring groups of the batch).  A result of rank
// below kTreeOcBits has one chunk whose rows wrap around its index space; the
// arena reserves 2^kTreeOcBits rows for it, so all rows of the chunk are
// stored and only the first 2^rank are read.
struct TreeTask {
    int32_t step;                               // bucket
    int32_t pad;
    int32_t out_row;                            // arena row of the chunk's first result row
    int32_t g_ent;                              // factor-table entry of (g(o0), w = 0, sigma = 0)
    int32_t in_row[kTreeMaxIn];                 // arena row of input t at (o0, v = 0)
};

// Factor-table record of one bucket (prologue kernel).
struct TreeGTab {
    int32_t gb, sb, k, kg;                      // entry e = (((g << kg) | w) << sb) | sigma; w >= 2^k gives 0
    int32_t fac_off, n_fac;
    int64_t g_off;
};

// Sigma-table record of one bucket: sigma bit i = bit q[i] of the bitstring.
struct TreeSigTab {
    int32_t sb;
    int32_t q[kTreeMaxSig];
    int32_t pad[3];
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

void launch_tree_prologue(const TreeGTab* gtabs, int n_gtabs, uint32_t max_entries, const TFactor* facs,
                          const double2* fixed, const float2* slots, float2* gtab, const TreeSigTab* sigtabs,
                          int n_sig, const uint64_t* bits, int64_t B, uint32_t B_eff, uint16_t* sigs, float2* ones,
                          hipStream_t stream);
void launch_tree_level(int nin, int k, const TreeTask* tasks, int32_t n_tasks, const TreeStepDev* steps,
                       const float2* ain, float2* aout, const float2* gtab, const uint16_t* sigs, uint32_t B_eff,
                       hipStream_t stream);
void launch_tree_final(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                       const float2* slots, const float2* arena, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       void* out, bool c128, hipStream_t stream);

}  // namespace qgm
