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
// field is 32- or 64-bit at its natural alignment).
struct TreeStepDev {
    int32_t r_out, n_in, sb, oc_bits;     // result rank, inputs, output bits, log2(o per wave unit)
    int32_t has_g, pad0;
    int64_t n_chunks;                     // 2^(r_out - oc_bits)
    int64_t g_off;                        // factor table: entry (((g << 1) | v) << sb) | sigma
    int64_t out_row;                      // arena row of the result
    int64_t in_row[kTreeMaxIn];           // arena row of each input
    int32_t in_v[kTreeMaxIn];             // row stride of v in input t (0: v is not an axis of t)
    int32_t in_str[kTreeMaxIn][kTreeMaxRank];   // row stride of result bit j in input t
    int32_t in_inc[kTreeMaxIn][kTreeOcBits];    // row change of input t when o -> o + 1 with ctz(o + 1) = j
    int32_t g_str[kTreeMaxRank];                // factor-table g stride of result bit j
    int32_t g_inc[kTreeOcBits];
    int32_t sig_q[kTreeMaxSig];                 // sigma bit i = bit sig_q[i] of the bitstring
};

// Factor-table record of one bucket (G builder).
struct TreeGTab {
    int32_t gb, sb, fac_off, n_fac;
    int64_t g_off;
};

// Buckets of one level launch; bucket k owns wave units [unit_start[k], unit_start[k + 1]).
struct TreeLevel {
    int32_t n;
    int32_t step[kTreeLevelSlots];
    int32_t unit_start[kTreeLevelSlots + 1];
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

void launch_tree_g(const TreeGTab* tabs, int n_tabs, uint32_t max_entries, const TFactor* facs, const double2* fixed,
                   const float2* slots, float2* gtab, hipStream_t stream);
void launch_tree_level(const TreeLevel& lv, const TreeStepDev* steps, float2* arena, const float2* gtab,
                       const uint64_t* bits, int64_t B, uint32_t B_eff, hipStream_t stream);
void launch_tree_final(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                       const float2* slots, const float2* arena, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       void* out, bool c128, hipStream_t stream);

}  // namespace qgm
