// Device kernels of the bucket-elimination path (ordering 1, gfx950).
//
// Every bucket result is a batch-minor [2^r][B_eff] complex64 array in one
// arena: element (o, b) lives at (row + o) * B_eff + b, so a wave that owns 64
// consecutive bitstrings reads and writes 512 contiguous bytes per tensor row
// whatever the bucket's axes.  The index arithmetic of a bucket (which input
// row belongs to result row o and value v of the summed variable) depends on
// o only, so it runs on the scalar unit; only the data and the per-bitstring
// factor variant sigma are per lane.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qgm {

namespace {

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cmuld(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 mat_entry(const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                             int32_t mat, uint32_t i) {
    if (mat < kFixedMats) return fixed[mat * 4 + int(i)];
    const float2 m = slots[size_t(mat - kFixedMats) * 4 + i];
    return make_double2(m.x, m.y);
}

// Value of one gate factor (Sec. III.B) for the given variable values.
__device__ __forceinline__ double2 factor_value(const TFactor& f, uint32_t a, uint32_t b, const double2* __restrict__ fixed,
                                                const float2* __restrict__ slots) {
    switch (f.type) {
        case TF_MAT: return mat_entry(fixed, slots, f.mat, a * 2u + b);   // row = the variable after the gate
        case TF_DIAG: return mat_entry(fixed, slots, f.mat, a * 3u);
        case TF_CZ: return make_double2((a & b) ? -1.0 : 1.0, 0.0);
        default: return make_double2(a ? 0.0 : 1.0, 0.0);              // TF_DELTA0
    }
}

}  // namespace

// Factor table of every bucket: entry e = (c << sb) | sigma with
// c = (g << 1) | v holds the product of the bucket's gate factors for those
// variable values (FP64, rounded to complex64 once).
__global__ void __launch_bounds__(256) k_tree_g(const TreeGTab* __restrict__ tabs, const TFactor* __restrict__ facs,
                                                const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                                float2* __restrict__ gtab) {
    const TreeGTab t = tabs[blockIdx.y];
    const uint32_t total = 1u << (t.gb + 1 + t.sb);
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= total) return;
    const uint32_t sig = e & ((1u << t.sb) - 1u);
    const uint32_t c = e >> t.sb;
    double2 acc = make_double2(1.0, 0.0);
    for (int i = 0; i < t.n_fac; ++i) {
        const TFactor f = facs[t.fac_off + i];
        const uint32_t a = f.src0 == TS_G ? (c >> f.bit0) & 1u : (f.src0 == TS_SIG ? (sig >> f.bit0) & 1u : 0u);
        const uint32_t b = f.src1 == TS_G ? (c >> f.bit1) & 1u : (f.src1 == TS_SIG ? (sig >> f.bit1) & 1u : 0u);
        acc = cmuld(acc, factor_value(f, a, b, fixed, slots));
    }
    gtab[t.g_off + e] = make_float2(float(acc.x), float(acc.y));
}

// One level of the elimination tree: every bucket of the level, each split
// into wave units of (2^oc_bits consecutive result rows) x (64 bitstrings).
// For each result row o and bitstring b:
//   R[o][b] = sum_{v = 0, 1} G[g(o), v, sigma(b)] * prod_t T_t[idx_t(o) + v * s_t][b].
__global__ void __launch_bounds__(256) k_tree_level(TreeLevel lv, const TreeStepDev* __restrict__ steps,
                                                    float2* __restrict__ arena, const float2* __restrict__ gtab,
                                                    const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                    uint32_t n_bg) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t total = uint32_t(lv.unit_start[lv.n]);
    for (uint32_t u = blockIdx.x * 4u + wave; u < total; u += gridDim.x * 4u) {
        int k = 0;
        while (k + 1 < lv.n && u >= uint32_t(lv.unit_start[k + 1])) ++k;
        const TreeStepDev* __restrict__ sd = steps + lv.step[k];
        const uint32_t lu = u - uint32_t(lv.unit_start[k]);
        const uint32_t chunk = lu / n_bg;
        const uint32_t bg = lu - chunk * n_bg;
        const uint32_t b = bg * 64u + lane;
        const int n_in = sd->n_in, sb = sd->sb, ocb = sd->oc_bits;
        const uint32_t o0 = chunk << ocb;
        uint32_t sig = 0;
        if (sb > 0) {
            const uint64_t x = int64_t(b) < B ? bits[b] : 0ull;
            for (int i = 0; i < sb; ++i) sig |= uint32_t((x >> sd->sig_q[i]) & 1ull) << i;
        }
        int64_t idx[kTreeMaxIn];
        int64_t vs[kTreeMaxIn];
#pragma unroll
        for (int t = 0; t < kTreeMaxIn; ++t) {
            idx[t] = 0;
            vs[t] = 0;
            if (t < n_in) {
                int64_t r = sd->in_row[t];
                for (uint32_t m = o0; m; m &= m - 1u) r += sd->in_str[t][__builtin_ctz(m)];
                idx[t] = r;
                vs[t] = int64_t(sd->in_v[t]) * B_eff;
            }
        }
        int64_t gi = 0;
        const bool has_g = sd->has_g != 0;
        if (has_g)
            for (uint32_t m = o0; m; m &= m - 1u) gi += sd->g_str[__builtin_ctz(m)];
        const float2* __restrict__ G = gtab + sd->g_off + sig;
        float2* __restrict__ out = arena + (sd->out_row + o0) * int64_t(B_eff) + b;
        const int n_oc = 1 << ocb;
#pragma unroll
        for (int oi = 0; oi < (1 << kTreeOcBits); ++oi) {
            if (oi >= n_oc) break;
            float2 p0 = make_float2(1.f, 0.f), p1 = p0;
            if (has_g) {
                p0 = G[(gi << 1) << sb];
                p1 = G[((gi << 1) | 1) << sb];
            }
#pragma unroll
            for (int t = 0; t < kTreeMaxIn; ++t) {
                if (t < n_in) {
                    const float2* __restrict__ src = arena + idx[t] * int64_t(B_eff) + b;
                    const float2 a0 = src[0];
                    const float2 a1 = vs[t] ? src[vs[t]] : a0;
                    p0 = cmulf(p0, a0);
                    p1 = cmulf(p1, a1);
                }
            }
            out[int64_t(oi) * B_eff] = make_float2(p0.x + p1.x, p0.y + p1.y);
            if (oi + 1 < n_oc) {
                const int j = __builtin_ctz(uint32_t(oi + 1));
#pragma unroll
                for (int t = 0; t < kTreeMaxIn; ++t)
                    if (t < n_in) idx[t] += sd->in_inc[t][j];
                gi += sd->g_inc[j];
            }
        }
    }
}

// Amplitude of every bitstring: the phase of the factors without free
// variables times the rank-0 bucket results, multiplied in FP64.
__global__ void __launch_bounds__(256) k_tree_final(const int64_t* __restrict__ final_rows, int n_final,
                                                    const TFactor* __restrict__ phase, int n_phase,
                                                    const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                                    const float2* __restrict__ arena, const uint64_t* __restrict__ bits,
                                                    int64_t B, uint32_t B_eff, void* __restrict__ out, int c128) {
    const uint32_t b = blockIdx.x * 256u + threadIdx.x;
    if (int64_t(b) >= B) return;
    const uint64_t x = bits[b];
    double2 acc = make_double2(1.0, 0.0);
    for (int i = 0; i < n_phase; ++i) {
        const TFactor f = phase[i];
        const uint32_t a = f.src0 == TS_SIG ? uint32_t((x >> f.bit0) & 1ull) : 0u;
        const uint32_t c = f.src1 == TS_SIG ? uint32_t((x >> f.bit1) & 1ull) : 0u;
        acc = cmuld(acc, factor_value(f, a, c, fixed, slots));
    }
    for (int i = 0; i < n_final; ++i) {
        const float2 r = arena[final_rows[i] * int64_t(B_eff) + b];
        acc = cmuld(acc, make_double2(r.x, r.y));
    }
    if (c128) static_cast<double2*>(out)[b] = acc;
    else static_cast<float2*>(out)[b] = make_float2(float(acc.x), float(acc.y));
}

void launch_tree_g(const TreeGTab* tabs, int n_tabs, uint32_t max_entries, const TFactor* facs, const double2* fixed,
                   const float2* slots, float2* gtab, hipStream_t stream) {
    if (n_tabs <= 0 || max_entries == 0) return;
    const dim3 grid((max_entries + 255) / 256, uint32_t(n_tabs));
    hipLaunchKernelGGL(k_tree_g, grid, dim3(256), 0, stream, tabs, facs, fixed, slots, gtab);
}

void launch_tree_level(const TreeLevel& lv, const TreeStepDev* steps, float2* arena, const float2* gtab,
                       const uint64_t* bits, int64_t B, uint32_t B_eff, hipStream_t stream) {
    const uint32_t total = uint32_t(lv.unit_start[lv.n]);
    if (total == 0) return;
    const uint32_t grid = std::min<uint32_t>((total + 3) / 4, kStepMaxGrid);
    hipLaunchKernelGGL(k_tree_level, dim3(grid), dim3(256), 0, stream, lv, steps, arena, gtab, bits, B, B_eff,
                       B_eff / 64u);
}

void launch_tree_final(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                       const float2* slots, const float2* arena, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       void* out, bool c128, hipStream_t stream) {
    const uint32_t grid = uint32_t((B + 255) / 256);
    hipLaunchKernelGGL(k_tree_final, dim3(grid), dim3(256), 0, stream, final_rows, n_final, phase, n_phase, fixed,
                       slots, arena, bits, B, B_eff, out, c128 ? 1 : 0);
}

}  // namespace qgm
