// Device kernels of the amplitude path (gfx950).
//
// Data layout.  A frontier tensor of rank r is stored "batch-minor":
// element (i, b) of the [2^r][B_eff] array lives at i*B_eff + b, where i is
// the tensor index over its axes (bit p of i = the variable at position p)
// and b runs over bitstrings (and slice copies).  B_eff is a multiple of 64,
// so each wave covers 64 consecutive b of one tensor row and every load and
// store of every step is one contiguous 512-byte access, whatever the axis
// permutation of the step.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qgm {

__device__ __forceinline__ uint32_t src_value(int32_t src, int32_t bit, uint32_t k, uint32_t v, uint32_t n, uint32_t sig) {
    switch (src) {
        case SRC_K: return (k >> bit) & 1u;
        case SRC_V: return (v >> bit) & 1u;
        case SRC_N: return (n >> bit) & 1u;
        case SRC_SIG: return (sig >> bit) & 1u;
        default: return 0u;
    }
}

// Per-bitstring boundary (the output deltas of Eq. (psi_x)): for every step,
// the variant index sigma of the step's operand, gathered from the output
// bits (and slice bits) the step's factors touch.
__global__ void __launch_bounds__(256) k_boundary(const uint64_t* __restrict__ bits, int64_t B, uint32_t B_pad,
                                                  uint32_t B_eff, int n_steps, const StepTab* __restrict__ steps,
                                                  const int32_t* __restrict__ sig_src, uint16_t* __restrict__ vids) {
    const uint32_t be = blockIdx.x * 256u + threadIdx.x;
    if (be >= B_eff) return;
    const uint32_t slice = be / B_pad;
    const uint32_t b = be - slice * B_pad;
    const uint64_t x = (int64_t(b) < B) ? bits[b] : 0ull;
    for (int s = 0; s < n_steps; ++s) {
        const StepTab st = steps[s];
        uint32_t v = 0;
        for (int i = 0; i < st.sb; ++i) {
            const int32_t src = sig_src[st.sig_off + i];
            const uint32_t bit = src >= 0 ? uint32_t((x >> src) & 1ull) : ((slice >> (-src - 1)) & 1u);
            v |= bit << i;
        }
        vids[size_t(s) * B_eff + be] = uint16_t(v);
    }
}

// Builds the small operand G of every step from the gate matrices: for each
// entry (v, k, n, sigma) the worldline of the step's qubit is swept in time
// order with a 2-vector over its current variable (Sec. IV, Eq. (1delim)),
// multiplying in the qubit's factors (Sec. III.B) and summing its internal
// variables.  FP64 arithmetic, rounded to complex64 at the end.
__global__ void __launch_bounds__(256) k_build_g(const StepTab* __restrict__ steps, const GOp* __restrict__ ops,
                                                 const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                                 float2* __restrict__ gtab) {
    const StepTab st = steps[blockIdx.y];
    const uint32_t total = 1u << (st.vb + st.kb + st.nb + st.sb);
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= total) return;
    const uint32_t sig = e & ((1u << st.sb) - 1u);
    const uint32_t n = (e >> st.sb) & ((1u << st.nb) - 1u);
    const uint32_t k = (e >> (st.sb + st.nb)) & ((1u << st.kb) - 1u);
    const uint32_t v = e >> (st.sb + st.nb + st.kb);
    double s0r = 1.0, s0i = 0.0, s1r = 0.0, s1i = 0.0, rr = 0.0, ri = 0.0;
    for (int i = 0; i < st.n_ops; ++i) {
        const GOp op = ops[st.ops_off + i];
        const uint32_t val = src_value(op.src, op.bit, k, v, n, sig);
        if (op.type == GOP_PROJECT) {
            if (val) { s0r = 0.0; s0i = 0.0; } else { s1r = 0.0; s1i = 0.0; }
        } else if (op.type == GOP_MAT || op.type == GOP_DIAG) {
            double2 m00, m01, m10, m11;
            if (op.mat < kFixedMats) {
                m00 = fixed[op.mat * 4 + 0]; m01 = fixed[op.mat * 4 + 1];
                m10 = fixed[op.mat * 4 + 2]; m11 = fixed[op.mat * 4 + 3];
            } else {
                const float2* m = slots + size_t(op.mat - kFixedMats) * 4;
                m00 = make_double2(m[0].x, m[0].y); m01 = make_double2(m[1].x, m[1].y);
                m10 = make_double2(m[2].x, m[2].y); m11 = make_double2(m[3].x, m[3].y);
            }
            if (op.type == GOP_MAT) {
                const double a0r = m00.x * s0r - m00.y * s0i + m01.x * s1r - m01.y * s1i;
                const double a0i = m00.x * s0i + m00.y * s0r + m01.x * s1i + m01.y * s1r;
                const double a1r = m10.x * s0r - m10.y * s0i + m11.x * s1r - m11.y * s1i;
                const double a1i = m10.x * s0i + m10.y * s0r + m11.x * s1i + m11.y * s1r;
                s0r = a0r; s0i = a0i; s1r = a1r; s1i = a1i;
            } else {
                const double a0r = m00.x * s0r - m00.y * s0i, a0i = m00.x * s0i + m00.y * s0r;
                const double a1r = m11.x * s1r - m11.y * s1i, a1i = m11.x * s1i + m11.y * s1r;
                s0r = a0r; s0i = a0i; s1r = a1r; s1i = a1i;
            }
        } else if (op.type == GOP_CZ) {
            if (val) { s1r = -s1r; s1i = -s1i; }
        } else {  // GOP_END
            rr = val ? s1r : s0r;
            ri = val ? s1i : s0i;
        }
    }
    gtab[st.g_off + e] = make_float2(float(rr), float(ri));
}

// One elimination step (bucket processing of App. A for one worldline):
//   F'[row, n] = sum_k F[row (+) k, ...] * G_sigma(b)[v(row), k, n]
// Each wave owns 64 consecutive batch entries of R output rows (R = 2 pairs
// rows that differ in one non-V bit, so they share v and sigma): it loads the
// 2^KB contracted inputs of those rows into registers, then streams over the
// 2^nb outputs in chunks of NCH.  G is staged in LDS transposed as
// [v][sigma][n][k], the sigma pitch padded by one element: a lane's base depends
// only on (v, sigma), so every read of the unrolled k, j loops uses an
// immediate offset (no address arithmetic per multiply-add), and lanes whose
// bitstrings select different variants hit different banks.  Large G is read
// through the cache in its [v][k][n][sigma] order instead.  R = 2 (two rows
// per thread that share v and sigma) lets one G read feed two multiply-adds.
template <int KB, int NCH, bool USE_LDS, int R>
__global__ void __launch_bounds__(256) k_step(StepParams sp, const float2* __restrict__ fin,
                                              float2* __restrict__ fout, const uint16_t* __restrict__ vids,
                                              const float2* __restrict__ gtab, uint32_t B_eff, uint32_t nbb,
                                              uint32_t n_units) {
    extern __shared__ float2 glds[];
    constexpr int K = 1 << KB;
    const int nb = sp.nb, sb = sp.sb;
    const int N = 1 << nb;
    const float2* __restrict__ G = gtab + sp.g_off;
    const uint32_t SS = (uint32_t(K) << nb) + 1u;   // LDS pitch of one variant (padded)
    if constexpr (USE_LDS) {
        const uint32_t total = 1u << (sp.vb + KB + nb + sb);
        for (uint32_t e = threadIdx.x; e < total; e += 256) {
            const uint32_t sg = e & ((1u << sb) - 1u);
            const uint32_t n = (e >> sb) & ((1u << nb) - 1u);
            const uint32_t k = (e >> (sb + nb)) & uint32_t(K - 1);
            const uint32_t v = e >> (sb + nb + KB);
            glds[((v << sb) + sg) * SS + (n << KB) + k] = G[e];
        }
        __syncthreads();
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    uint32_t koff[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < KB; ++i) o |= uint32_t((k >> i) & 1) << sp.kpos[i];
        koff[k] = o;
    }
    for (uint32_t unit = blockIdx.x * 4u + wave; unit < n_units; unit += gridDim.x * 4u) {
        const uint32_t urow = unit / nbb;
        const uint32_t b = (unit - urow * nbb) * 64u + lane;
        uint32_t row = urow;
        if constexpr (R == 2) {
            const uint32_t p = uint32_t(sp.pair_bit);
            row = ((urow >> p) << (p + 1)) | (urow & ((1u << p) - 1u));
        }
        const uint32_t sig = vids[b];
        uint32_t inrow = row;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            const uint32_t p = uint32_t(sp.kpos[i]);
            inrow = ((inrow >> p) << (p + 1)) | (inrow & ((1u << p) - 1u));
        }
        uint32_t v = 0;
        for (int i = 0; i < sp.vb; ++i) v |= ((row >> sp.vpos[i]) & 1u) << i;
        float2 a[R][K];
        if (sp.input_is_one) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < K; ++k) a[r][k] = make_float2(k == 0 ? 1.f : 0.f, 0.f);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t ir = inrow + (r ? uint32_t(sp.pair_in) : 0u);
#pragma unroll
                for (int k = 0; k < K; ++k) a[r][k] = fin[size_t(ir + koff[k]) * B_eff + b];
            }
        }
        const uint32_t gv = (v << KB);
        const float2* gl = glds + ((v << sb) + sig) * SS;
        for (int nc = 0; nc < N; nc += NCH) {
            float2 acc[R][NCH];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < NCH; ++j) acc[r][j] = make_float2(0.f, 0.f);
            const float2* gc = gl + (uint32_t(nc) << KB);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t gbase = (((gv + k) << nb) + nc) << sb;
#pragma unroll
                for (int j = 0; j < NCH; ++j) {
                    const float2 g = USE_LDS ? gc[j * K + k] : G[gbase + (uint32_t(j) << sb) + sig];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        acc[r][j].x = fmaf(a[r][k].x, g.x, acc[r][j].x);
                        acc[r][j].x = fmaf(-a[r][k].y, g.y, acc[r][j].x);
                        acc[r][j].y = fmaf(a[r][k].x, g.y, acc[r][j].y);
                        acc[r][j].y = fmaf(a[r][k].y, g.x, acc[r][j].y);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t orow = row + (r ? (1u << sp.pair_bit) : 0u);
#pragma unroll
                for (int j = 0; j < NCH; ++j)
                    fout[size_t(orow + (uint32_t(nc + j) << sp.row_bits)) * B_eff + b] = acc[r][j];
            }
        }
    }
}

// Output stage: sum the slice copies in FP64 (the sliced variables of the
// plan) and reorder the open axes into the caller's order.
template <typename OutT>
__global__ void __launch_bounds__(256) k_finalize(const float2* __restrict__ f, uint32_t B_eff, uint32_t B_pad,
                                                  int64_t B, int n_slices, int n_open,
                                                  const int32_t* __restrict__ final_pos, OutT* __restrict__ out) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t n_out = int64_t(1) << n_open;
    if (t >= B * n_out) return;
    const int64_t b = t / n_out;
    const uint32_t o = uint32_t(t - b * n_out);
    uint32_t pos = 0;
    for (int i = 0; i < n_open; ++i) pos |= ((o >> i) & 1u) << final_pos[i];
    double re = 0.0, im = 0.0;
    for (int s = 0; s < n_slices; ++s) {
        const float2 v = f[size_t(pos) * B_eff + size_t(s) * B_pad + size_t(b)];
        re += double(v.x);
        im += double(v.y);
    }
    if constexpr (sizeof(OutT) == 16) out[t] = make_double2(re, im);
    else out[t] = make_float2(float(re), float(im));
}

// ---------------------------------------------------------------------------
// launch helpers

template <int KB, int NCH, bool L, int R>
static void launch_step_t(const StepParams& sp, const float2* fin, float2* fout, const uint16_t* vids,
                          const float2* gtab, uint32_t B_eff, uint32_t nbb, uint32_t n_units, size_t lds,
                          hipStream_t stream) {
    uint32_t grid = (n_units + 3) / 4;
    if (grid > kStepMaxGrid) grid = kStepMaxGrid;
    hipLaunchKernelGGL((k_step<KB, NCH, L, R>), dim3(grid), dim3(256), L ? lds : 0, stream, sp, fin, fout, vids,
                       gtab, B_eff, nbb, n_units);
}

template <int KB, bool L, int R>
static void launch_step_nch(int nch, const StepParams& sp, const float2* fin, float2* fout, const uint16_t* vids,
                            const float2* gtab, uint32_t B_eff, uint32_t nbb, uint32_t n_units, size_t lds,
                            hipStream_t stream) {
    switch (nch) {
        case 1: launch_step_t<KB, 1, L, R>(sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        case 2: launch_step_t<KB, 2, L, R>(sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        case 4: launch_step_t<KB, 4, L, R>(sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        default: launch_step_t<KB, 8, L, R>(sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
    }
}

template <bool L>
static void launch_step_kb(int kb, bool pair, int nch, const StepParams& sp, const float2* fin, float2* fout,
                           const uint16_t* vids, const float2* gtab, uint32_t B_eff, uint32_t nbb,
                           uint32_t n_units, size_t lds, hipStream_t stream) {
    if (pair) {   // row pairs: dense steps (K of 2^3..2^5)
        switch (kb) {
            case 3: launch_step_nch<3, L, 2>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
            case 4: launch_step_nch<4, L, 2>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
            default: launch_step_nch<5, L, 2>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        }
        return;
    }
    switch (kb) {
        case 0: launch_step_nch<0, L, 1>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        case 1: launch_step_nch<1, L, 1>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        case 2: launch_step_nch<2, L, 1>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        case 3: launch_step_nch<3, L, 1>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        case 4: launch_step_nch<4, L, 1>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        case 5: launch_step_nch<5, L, 1>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
        default: launch_step_nch<6, L, 1>(nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds, stream); break;
    }
}

void launch_step(const StepParams& sp, const float2* fin, float2* fout, const uint16_t* vids, const float2* gtab,
                 uint32_t B_eff, hipStream_t stream) {
    const uint32_t nbb = B_eff / 64;
    const bool pair = sp.pair_bit >= 0;
    const uint32_t n_units = (1u << (sp.row_bits - (pair ? 1 : 0))) * nbb;
    const int N = 1 << sp.nb;
    const int nch = N >= 8 ? 8 : N;
    const size_t lds_bytes = size_t(8) * ((size_t(1) << (sp.vb + sp.sb)) * ((size_t(1) << (sp.kb + sp.nb)) + 1));
    if (lds_bytes <= kStepLdsBytes)
        launch_step_kb<true>(sp.kb, pair, nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, lds_bytes, stream);
    else
        launch_step_kb<false>(sp.kb, pair, nch, sp, fin, fout, vids, gtab, B_eff, nbb, n_units, 0, stream);
}

void launch_boundary(const uint64_t* bits, int64_t B, uint32_t B_pad, uint32_t B_eff, int n_steps,
                     const StepTab* steps, const int32_t* sig_src, uint16_t* vids, hipStream_t stream) {
    hipLaunchKernelGGL(k_boundary, dim3((B_eff + 255) / 256), dim3(256), 0, stream, bits, B, B_pad, B_eff, n_steps,
                       steps, sig_src, vids);
}

void launch_build_g(const StepTab* steps, int n_steps, uint32_t max_entries, const GOp* ops, const double2* fixed,
                    const float2* slots, float2* gtab, hipStream_t stream) {
    hipLaunchKernelGGL(k_build_g, dim3((max_entries + 255) / 256, n_steps), dim3(256), 0, stream, steps, ops, fixed,
                       slots, gtab);
}

void launch_finalize(const float2* f, uint32_t B_eff, uint32_t B_pad, int64_t B, int n_slices, int n_open,
                     const int32_t* final_pos, void* out, bool c128, hipStream_t stream) {
    const int64_t total = B << n_open;
    const uint32_t grid = uint32_t((total + 255) / 256);
    if (c128)
        hipLaunchKernelGGL(k_finalize<double2>, dim3(grid), dim3(256), 0, stream, f, B_eff, B_pad, B, n_slices, n_open,
                           final_pos, static_cast<double2*>(out));
    else
        hipLaunchKernelGGL(k_finalize<float2>, dim3(grid), dim3(256), 0, stream, f, B_eff, B_pad, B, n_slices, n_open,
                           final_pos, static_cast<float2*>(out));
}

}  // namespace qgm
