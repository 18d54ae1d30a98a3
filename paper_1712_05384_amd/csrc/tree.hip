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

constexpr int kTreeMaxPrologueFactors = 64;

// Prologue of a call: the factor table of every bucket (blockIdx.y <
// n_gtabs; a bucket without factors has a table of ones), the sigma rows
// (n_gtabs <= blockIdx.y < n_gtabs + n_sig) and the arena's constant-1 row
// (last blockIdx.y).  Table entry e = (c << sb) | sigma with
// c = (g << 1) | v holds the product of the bucket's gate factors (Sec. III.B)
// for those variable values, in FP64 rounded once to complex64; entries of
// summed-variable values w >= 2^k (a bucket summing fewer variables than its
// launch) are 0.
__global__ void __launch_bounds__(256) k_tree_prologue(const TreeGTab* __restrict__ gtabs, int n_gtabs,
                                                       const TFactor* __restrict__ facs,
                                                       const double2* __restrict__ fixed,
                                                       const float2* __restrict__ slots, float2* __restrict__ gtab,
                                                       const TreeSigTab* __restrict__ sigtabs, int n_sig,
                                                       const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                       uint16_t* __restrict__ sigs, float2* __restrict__ ones) {
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (int(blockIdx.y) < n_gtabs) {
        // the four values of every factor of this bucket, and the index bits
        // feeding its variables, staged in LDS once per block
        __shared__ double2 fv[kTreeMaxPrologueFactors][4];
        __shared__ int32_t fs[kTreeMaxPrologueFactors][4];
        const TreeGTab t = gtabs[blockIdx.y];
        const uint32_t total = 1u << (t.gb + t.kg + t.sb);
        if (blockIdx.x * 256u >= total) return;   // whole block beyond this table (uniform)
        const int nf = t.n_fac < kTreeMaxPrologueFactors ? t.n_fac : kTreeMaxPrologueFactors;
        for (int i = threadIdx.x; i < nf * 4; i += 256) {
            const TFactor f = facs[t.fac_off + (i >> 2)];
            fv[i >> 2][i & 3] = factor_value(f, (i >> 1) & 1u, i & 1u, fixed, slots);
            if ((i & 3) == 0) {
                fs[i >> 2][0] = f.src0;
                fs[i >> 2][1] = f.bit0;
                fs[i >> 2][2] = f.src1;
                fs[i >> 2][3] = f.bit1;
            }
        }
        __syncthreads();
        if (e >= total) return;
        const uint32_t sig = e & ((1u << t.sb) - 1u);
        const uint32_t c = e >> t.sb;
        if (((c & ((1u << t.kg) - 1u)) >> t.k) != 0u) {   // summed-variable slots the bucket does not have
            gtab[t.g_off + e] = make_float2(0.f, 0.f);
            return;
        }
        auto val = [&](int32_t src, int32_t bit) -> uint32_t {
            return src == TS_G ? (c >> bit) & 1u : (src == TS_SIG ? (sig >> bit) & 1u : 0u);
        };
        double2 acc = make_double2(1.0, 0.0);
        for (int i = 0; i < nf; ++i) acc = cmuld(acc, fv[i][val(fs[i][0], fs[i][1]) * 2u + val(fs[i][2], fs[i][3])]);
        for (int i = nf; i < t.n_fac; ++i) {   // beyond the LDS copy: read the records directly
            const TFactor f = facs[t.fac_off + i];
            acc = cmuld(acc, factor_value(f, val(f.src0, f.bit0), val(f.src1, f.bit1), fixed, slots));
        }
        gtab[t.g_off + e] = make_float2(float(acc.x), float(acc.y));
        return;
    }
    if (e >= B_eff) return;
    const int r = int(blockIdx.y) - n_gtabs;
    if (r == n_sig) {   // the arena's constant-1 row
        ones[e] = make_float2(1.f, 0.f);
        return;
    }
    const TreeSigTab st = sigtabs[r];
    const uint64_t x = int64_t(e) < B ? bits[e] : 0ull;
    uint32_t sig = 0;
    for (int i = 0; i < st.sb; ++i) sig |= uint32_t((x >> st.q[i]) & 1ull) << i;
    sigs[size_t(r) * B_eff + e] = uint16_t(sig);
}

// One level of the elimination tree.  Wave unit u handles task u / n_bg
// (2^kTreeOcBits consecutive result rows of one bucket) for the 64
// bitstrings of group u % n_bg:
//   R[o][b] = sum_{w < 2^K} G[g(o), w, sigma(b)] * prod_t T_t[idx_t(o) + off_t(w)][b],
// w running over the values of the bucket's summed variables (one, or up to
// three for a merged chain).  The code has no data-dependent branch: a
// bucket with fewer inputs than NIN multiplies the arena's constant-1 row,
// one summing fewer variables than K has zeros in its table at the extra w,
// one without output bits reads the all-zero sigma row, and the chunk of a
// result with fewer than 2^kTreeOcBits rows wraps onto valid rows and stores
// into rows the arena reserves for it.  Inputs (ain) and results (aout) are
// views of one arena that a level never reads and writes at the same rows, so
// the loads of a batch of rows can all be in flight at once.
template <int NIN, int K>
__global__ void __launch_bounds__(256) k_tree_level(const TreeTask* __restrict__ tasks, uint32_t n_units,
                                                    const TreeStepDev* __restrict__ steps,
                                                    const float2* __restrict__ ain, float2* __restrict__ aout,
                                                    const float2* __restrict__ gtab, const uint16_t* __restrict__ sigs,
                                                    uint32_t B_eff, uint32_t n_bg) {
    constexpr int OC = 1 << kTreeOcBits;
    constexpr int W = 1 << K;
    constexpr int WC = W < 8 ? W : 8;          // summed-variable values per load batch
    constexpr int LPB = (NIN + 1) * WC;         // loads per row and batch
    // rows whose loads are issued together: up to about 64 loads in flight per wave
    constexpr int OB = LPB <= 8 ? OC : (LPB <= 16 ? OC / 2 : (LPB <= 32 ? OC / 4 : OC / 8));
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t be = int64_t(B_eff);
    for (uint32_t u = blockIdx.x * 4u + wave; u < n_units; u += gridDim.x * 4u) {
        const uint32_t ti = u / n_bg;
        const uint32_t bg = u - ti * n_bg;
        const TreeTask tk = tasks[ti];
        const TreeStepDev sd = steps[tk.step];
        const uint32_t b = bg * 64u + lane;
        const int64_t sig = sigs[int64_t(sd.sig_row) * be + b];
        // input rows and factor-table entry of every row of the chunk, and the
        // row offset of each summed-variable value w in each input (scalar)
        int64_t row[OC][NIN], gent[OC], off[NIN][W];
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            row[0][t] = tk.in_row[t];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                int64_t o = 0;
#pragma unroll
                for (int i = 0; i < K; ++i)
                    if ((w >> i) & 1) o += sd.in_vs[t][i];
                off[t][w] = o * be;
            }
        }
        gent[0] = tk.g_ent;
#pragma unroll
        for (int oi = 1; oi < OC; ++oi) {
            const int j = __builtin_ctz(uint32_t(oi));
#pragma unroll
            for (int t = 0; t < NIN; ++t) row[oi][t] = row[oi - 1][t] + sd.in_inc[t][j];
            gent[oi] = gent[oi - 1] + (int64_t(sd.g_inc[j]) << sd.gshift);
        }
        float2* __restrict__ out = aout + int64_t(tk.out_row) * be + b;
#pragma unroll
        for (int o0 = 0; o0 < OC; o0 += OB) {
            float2 acc[OB];
#pragma unroll
            for (int i = 0; i < OB; ++i) acc[i] = make_float2(0.f, 0.f);
#pragma unroll
            for (int w0 = 0; w0 < W; w0 += WC) {
                float2 a[OB][NIN][WC], q[OB][WC];
#pragma unroll
                for (int i = 0; i < OB; ++i)
#pragma unroll
                    for (int t = 0; t < NIN; ++t) {
                        const float2* __restrict__ src = ain + row[o0 + i][t] * be + b;
#pragma unroll
                        for (int w = 0; w < WC; ++w) a[i][t][w] = src[off[t][w0 + w]];
                    }
#pragma unroll
                for (int i = 0; i < OB; ++i)
#pragma unroll
                    for (int w = 0; w < WC; ++w) q[i][w] = gtab[gent[o0 + i] + (int64_t(w0 + w) << sd.sb) + sig];
#pragma unroll
                for (int i = 0; i < OB; ++i)
#pragma unroll
                    for (int w = 0; w < WC; ++w) {
                        float2 pw = q[i][w];
#pragma unroll
                        for (int t = 0; t < NIN; ++t) pw = cmulf(pw, a[i][t][w]);
                        acc[i].x += pw.x;
                        acc[i].y += pw.y;
                    }
            }
#pragma unroll
            for (int i = 0; i < OB; ++i) out[int64_t(o0 + i) * be] = acc[i];
        }
    }
}

// Amplitude of every bitstring: the phase of the factors without free
// variables times the rank-0 bucket results, multiplied in FP64.  The phase
// factors and their four values each are staged in LDS once per block.
constexpr int kTreeMaxPhaseLds = 512;

__global__ void __launch_bounds__(256) k_tree_final(const int64_t* __restrict__ final_rows, int n_final,
                                                    const TFactor* __restrict__ phase, int n_phase,
                                                    const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                                    const float2* __restrict__ arena, const uint64_t* __restrict__ bits,
                                                    int64_t B, uint32_t B_eff, void* __restrict__ out, int c128) {
    __shared__ double2 pv[kTreeMaxPhaseLds][4];
    __shared__ int32_t pq[kTreeMaxPhaseLds][2];   // bit of x feeding each variable (-1: fixed 0)
    const int n_lds = n_phase < kTreeMaxPhaseLds ? n_phase : kTreeMaxPhaseLds;
    for (int i = threadIdx.x; i < n_lds * 4; i += 256) {
        const TFactor f = phase[i >> 2];
        const uint32_t a = (i >> 1) & 1, c = i & 1;
        pv[i >> 2][i & 3] = factor_value(f, a, c, fixed, slots);
        if ((i & 3) == 0) {
            pq[i >> 2][0] = f.src0 == TS_SIG ? f.bit0 : -1;
            pq[i >> 2][1] = f.src1 == TS_SIG ? f.bit1 : -1;
        }
    }
    __syncthreads();
    const uint32_t b = blockIdx.x * 256u + threadIdx.x;
    if (int64_t(b) >= B) return;
    const uint64_t x = bits[b];
    double2 acc = make_double2(1.0, 0.0);
    for (int i = 0; i < n_lds; ++i) {
        const uint32_t a = pq[i][0] >= 0 ? uint32_t((x >> pq[i][0]) & 1ull) : 0u;
        const uint32_t c = pq[i][1] >= 0 ? uint32_t((x >> pq[i][1]) & 1ull) : 0u;
        acc = cmuld(acc, pv[i][a * 2 + c]);
    }
    for (int i = n_lds; i < n_phase; ++i) {   // beyond the LDS copy: read the records directly
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

void launch_tree_prologue(const TreeGTab* gtabs, int n_gtabs, uint32_t max_entries, const TFactor* facs,
                          const double2* fixed, const float2* slots, float2* gtab, const TreeSigTab* sigtabs,
                          int n_sig, const uint64_t* bits, int64_t B, uint32_t B_eff, uint16_t* sigs, float2* ones,
                          hipStream_t stream) {
    const uint32_t ny = uint32_t(n_gtabs + n_sig + 1);
    const uint32_t nx = std::max<uint32_t>(n_gtabs > 0 ? (max_entries + 255) / 256 : 1, (B_eff + 255) / 256);
    hipLaunchKernelGGL(k_tree_prologue, dim3(nx, ny), dim3(256), 0, stream, gtabs, n_gtabs, facs, fixed, slots, gtab,
                       sigtabs, n_sig, bits, B, B_eff, sigs, ones);
}

template <int NIN, int K>
static void launch_level_nk(uint32_t grid, hipStream_t stream, const TreeTask* tk, uint32_t n_units,
                            const TreeStepDev* steps, const float2* ain, float2* aout, const float2* gtab,
                            const uint16_t* sigs, uint32_t B_eff, uint32_t n_bg) {
    hipLaunchKernelGGL((k_tree_level<NIN, K>), dim3(grid), dim3(256), 0, stream, tk, n_units, steps, ain, aout, gtab,
                       sigs, B_eff, n_bg);
}

static_assert(kTreeMaxSum == 3, "launch_tree_level dispatches K = 1 .. 3");

template <int K>
static void launch_level_k(int nin, uint32_t grid, hipStream_t stream, const TreeTask* tk, uint32_t n_units,
                           const TreeStepDev* steps, const float2* ain, float2* aout, const float2* gtab,
                           const uint16_t* sigs, uint32_t B_eff, uint32_t n_bg) {
    if (nin <= 1) launch_level_nk<1, K>(grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
    else if (nin == 2) launch_level_nk<2, K>(grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
    else if (nin == 3) launch_level_nk<3, K>(grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
    else if (nin == 4) launch_level_nk<4, K>(grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
    else launch_level_nk<kTreeMaxIn, K>(grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
}

void launch_tree_level(int nin, int k, const TreeTask* tasks, int32_t n_tasks, const TreeStepDev* steps,
                       const float2* ain, float2* aout, const float2* gtab, const uint16_t* sigs, uint32_t B_eff,
                       hipStream_t stream) {
    const uint32_t n_bg = B_eff / 64u;
    // launches of at most 2^31 wave units (tasks of one level are independent)
    const int64_t per = std::max<int64_t>(1, (int64_t(1) << 31) / n_bg);
    for (int64_t t0 = 0; t0 < n_tasks; t0 += per) {
        const int64_t nt = std::min<int64_t>(per, n_tasks - t0);
        const uint32_t n_units = uint32_t(nt * n_bg);
        const uint32_t grid = uint32_t(std::min<int64_t>((int64_t(n_units) + 3) / 4, kStepMaxGrid));
        const TreeTask* tk = tasks + t0;
        if (k <= 1) launch_level_k<1>(nin, grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
        else if (k == 2) launch_level_k<2>(nin, grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
        else launch_level_k<3>(nin, grid, stream, tk, n_units, steps, ain, aout, gtab, sigs, B_eff, n_bg);
    }
}

void launch_tree_final(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                       const float2* slots, const float2* arena, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       void* out, bool c128, hipStream_t stream) {
    const uint32_t grid = uint32_t((B + 255) / 256);
    hipLaunchKernelGGL(k_tree_final, dim3(grid), dim3(256), 0, stream, final_rows, n_final, phase, n_phase, fixed,
                       slots, arena, bits, B, B_eff, out, c128 ? 1 : 0);
}

}  // namespace qgm
