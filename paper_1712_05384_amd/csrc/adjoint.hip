// Adjoint of the elimination path (gradients with respect to the gate values).
//
// Notation of the forward step s:  C[row, n] = sum_k A[row (+) k] G_sigma[v, k, n]
// with A = F_s (the frontier entering step s) and C = F_{s+1}.  All adjoints
// here are holomorphic: Xbar = d(sum_x w_x A_x)/dX for the seed w on the
// amplitudes, so that for a real loss L with torch gradient g_x on the
// amplitudes, w_x = conj(g_x) and dL/dRe U + i dL/dIm U = conj(Ubar).
//
//   Abar[row (+) k] = sum_n Cbar[row, n] G_sigma[v, k, n]          (k_step_t)
//   Gbar_sigma[v, k, n] = sum over (row, b) with sigma(b) = sigma and v(row) = v
//                         of A[row (+) k, b] Cbar[row, n, b]       (k_gbar + k_gbar_reduce)
// and Ubar for every gate of the step follows from Gbar by differentiating the
// worldline sweep that builds G (k_gadj): G[e] = e_end^T O_m ... O_1 e_0 with
// each O_i a 2x2 linear map, so dG[e]/dO_i = lambda_i s_{i-1}^T where
// s_{i-1} = O_{i-1} ... O_1 e_0 and lambda_i^T = e_end^T O_m ... O_{i+1}.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qgm {

__device__ __forceinline__ uint32_t src_val(int32_t src, int32_t bit, uint32_t k, uint32_t v, uint32_t n,
                                            uint32_t sig) {
    switch (src) {
        case SRC_K: return (k >> bit) & 1u;
        case SRC_V: return (v >> bit) & 1u;
        case SRC_N: return (n >> bit) & 1u;
        case SRC_SIG: return (sig >> bit) & 1u;
        default: return 0u;
    }
}

// Transposed step: reads the 2^nb adjoint outputs of a row and writes the 2^KB
// adjoint inputs.  Same wave layout as k_step (64 consecutive b of one row),
// G staged in LDS as [v][sigma][n][k] with a padded sigma pitch.
template <int KB, bool USE_LDS>
__global__ void __launch_bounds__(256) k_step_t(StepParams sp, const float2* __restrict__ cbar,
                                                float2* __restrict__ abar, const uint16_t* __restrict__ vids,
                                                const float2* __restrict__ gtab, uint32_t B_eff, uint32_t nbb,
                                                uint32_t n_units) {
    extern __shared__ float2 glds[];
    constexpr int K = 1 << KB;
    const int nb = sp.nb, sb = sp.sb;
    const int N = 1 << nb;
    const float2* __restrict__ G = gtab + sp.g_off;
    const uint32_t SS = (uint32_t(K) << nb) + 1u;
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
        const uint32_t row = unit / nbb;
        const uint32_t b = (unit - row * nbb) * 64u + lane;
        const uint32_t sig = vids[b];
        uint32_t inrow = row;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            const uint32_t p = uint32_t(sp.kpos[i]);
            inrow = ((inrow >> p) << (p + 1)) | (inrow & ((1u << p) - 1u));
        }
        uint32_t v = 0;
        for (int i = 0; i < sp.vb; ++i) v |= ((row >> sp.vpos[i]) & 1u) << i;
        const float2* gl = glds + ((v << sb) + sig) * SS;
        float2 acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = make_float2(0.f, 0.f);
        for (int n = 0; n < N; ++n) {
            const float2 c = cbar[size_t(row + (uint32_t(n) << sp.row_bits)) * B_eff + b];
            const float2* gn = gl + (n << KB);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float2 g = USE_LDS ? gn[k] : G[((((v << KB) + uint32_t(k)) << nb) + uint32_t(n)) << sb | sig];
                acc[k].x = fmaf(c.x, g.x, acc[k].x);
                acc[k].x = fmaf(-c.y, g.y, acc[k].x);
                acc[k].y = fmaf(c.x, g.y, acc[k].y);
                acc[k].y = fmaf(c.y, g.x, acc[k].y);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) abar[size_t(inrow + koff[k]) * B_eff + b] = acc[k];
    }
}

// Partial Gbar: thread (unit, b) with unit = ((v * n_rc + rc) * n_kc + kc) * n_nc + nc
// accumulates, over the RC rows of chunk rc (rows with V bits = v), the outer
// product of its 8-wide slices of A[., k] and Cbar[., n] for bitstring b.
// Output: part[unit][k'][n'][b] (complex64, b fastest).
__global__ void __launch_bounds__(256) k_gbar(GbarParams gp, const float2* __restrict__ a,
                                              const float2* __restrict__ cbar, float2* __restrict__ part,
                                              uint32_t B_eff) {
    const uint32_t b = blockIdx.x * 256u + threadIdx.x;
    if (b >= B_eff) return;
    const uint32_t unit = blockIdx.y;
    const StepParams& sp = gp.sp;
    const uint32_t nc = unit % gp.n_nc;
    const uint32_t kc = (unit / gp.n_nc) % gp.n_kc;
    const uint32_t rc = (unit / (gp.n_nc * gp.n_kc)) % gp.n_rc;
    const uint32_t v = unit / (gp.n_nc * gp.n_kc * gp.n_rc);
    const int kw = gp.kw, nw = gp.nw;   // slice widths (<= 8)
    uint32_t vdep = 0;
    for (int i = 0; i < sp.vb; ++i) vdep |= ((v >> i) & 1u) << sp.vpos[i];
    float2 acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = make_float2(0.f, 0.f);
    for (uint32_t r = 0; r < gp.rc_rows; ++r) {
        const uint32_t m = rc * gp.rc_rows + r;
        uint32_t row = vdep;
        for (int i = 0; i < gp.n_free; ++i) row |= ((m >> i) & 1u) << gp.free_pos[i];
        uint32_t inrow = row;
        for (int i = 0; i < sp.kb; ++i) {
            const uint32_t p = uint32_t(sp.kpos[i]);
            inrow = ((inrow >> p) << (p + 1)) | (inrow & ((1u << p) - 1u));
        }
        float2 av[8], cv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            av[i] = make_float2(0.f, 0.f);
            if (i < kw) {
                const uint32_t k = kc * uint32_t(kw) + uint32_t(i);
                if (sp.input_is_one) {
                    av[i] = make_float2(k == 0 ? 1.f : 0.f, 0.f);
                } else {
                    uint32_t o = 0;
                    for (int t = 0; t < sp.kb; ++t) o |= ((k >> t) & 1u) << sp.kpos[t];
                    av[i] = a[size_t(inrow + o) * B_eff + b];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            cv[j] = make_float2(0.f, 0.f);
            if (j < nw) {
                const uint32_t n = nc * uint32_t(nw) + uint32_t(j);
                cv[j] = cbar[size_t(row + (n << sp.row_bits)) * B_eff + b];
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                acc[i][j].x = fmaf(av[i].x, cv[j].x, acc[i][j].x);
                acc[i][j].x = fmaf(-av[i].y, cv[j].y, acc[i][j].x);
                acc[i][j].y = fmaf(av[i].x, cv[j].y, acc[i][j].y);
                acc[i][j].y = fmaf(av[i].y, cv[j].x, acc[i][j].y);
            }
    }
    float2* out = part + size_t(unit) * 64 * B_eff;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (i < kw && j < nw) out[size_t(i * 8 + j) * B_eff + b] = acc[i][j];
}

// Gbar[v][k][n][sigma] (complex128) = sum over row chunks and over the b with
// sigma(b) = sigma of the partials.  One work-group per (v, k, n): each thread
// walks its bitstrings (b = tid, tid + 256, ...) over all row chunks, adding
// into one of 16 register accumulators selected by sigma (a chunk of 16
// variants per pass), then the work-group sums each accumulator with a fixed
// LDS tree: the result does not depend on scheduling.
__global__ void __launch_bounds__(256) k_gbar_reduce(GbarParams gp, const float2* __restrict__ part,
                                                     const uint16_t* __restrict__ vids, uint32_t B_eff,
                                                     double2* __restrict__ gbar) {
    __shared__ double red[256][2];
    const StepParams& sp = gp.sp;
    const uint32_t vkn = blockIdx.x;                 // (v, k, n) without sigma
    const uint32_t n = vkn & ((1u << sp.nb) - 1u);
    const uint32_t k = (vkn >> sp.nb) & ((1u << sp.kb) - 1u);
    const uint32_t v = vkn >> (sp.nb + sp.kb);
    const uint32_t kc = k / uint32_t(gp.kw), ki = k % uint32_t(gp.kw);
    const uint32_t nc = n / uint32_t(gp.nw), nj = n % uint32_t(gp.nw);
    const uint32_t S = 1u << sp.sb;
    const int tid = threadIdx.x;
    for (uint32_t s0 = 0; s0 < S; s0 += 16) {
        double re[16], im[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) { re[q] = 0.0; im[q] = 0.0; }
        for (uint32_t b = uint32_t(tid); b < B_eff; b += 256) {
            const uint32_t sg = uint32_t(vids[b]) - s0;
            if (sg >= 16u) continue;
            // the row chunks' partials in order; 16 loads in flight before their adds (the order of the adds,
            // and so the sums, as one at a time)
            double xr = 0.0, xi = 0.0;
            auto at = [&](uint32_t rc) {
                const uint32_t unit = ((v * gp.n_rc + rc) * gp.n_kc + kc) * gp.n_nc + nc;
                return part[(size_t(unit) * 64 + ki * 8 + nj) * B_eff + b];
            };
            uint32_t rc = 0;
            for (; rc + 16 <= uint32_t(gp.n_rc); rc += 16) {
                float2 x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) x[u] = at(rc + uint32_t(u));
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    xr += double(x[u].x);
                    xi += double(x[u].y);
                }
            }
            for (; rc < uint32_t(gp.n_rc); ++rc) {
                const float2 x = at(rc);
                xr += double(x.x);
                xi += double(x.y);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const bool hit = sg == uint32_t(q);
                re[q] += hit ? xr : 0.0;
                im[q] += hit ? xi : 0.0;
            }
        }
        const uint32_t nq = S - s0 < 16u ? S - s0 : 16u;
        for (uint32_t q = 0; q < nq; ++q) {
            double r = 0.0, i = 0.0;
#pragma unroll
            for (int t = 0; t < 16; ++t) if (uint32_t(t) == q) { r = re[t]; i = im[t]; }
            red[tid][0] = r;
            red[tid][1] = i;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (tid < w) { red[tid][0] += red[tid + w][0]; red[tid][1] += red[tid + w][1]; }
                __syncthreads();
            }
            if (tid == 0) gbar[sp.g_off + (size_t(vkn) << sp.sb) + s0 + q] = make_double2(red[0][0], red[0][1]);
            __syncthreads();
        }
    }
}

// Gate environments of every step: thread per (step, G entry); per-wave sums of
// the contributions to each op's 2x2 matrix are written to
// wpart[(step_wave_base + wave)][op][4] (complex128).
__global__ void __launch_bounds__(256) k_gadj(const StepTab* __restrict__ steps, const GOp* __restrict__ ops,
                                              const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                              const double2* __restrict__ gbar, const int64_t* __restrict__ wave_base,
                                              double2* __restrict__ wpart, int max_ops) {
    const int s = blockIdx.y;
    const StepTab st = steps[s];
    const uint32_t total = 1u << (st.vb + st.kb + st.nb + st.sb);
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = (blockIdx.x * 256u + threadIdx.x) >> 6;   // wave index within the step
    if ((wv << 6) >= total) return;                               // whole wave out of range
    const bool live = e < total;
    const uint32_t sig = e & ((1u << st.sb) - 1u);
    const uint32_t n = (e >> st.sb) & ((1u << st.nb) - 1u);
    const uint32_t k = (e >> (st.sb + st.nb)) & ((1u << st.kb) - 1u);
    const uint32_t v = e >> (st.sb + st.nb + st.kb);
    // forward sweep, keeping the state before each op
    double2 sv[kMaxOps][2];
    double2 s0 = make_double2(1.0, 0.0), s1 = make_double2(0.0, 0.0);
    uint32_t endval = 0;
    auto mat = [&](int m, double2* out4) {
        if (m < kFixedMats) {
            for (int i = 0; i < 4; ++i) out4[i] = fixed[m * 4 + i];
        } else {
            const float2* p = slots + size_t(m - kFixedMats) * 4;
            for (int i = 0; i < 4; ++i) out4[i] = make_double2(p[i].x, p[i].y);
        }
    };
    auto cm = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
    auto ca = [](double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); };
    for (int i = 0; i < st.n_ops; ++i) {
        const GOp op = ops[st.ops_off + i];
        sv[i][0] = s0;
        sv[i][1] = s1;
        const uint32_t val = src_val(op.src, op.bit, k, v, n, sig);
        if (op.type == GOP_PROJECT) {
            if (val) s0 = make_double2(0.0, 0.0); else s1 = make_double2(0.0, 0.0);
        } else if (op.type == GOP_MAT) {
            double2 m[4];
            mat(op.mat, m);
            const double2 a0 = ca(cm(m[0], s0), cm(m[1], s1));
            const double2 a1 = ca(cm(m[2], s0), cm(m[3], s1));
            s0 = a0;
            s1 = a1;
        } else if (op.type == GOP_DIAG) {
            double2 m[4];
            mat(op.mat, m);
            s0 = cm(m[0], s0);
            s1 = cm(m[3], s1);
        } else if (op.type == GOP_CZ) {
            if (val) s1 = make_double2(-s1.x, -s1.y);
        } else {
            endval = val;
        }
    }
    // backward: lambda^T = gbar * e_end^T, pulled back through the ops
    const double2 gb = live ? gbar[st.g_off + e] : make_double2(0.0, 0.0);
    double2 l0 = endval ? make_double2(0.0, 0.0) : gb;
    double2 l1 = endval ? gb : make_double2(0.0, 0.0);
    double2* out = wpart + (size_t(wave_base[s]) + wv) * size_t(max_ops) * 4;
    for (int i = st.n_ops - 1; i >= 0; --i) {
        const GOp op = ops[st.ops_off + i];
        const uint32_t val = src_val(op.src, op.bit, k, v, n, sig);
        double2 c[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                        make_double2(0.0, 0.0)};
        if (op.type == GOP_PROJECT) {
            if (val) l0 = make_double2(0.0, 0.0); else l1 = make_double2(0.0, 0.0);
        } else if (op.type == GOP_MAT) {
            double2 m[4];
            mat(op.mat, m);
            // Mbar[a][b] += lambda[a] * s_prev[b]
            c[0] = cm(l0, sv[i][0]); c[1] = cm(l0, sv[i][1]);
            c[2] = cm(l1, sv[i][0]); c[3] = cm(l1, sv[i][1]);
            // lambda_prev = M^T lambda
            const double2 n0 = ca(cm(m[0], l0), cm(m[2], l1));
            const double2 n1 = ca(cm(m[1], l0), cm(m[3], l1));
            l0 = n0;
            l1 = n1;
        } else if (op.type == GOP_DIAG) {
            double2 m[4];
            mat(op.mat, m);
            c[0] = cm(l0, sv[i][0]);
            c[3] = cm(l1, sv[i][1]);
            l0 = cm(m[0], l0);
            l1 = cm(m[3], l1);
        } else if (op.type == GOP_CZ) {
            if (val) l1 = make_double2(-l1.x, -l1.y);
        }
        // wave sums of the contribution (zero for non-matrix ops and dead lanes)
        if (op.type == GOP_MAT || op.type == GOP_DIAG) {
            for (int q = 0; q < 4; ++q) {
                double re = live ? c[q].x : 0.0, im = live ? c[q].y : 0.0;
                for (int off = 32; off > 0; off >>= 1) {
                    re += __shfl_xor(re, off, 64);
                    im += __shfl_xor(im, off, 64);
                }
                if (lane == 0) out[i * 4 + q] = make_double2(re, im);
            }
        } else if (lane == 0) {
            for (int q = 0; q < 4; ++q) out[i * 4 + q] = make_double2(0.0, 0.0);
        }
    }
}

// Gate gradients: grads[slot] = conj(sum over the (step, op) that read the slot
// of the per-wave partials), in a fixed order.  torch convention.
__global__ void __launch_bounds__(64) k_slot_grads(const int32_t* __restrict__ slot_ops_off,
                                                   const int32_t* __restrict__ slot_ops,
                                                   const int64_t* __restrict__ wave_base,
                                                   const int32_t* __restrict__ step_waves,
                                                   const double2* __restrict__ wpart, int max_ops, int n_slots,
                                                   float2* __restrict__ grads) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= n_slots * 4) return;
    const int slot = t >> 2, q = t & 3;
    double re = 0.0, im = 0.0;
    for (int j = slot_ops_off[slot]; j < slot_ops_off[slot + 1]; ++j) {
        const int code = slot_ops[j];          // step * 65536 + op index in the step
        const int s = code >> 16, i = code & 0xffff;
        for (int w = 0; w < step_waves[s]; ++w) {
            const double2 x = wpart[((size_t(wave_base[s]) + w) * size_t(max_ops) + i) * 4 + q];
            re += x.x;
            im += x.y;
        }
    }
    grads[t] = make_float2(float(re), float(-im));
}

// Seed of the adjoint: Fbar[pos(o)][slice * B_pad + b] = conj(g[b][o]) (zero for padding).
__global__ void __launch_bounds__(256) k_seed(const float2* __restrict__ g, uint32_t B_eff, uint32_t B_pad,
                                              int64_t B, int n_open, const int32_t* __restrict__ final_pos,
                                              float2* __restrict__ fbar) {
    const uint32_t be = blockIdx.x * 256u + threadIdx.x;
    const uint32_t o = blockIdx.y;
    if (be >= B_eff) return;
    const uint32_t b = be % B_pad;
    uint32_t pos = 0;
    for (int i = 0; i < n_open; ++i) pos |= ((o >> i) & 1u) << final_pos[i];
    float2 x = make_float2(0.f, 0.f);
    if (int64_t(b) < B) {
        const float2 gv = g[size_t(b) * (size_t(1) << n_open) + o];
        x = make_float2(gv.x, -gv.y);
    }
    fbar[size_t(pos) * B_eff + be] = x;
}

// ---------------------------------------------------------------------------

template <int KB>
static void launch_step_t_kb(const StepParams& sp, const float2* cbar, float2* abar, const uint16_t* vids,
                             const float2* gtab, uint32_t B_eff, size_t lds, hipStream_t stream) {
    const uint32_t nbb = B_eff / 64;
    const uint32_t n_units = (1u << sp.row_bits) * nbb;
    uint32_t grid = (n_units + 3) / 4;
    if (grid > kStepMaxGrid) grid = kStepMaxGrid;
    if (lds <= kStepLdsBytes)
        hipLaunchKernelGGL((k_step_t<KB, true>), dim3(grid), dim3(256), lds, stream, sp, cbar, abar, vids, gtab, B_eff,
                           nbb, n_units);
    else
        hipLaunchKernelGGL((k_step_t<KB, false>), dim3(grid), dim3(256), 0, stream, sp, cbar, abar, vids, gtab, B_eff,
                           nbb, n_units);
}

void launch_step_t(const StepParams& sp, const float2* cbar, float2* abar, const uint16_t* vids, const float2* gtab,
                   uint32_t B_eff, hipStream_t stream) {
    const size_t lds = size_t(8) * ((size_t(1) << (sp.vb + sp.sb)) * ((size_t(1) << (sp.kb + sp.nb)) + 1));
    switch (sp.kb) {
        case 0: launch_step_t_kb<0>(sp, cbar, abar, vids, gtab, B_eff, lds, stream); break;
        case 1: launch_step_t_kb<1>(sp, cbar, abar, vids, gtab, B_eff, lds, stream); break;
        case 2: launch_step_t_kb<2>(sp, cbar, abar, vids, gtab, B_eff, lds, stream); break;
        case 3: launch_step_t_kb<3>(sp, cbar, abar, vids, gtab, B_eff, lds, stream); break;
        case 4: launch_step_t_kb<4>(sp, cbar, abar, vids, gtab, B_eff, lds, stream); break;
        case 5: launch_step_t_kb<5>(sp, cbar, abar, vids, gtab, B_eff, lds, stream); break;
        default: launch_step_t_kb<6>(sp, cbar, abar, vids, gtab, B_eff, lds, stream); break;
    }
}

void launch_gbar(const GbarParams& gp, const float2* a, const float2* cbar, float2* part, const uint16_t* vids,
                 uint32_t B_eff, double2* gbar, hipStream_t stream) {
    const uint32_t units = uint32_t(gp.n_nc) * gp.n_kc * gp.n_rc * (1u << gp.sp.vb);
    hipLaunchKernelGGL(k_gbar, dim3((B_eff + 255) / 256, units), dim3(256), 0, stream, gp, a, cbar, part, B_eff);
    const uint32_t vkn = 1u << (gp.sp.vb + gp.sp.kb + gp.sp.nb);
    hipLaunchKernelGGL(k_gbar_reduce, dim3(vkn), dim3(256), 0, stream, gp, part, vids, B_eff, gbar);
}

void launch_gadj(const StepTab* steps, int n_steps, uint32_t max_entries, const GOp* ops, const double2* fixed,
                 const float2* slots, const double2* gbar, const int64_t* wave_base, double2* wpart, int max_ops,
                 hipStream_t stream) {
    hipLaunchKernelGGL(k_gadj, dim3((max_entries + 255) / 256, n_steps), dim3(256), 0, stream, steps, ops, fixed,
                       slots, gbar, wave_base, wpart, max_ops);
}

void launch_slot_grads(const int32_t* slot_ops_off, const int32_t* slot_ops, const int64_t* wave_base,
                       const int32_t* step_waves, const double2* wpart, int max_ops, int n_slots, float2* grads,
                       hipStream_t stream) {
    if (n_slots <= 0) return;
    hipLaunchKernelGGL(k_slot_grads, dim3((n_slots * 4 + 63) / 64), dim3(64), 0, stream, slot_ops_off, slot_ops,
                       wave_base, step_waves, wpart, max_ops, n_slots, grads);
}

void launch_seed(const float2* g, uint32_t B_eff, uint32_t B_pad, int64_t B, int n_open, const int32_t* final_pos,
                 float2* fbar, hipStream_t stream) {
    hipLaunchKernelGGL(k_seed, dim3((B_eff + 255) / 256, 1u << n_open), dim3(256), 0, stream, g, B_eff, B_pad, B,
                       n_open, final_pos, fbar);
}

}  // namespace qgm
