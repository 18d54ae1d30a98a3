// Adjoint of the bucket-elimination path (qgm_backward with ordering 1, gfx950).
//
// Holomorphic adjoints are propagated through the buckets in reverse level
// order.  For bucket s with result R[o] = sum_w G[c(o, w), sigma] prod_t T_t[idx_t(o, w)]
// and index space a = (o << k) | w:
//   T_t-bar[j] = sum_{a : idx_t(a) = j} R-bar[o(a)] G[c(a), sigma] prod_{t' != t} T_t'[idx_t'(a)]
//   G-bar[c][sigma] = sum_b [sigma(b) = sigma] sum_{a : c(a) = c} R-bar[o(a)] prod_t T_t[idx_t(a)]
// computed in two passes: an expansion over the whole index space (writing
// H = R-bar prod_t T_t and Q_t = R-bar G prod_{t' != t} T_t' per row a), then
// reductions over the a-bits that an input (or the table index) does not
// carry.  The table adjoints then flow through the factor groups to every gate
// factor (product rule; an absorbed bucket's group is a sum over its own
// variables), and the factors of each gate slot are summed into its gradient.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "tree_dev.hpp"

namespace qgm {

using namespace tree_dev;

namespace {

constexpr int kTbMaxGroups = 16;    // factor groups of one table (the planner keeps them below this)
constexpr int kTbGbarLds = 1 << kTreeMaxSig;

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// Sum of v over the 256 threads of a block, for 4 values per thread, in a
// fixed order (a butterfly within each wave, then the four waves in turn), so
// that the same inputs always give the same bits.  Every thread of the block
// must call it; the sums are valid in thread 0.  `red` is 16 double2 of LDS.
__device__ __forceinline__ void block_sum4(double2 (&v)[4], double2* red) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            v[a].x += __shfl_xor(v[a].x, m, 64);
            v[a].y += __shfl_xor(v[a].y, m, 64);
        }
    const int wave = int(threadIdx.x >> 6);
    if ((threadIdx.x & 63u) == 0)
#pragma unroll
        for (int a = 0; a < 4; ++a) red[wave * 4 + a] = v[a];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double2 s = red[a];
            for (int w = 1; w < 4; ++w) {
                s.x += red[w * 4 + a].x;
                s.y += red[w * 4 + a].y;
            }
            v[a] = s;
        }
    __syncthreads();
}

__device__ __forceinline__ bool slot_factor(const TFactor& f) {
    return (f.type == TF_MAT || f.type == TF_DIAG) && f.mat >= kFixedMats;
}

// Entry of an item list whose rows cover `row` (items sorted by row0).
__device__ __forceinline__ TreeBwdItem find_item(const TreeBwdItem* __restrict__ items, int n_items, int64_t row) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (int64_t(items[mid].row0) <= row) lo = mid;
        else hi = mid - 1;
    }
    return items[lo];
}

}  // namespace

// Seed: A = phase x prod of the rank-0 results (FP64), A-bar = conj(grad_amps);
// the adjoint of every rank-0 result, and the phase factors' share of the
// gate-slot gradients.  Padded bitstrings (b >= B) get zero adjoints.
__global__ void __launch_bounds__(256) k_tb_seed(const int64_t* __restrict__ final_rows, int n_final,
                                                 const TFactor* __restrict__ phase, int n_phase,
                                                 const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                                 const float2* __restrict__ arena, float2* __restrict__ adj,
                                                 const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                 const float2* __restrict__ grad_amps, void* __restrict__ amps_out,
                                                 int c128, double2* __restrict__ phibar_out) {
    const uint32_t b = blockIdx.x * 256u + threadIdx.x;
    if (b >= B_eff) return;
    const bool live = int64_t(b) < B;
    const uint64_t x = live ? bits[b] : 0ull;
    auto phase_value = [&](int i) {
        const TFactor f = phase[i];
        const uint32_t a = f.src0 == TS_SIG ? uint32_t((x >> f.bit0) & 1ull) : 0u;
        const uint32_t c = f.src1 == TS_SIG ? uint32_t((x >> f.bit1) & 1ull) : 0u;
        return factor_value(f, a, c, fixed, slots);
    };
    double2 phi = make_double2(1.0, 0.0);
    for (int i = 0; i < n_phase; ++i) phi = cmuld(phi, phase_value(i));
    double2 prod = make_double2(1.0, 0.0);
    for (int f = 0; f < n_final; ++f) {
        const float2 r = arena[final_rows[f] * int64_t(B_eff) + b];
        prod = cmuld(prod, make_double2(r.x, r.y));
    }
    const double2 amp = cmuld(phi, prod);
    if (live && amps_out) {
        if (c128) static_cast<double2*>(amps_out)[b] = amp;
        else static_cast<float2*>(amps_out)[b] = make_float2(float(amp.x), float(amp.y));
    }
    double2 abar = make_double2(0.0, 0.0);
    if (live) {
        const float2 g = grad_amps[b];
        abar = make_double2(g.x, -g.y);
    }
    for (int f = 0; f < n_final; ++f) {
        double2 v = cmuld(abar, phi);
        for (int f2 = 0; f2 < n_final; ++f2) {
            if (f2 == f) continue;
            const float2 r = arena[final_rows[f2] * int64_t(B_eff) + b];
            v = cmuld(v, make_double2(r.x, r.y));
        }
        adj[final_rows[f] * int64_t(B_eff) + b] = make_float2(float(v.x), float(v.y));
    }
    // the adjoint of the phase (zero for padded bitstrings), summed per phase factor by k_tb_phase_adj
    phibar_out[b] = cmuld(abar, prod);
}

// Adjoints of the phase factors that read gate slots: factor i receives
// phibar(b) * prod_{j != i} phase_j(b) at its entry (a, c) selected by the
// bits of bitstring b.  Block k sums the bitstrings b = k * 256 + tid +
// m * 256 * gridDim.x in increasing m per thread, then over the block in a
// fixed order, and writes its partial sums to fpart[part_off[f0 + i] + k].
__global__ void __launch_bounds__(256) k_tb_phase_adj(const TFactor* __restrict__ phase, int n_phase,
                                                      const double2* __restrict__ fixed,
                                                      const float2* __restrict__ slots,
                                                      const uint64_t* __restrict__ bits, int64_t B,
                                                      const double2* __restrict__ phibar,
                                                      const int64_t* __restrict__ part_off, int64_t f0,
                                                      double2* __restrict__ fpart) {
    __shared__ double2 red[16];
    for (int i = 0; i < n_phase; ++i) {
        const TFactor f = phase[i];
        if (!slot_factor(f)) continue;   // uniform over the block
        double2 acc[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a] = make_double2(0.0, 0.0);
        for (int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x; b < B; b += int64_t(gridDim.x) * 256) {
            const uint64_t x = bits[b];
            double2 v = phibar[b];
            for (int j = 0; j < n_phase; ++j) {
                if (j == i) continue;
                const TFactor g = phase[j];
                const uint32_t ga = g.src0 == TS_SIG ? uint32_t((x >> g.bit0) & 1ull) : 0u;
                const uint32_t gc = g.src1 == TS_SIG ? uint32_t((x >> g.bit1) & 1ull) : 0u;
                v = cmuld(v, factor_value(g, ga, gc, fixed, slots));
            }
            const uint32_t a = f.src0 == TS_SIG ? uint32_t((x >> f.bit0) & 1ull) : 0u;
            const uint32_t c = f.src1 == TS_SIG ? uint32_t((x >> f.bit1) & 1ull) : 0u;
            const uint32_t e = a * 2u + c;
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k)
                if (k == e) {
                    acc[k].x += v.x;
                    acc[k].y += v.y;
                }
        }
        block_sum4(acc, red);
        if (threadIdx.x == 0) {
            double2* dst = fpart + (part_off[f0 + i] + blockIdx.x) * 4;
#pragma unroll
            for (int a = 0; a < 4; ++a) dst[a] = acc[a];
        }
    }
}

// Expansion over a bucket's index space: wave unit u handles row a of one
// bucket of the level for 64 bitstrings, writing H[a] and every Q_t[a].
__global__ void __launch_bounds__(256) k_tb_expand(const TreeBwdItem* __restrict__ items, int n_items,
                                                   int64_t n_units, const TreeBwd* __restrict__ bwd,
                                                   const float2* __restrict__ arena, const float2* __restrict__ adj,
                                                   const float2* __restrict__ gtab, float2* __restrict__ scratch,
                                                   const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                   int write_h) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t be = int64_t(B_eff);
    const uint32_t n_bg = B_eff / 64u;
    for (int64_t u = int64_t(blockIdx.x) * 4 + wave; u < n_units; u += int64_t(gridDim.x) * 4) {
        const int64_t R = u / n_bg;
        const uint32_t bg = uint32_t(u - R * n_bg);
        const TreeBwdItem it = find_item(items, n_items, R);
        const TreeBwd* __restrict__ d = bwd + it.idx;
        const uint32_t a = uint32_t(R - it.row0);
        const uint32_t b = bg * 64u + lane;
        const uint64_t x = int64_t(b) < B ? bits[b] : 0ull;
        const int n_in = d->n_in;
        const uint32_t sig = gather_sigma(x, d->sig_q, d->sb);
        int64_t idx[kTreeMaxIn];
#pragma unroll
        for (int t = 0; t < kTreeMaxIn; ++t) idx[t] = t < n_in ? int64_t(d->in_row[t]) : 0;
        int64_t c = 0;
        for (uint32_t m = a; m; m &= m - 1u) {
            const int i = __builtin_ctz(m);
#pragma unroll
            for (int t = 0; t < kTreeMaxIn; ++t)
                if (t < n_in) idx[t] += d->in_str[t][i];
            c += d->g_str[i];
        }
        const float2 rb = adj[(int64_t(d->out_row) + (a >> d->k)) * be + b];
        const float2 gv = gtab[d->g_off + (c << d->sb) + sig];
        float2 T[kTreeMaxIn];
#pragma unroll
        for (int t = 0; t < kTreeMaxIn; ++t) T[t] = t < n_in ? arena[idx[t] * be + b] : make_float2(1.f, 0.f);
        const int64_t rows = int64_t(1) << d->a_bits;
        if (write_h) {
            float2 h = rb;
#pragma unroll
            for (int t = 0; t < kTreeMaxIn; ++t) h = cmulf(h, T[t]);
            scratch[(d->scratch_row + a) * be + b] = h;
        }
        const float2 base = cmulf(rb, gv);
#pragma unroll
        for (int t = 0; t < kTreeMaxIn; ++t) {
            if (t >= n_in) break;
            float2 q = base;
#pragma unroll
            for (int t2 = 0; t2 < kTreeMaxIn; ++t2)
                if (t2 != t) q = cmulf(q, T[t2]);
            scratch[(d->scratch_row + (1 + t) * rows + a) * be + b] = q;
        }
    }
}

// Staged sums (input adjoints, and H summed within each factor-table row):
// wave unit (output row j of one record, 64-bitstring group) adds the 2^n_sum
// source rows of its class, all loads issued before the first add.  A sum over
// more than kTbSumBits a-bits is split by the host into stages that pass partial
// rows between two partial areas.
template <int NS>
__device__ __forceinline__ float2 tb_sum_rows(const float2* __restrict__ src, const int32_t* __restrict__ foff,
                                              int64_t row0, int64_t be, uint32_t b) {
    float2 v[1 << NS];
#pragma unroll
    for (int f = 0; f < (1 << NS); ++f) v[f] = src[(row0 + foff[f]) * be + b];
#pragma unroll
    for (int w = (1 << NS) / 2; w >= 1; w /= 2)
#pragma unroll
        for (int f = 0; f < w; ++f) {
            v[f].x += v[f + w].x;
            v[f].y += v[f + w].y;
        }
    return v[0];
}

__global__ void __launch_bounds__(256) k_tb_reduce(const TreeBwdItem* __restrict__ items, int n_items, int64_t n_units,
                                                   const TreeBwdIn* __restrict__ bin, const float2* __restrict__ src,
                                                   float2* __restrict__ dst_adj, float2* __restrict__ dst_hsum,
                                                   float2* __restrict__ dst_part, uint32_t B_eff) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t be = int64_t(B_eff);
    const uint32_t n_bg = B_eff / 64u;
    for (int64_t u = int64_t(blockIdx.x) * 4 + wave; u < n_units; u += int64_t(gridDim.x) * 4) {
        const int64_t R = u / n_bg;
        const uint32_t bg = uint32_t(u - R * n_bg);
        const TreeBwdItem it = find_item(items, n_items, R);
        const TreeBwdIn* __restrict__ d = bin + it.idx;
        const uint32_t j = uint32_t(R - it.row0);
        const uint32_t b = bg * 64u + lane;
        int64_t a0 = 0;
        for (int p = 0; p < d->r_t; ++p) a0 |= int64_t((j >> p) & 1u) << d->pos[p];
        const int64_t row0 = d->q_row + a0;
        float2 s;
        switch (d->n_sum) {
            case 0: s = tb_sum_rows<0>(src, d->foff, row0, be, b); break;
            case 1: s = tb_sum_rows<1>(src, d->foff, row0, be, b); break;
            case 2: s = tb_sum_rows<2>(src, d->foff, row0, be, b); break;
            case 3: s = tb_sum_rows<3>(src, d->foff, row0, be, b); break;
            case 4: s = tb_sum_rows<4>(src, d->foff, row0, be, b); break;
            default: s = tb_sum_rows<5>(src, d->foff, row0, be, b); break;
        }
        float2* __restrict__ dst = d->dst_sel == 0 ? dst_adj : d->dst_sel == 1 ? dst_hsum : dst_part;
        dst[(int64_t(d->dst_row) + j) * be + b] = s;
    }
}

// Factor-table adjoint, second pass: block = one table row c; G-bar[c][s] is
// the sum of that row of H' (H summed over the rows of class c) over the
// bitstrings whose output bits give sigma = s.  Up to 8 values of sigma: each
// thread bins a strided share of the bitstrings in registers, then a fixed-order
// wave and block reduction (deterministic).
template <int NSIG>
__device__ void tb_gbin_small(const TreeBwdG* __restrict__ d, uint32_t c, const float2* __restrict__ hsum,
                              const uint64_t* __restrict__ bits, int64_t B, int64_t be, double2* __restrict__ gbar) {
    __shared__ double2 part[4][NSIG];
    double2 acc[NSIG];
#pragma unroll
    for (int s = 0; s < NSIG; ++s) acc[s] = make_double2(0.0, 0.0);
    const float2* __restrict__ h = hsum + (d->h_row + c) * be;
    for (int64_t b = threadIdx.x; b < B; b += 256) {
        const float2 v = h[b];
        const uint32_t sg = NSIG == 1 ? 0u : gather_sigma(bits[b], d->sig_q, d->sb);
#pragma unroll
        for (int s = 0; s < NSIG; ++s)
            if (sg == uint32_t(s)) {
                acc[s].x += v.x;
                acc[s].y += v.y;
            }
    }
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NSIG; ++s) {
        double x = acc[s].x, y = acc[s].y;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            x += __shfl_xor(x, o);
            y += __shfl_xor(y, o);
        }
        if (lane == 0) part[wave][s] = make_double2(x, y);
    }
    __syncthreads();
    if (threadIdx.x < NSIG) {
        double2 t = part[0][threadIdx.x];
        for (int w = 1; w < 4; ++w) {
            t.x += part[w][threadIdx.x].x;
            t.y += part[w][threadIdx.x].y;
        }
        gbar[d->g_off + (int64_t(c) << d->sb) + threadIdx.x] = t;
    }
}

// More than 8 values of sigma: the row of H' is staged in LDS with each
// bitstring's sigma; thread s sums the entries with sigma(b) = s.
__device__ void tb_gbin_wide(const TreeBwdG* __restrict__ d, uint32_t c, const float2* __restrict__ hsum,
                             const uint64_t* __restrict__ bits, int64_t B, int64_t be, double2* __restrict__ gbar) {
    constexpr int CH = 1024;   // bitstrings staged per round
    __shared__ float2 hv[CH];
    __shared__ uint16_t sv[CH];
    const int sb = d->sb;
    const int n_sig = 1 << sb;
    double2 acc[kTbGbarLds / 256];
#pragma unroll
    for (int i = 0; i < kTbGbarLds / 256; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int64_t b0 = 0; b0 < B; b0 += CH) {
        const int nb = int(std::min<int64_t>(CH, B - b0));
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += 256) {
            hv[i] = hsum[(d->h_row + c) * be + b0 + i];
            sv[i] = uint16_t(gather_sigma(bits[b0 + i], d->sig_q, sb));
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTbGbarLds / 256; ++r) {
            const int sg = threadIdx.x + r * 256;
            if (sg >= n_sig) break;
            double2 a = acc[r];
            for (int i = 0; i < nb; ++i)
                if (sv[i] == sg) {
                    a.x += hv[i].x;
                    a.y += hv[i].y;
                }
            acc[r] = a;
        }
    }
#pragma unroll
    for (int r = 0; r < kTbGbarLds / 256; ++r) {
        const int sg = threadIdx.x + r * 256;
        if (sg < n_sig) gbar[d->g_off + (int64_t(c) << sb) + sg] = acc[r];
    }
}

__global__ void __launch_bounds__(256) k_tb_gbin(const TreeBwdItem* __restrict__ items, int n_items,
                                                 const TreeBwdG* __restrict__ bgd, const float2* __restrict__ hsum,
                                                 const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                 double2* __restrict__ gbar) {
    const TreeBwdItem it = find_item(items, n_items, blockIdx.x);
    const TreeBwdG* __restrict__ d = bgd + it.idx;
    const uint32_t c = uint32_t(int64_t(blockIdx.x) - it.row0);
    const int64_t be = int64_t(B_eff);
    switch (d->sb) {
        case 0: tb_gbin_small<1>(d, c, hsum, bits, B, be, gbar); break;
        case 1: tb_gbin_small<2>(d, c, hsum, bits, B, be, gbar); break;
        case 2: tb_gbin_small<4>(d, c, hsum, bits, B, be, gbar); break;
        case 3: tb_gbin_small<8>(d, c, hsum, bits, B, be, gbar); break;
        default: tb_gbin_wide(d, c, hsum, bits, B, be, gbar); break;
    }
}

// Factor adjoints from the table adjoints: per table entry e (blocks as in
// the factor-table build), for every group q and value iv of its own
// variables, each gate-slot factor f of q receives
//   G-bar[e] * prod_{q' != q} S_q' * prod_{f' in q, f' != f} f'
// at the entry of its table that (c, sigma, iv) selects.  Each block sums its
// 256 entries' shares per factor in a fixed order (block_sum4) and writes
// them to fpart[part_off[f] + sub]; k_tb_fsum adds the blocks of a factor in
// order, so the result does not depend on scheduling.  Block (x, y) handles
// the y-th of every kTbGadjParts slot factors of its table.
__global__ void __launch_bounds__(256) k_tb_gadj(const TreeProBlock* __restrict__ blocks,
                                                 const TreeGTab* __restrict__ gtabs,
                                                 const TreeGroup* __restrict__ groups,
                                                 const TFactor* __restrict__ facs, const double2* __restrict__ fixed,
                                                 const float2* __restrict__ slots, const double2* __restrict__ gbar,
                                                 const int64_t* __restrict__ part_off, double2* __restrict__ fpart) {
    __shared__ FactorLds L;
    __shared__ double2 red[16];
    const TreeProBlock blk = blocks[blockIdx.x];
    const TreeGTab t = gtabs[blk.idx];
    const TreeGroup* __restrict__ gr = groups + t.group_off;
    const int fac0 = gr[0].fac_off;
    const TFactor* __restrict__ tf = facs + fac0;
    const int nf = stage_factors(L, tf, t.n_fac, fixed, slots);   // ends with a block barrier
    const int part = int(blockIdx.y), n_parts = int(gridDim.y);
    const int64_t e = int64_t(blk.sub) * 256 + threadIdx.x;
    const bool valid = e < (int64_t(1) << (t.gb + t.k + t.sb));
    const double2 gb = valid ? gbar[t.g_off + e] : make_double2(0.0, 0.0);
    const uint32_t sig = valid ? uint32_t(e) & ((1u << t.sb) - 1u) : 0u;
    const uint32_t c = valid ? uint32_t(e) >> t.sb : 0u;
    double2 S[kTbMaxGroups];
#pragma unroll
    for (int q = 0; q < kTbMaxGroups; ++q) {
        S[q] = make_double2(1.0, 0.0);
        if (q < t.n_groups) {
            const TreeGroup g = gr[q];
            const int f0 = g.fac_off - fac0, f1 = f0 + g.n_fac;
            double2 sum = make_double2(0.0, 0.0);
            for (uint32_t iv = 0; iv < (1u << g.k_int); ++iv) {
                const double2 v = factor_product(L, nf, tf, f0, f1, fixed, slots, c, sig, iv);
                sum.x += v.x;
                sum.y += v.y;
            }
            S[q] = sum;
        }
    }
    auto val = [&](int32_t src, int32_t bit, uint32_t iv) -> uint32_t {
        switch (src) {
            case TS_G: return (c >> bit) & 1u;
            case TS_SIG: return (sig >> bit) & 1u;
            case TS_INT: return (iv >> bit) & 1u;
            default: return 0u;
        }
    };
    int n_seen = 0;   // slot factors met so far (uniform over the block)
    for (int q = 0; q < t.n_groups; ++q) {
        double2 pq = gb;
#pragma unroll
        for (int q2 = 0; q2 < kTbMaxGroups; ++q2)
            if (q2 != q && q2 < t.n_groups) pq = cmuld(pq, S[q2]);
        const TreeGroup g = gr[q];
        const int f0 = g.fac_off - fac0, f1 = f0 + g.n_fac;
        for (int i = f0; i < f1; ++i) {
            const TFactor f = tf[i];
            if (!slot_factor(f)) continue;
            if (n_seen++ % n_parts != part) continue;
            double2 acc[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] = make_double2(0.0, 0.0);
            if (valid && (gb.x != 0.0 || gb.y != 0.0)) {
                for (uint32_t iv = 0; iv < (1u << g.k_int); ++iv) {
                    double2 v = pq;
                    for (int i2 = f0; i2 < f1; ++i2)
                        if (i2 != i) v = cmuld(v, factor_product(L, nf, tf, i2, i2 + 1, fixed, slots, c, sig, iv));
                    const uint32_t args = val(f.src0, f.bit0, iv) * 2u + val(f.src1, f.bit1, iv);
#pragma unroll
                    for (uint32_t k = 0; k < 4; ++k)
                        if (k == args) {
                            acc[k].x += v.x;
                            acc[k].y += v.y;
                        }
                }
            }
            block_sum4(acc, red);
            if (threadIdx.x == 0) {
                double2* dst = fpart + (part_off[fac0 + i] + blk.sub) * 4;
#pragma unroll
                for (int a = 0; a < 4; ++a) dst[a] = acc[a];
            }
        }
    }
}

// fbar[f][a] = sum over the partial sums of factor f in order (zero for a
// factor that reads no gate slot: it has none).
__global__ void __launch_bounds__(256) k_tb_fsum(const int64_t* __restrict__ part_off, int64_t n_fbar,
                                                 const double2* __restrict__ fpart, double2* __restrict__ fbar) {
    const int64_t id = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (id >= n_fbar * 4) return;
    const int64_t f = id >> 2;
    const int a = int(id & 3);
    double2 s = make_double2(0.0, 0.0);
    for (int64_t k = part_off[f]; k < part_off[f + 1]; ++k) {
        s.x += fpart[k * 4 + a].x;
        s.y += fpart[k * 4 + a].y;
    }
    fbar[id] = s;
}

// Gradient of every gate slot: the sum of its factors' adjoints (a diagonal
// gate's factor value at (a, c) is the slot entry (a, a)), conjugated for the
// torch convention.
__global__ void __launch_bounds__(256) k_tb_slots(const int32_t* __restrict__ slot_off,
                                                  const int32_t* __restrict__ slot_occ, int n_slots,
                                                  const double2* __restrict__ fbar, float2* __restrict__ grads) {
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= n_slots * 4) return;
    const int s = id >> 2, el = id & 3;
    const int ra = el >> 1, rc = el & 1;
    double2 acc = make_double2(0.0, 0.0);
    for (int o = slot_off[s]; o < slot_off[s + 1]; ++o) {
        const int32_t occ = slot_occ[o];
        const double2* fb = fbar + size_t(occ >> 1) * 4;
        if (occ & 1) {   // diagonal gate: entries (a, 0) and (a, 1) of the factor both hold M[a][a]
            if (ra == rc) {
                acc.x += fb[ra * 2].x + fb[ra * 2 + 1].x;
                acc.y += fb[ra * 2].y + fb[ra * 2 + 1].y;
            }
        } else {
            acc.x += fb[el].x;
            acc.y += fb[el].y;
        }
    }
    grads[id] = conjf2(make_float2(float(acc.x), float(acc.y)));
}

void launch_tb_seed(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                    const float2* slots, const float2* arena, float2* adj, const uint64_t* bits, int64_t B,
                    uint32_t B_eff, const float2* grad_amps, void* amps_out, bool c128, double2* phibar,
                    hipStream_t stream) {
    hipLaunchKernelGGL(k_tb_seed, dim3((B_eff + 255) / 256), dim3(256), 0, stream, final_rows, n_final, phase, n_phase,
                       fixed, slots, arena, adj, bits, B, B_eff, grad_amps, amps_out, c128 ? 1 : 0, phibar);
}

void launch_tb_phase_adj(const TFactor* phase, int n_phase, const double2* fixed, const float2* slots,
                         const uint64_t* bits, int64_t B, const double2* phibar, const int64_t* part_off, int64_t f0,
                         double2* fpart, hipStream_t stream) {
    if (n_phase <= 0 || B <= 0) return;
    hipLaunchKernelGGL(k_tb_phase_adj, dim3(kTbPhaseBlocks), dim3(256), 0, stream, phase, n_phase, fixed, slots, bits,
                       B, phibar, part_off, f0, fpart);
}

void launch_tb_fsum(const int64_t* part_off, int64_t n_fbar, const double2* fpart, double2* fbar,
                    hipStream_t stream) {
    if (n_fbar <= 0) return;
    hipLaunchKernelGGL(k_tb_fsum, dim3(uint32_t((n_fbar * 4 + 255) / 256)), dim3(256), 0, stream, part_off, n_fbar,
                       fpart, fbar);
}

void launch_tb_expand(const TreeBwdItem* items, int n_items, int64_t total_rows, const TreeBwd* bwd,
                      const float2* arena, const float2* adj, const float2* gtab, float2* scratch,
                      const uint64_t* bits, int64_t B, uint32_t B_eff, bool write_h, hipStream_t stream) {
    const int64_t n_units = total_rows * (B_eff / 64u);
    if (n_units <= 0) return;
    const uint32_t grid = uint32_t(std::min<int64_t>((n_units + 3) / 4, kStepMaxGrid));
    hipLaunchKernelGGL(k_tb_expand, dim3(grid), dim3(256), 0, stream, items, n_items, n_units, bwd, arena, adj, gtab,
                       scratch, bits, B, B_eff, write_h ? 1 : 0);
}

void launch_tb_reduce(const TreeBwdItem* items, int n_items, int64_t total_rows, const TreeBwdIn* bin,
                      const float2* src, float2* dst_adj, float2* dst_hsum, float2* dst_part, uint32_t B_eff,
                      hipStream_t stream) {
    const int64_t n_units = total_rows * (B_eff / 64u);
    if (n_units <= 0) return;
    const uint32_t grid = uint32_t(std::min<int64_t>((n_units + 3) / 4, kStepMaxGrid));
    hipLaunchKernelGGL(k_tb_reduce, dim3(grid), dim3(256), 0, stream, items, n_items, n_units, bin, src, dst_adj,
                       dst_hsum, dst_part, B_eff);
}

void launch_tb_gbin(const TreeBwdItem* items, int n_items, int64_t total_rows, const TreeBwdG* bg, const float2* hsum,
                    const uint64_t* bits, int64_t B, uint32_t B_eff, double2* gbar, hipStream_t stream) {
    if (total_rows <= 0) return;
    hipLaunchKernelGGL(k_tb_gbin, dim3(uint32_t(total_rows)), dim3(256), 0, stream, items, n_items, bg, hsum, bits, B,
                       B_eff, gbar);
}

void launch_tb_gadj(const TreeProBlock* blocks, int n_blocks, const TreeGTab* gtabs, const TreeGroup* groups,
                    const TFactor* facs, const double2* fixed, const float2* slots, const double2* gbar,
                    const int64_t* part_off, double2* fpart, hipStream_t stream) {
    if (n_blocks <= 0) return;
    hipLaunchKernelGGL(k_tb_gadj, dim3(uint32_t(n_blocks), kTbGadjParts), dim3(256), 0, stream, blocks, gtabs, groups,
                       facs, fixed, slots, gbar, part_off, fpart);
}

void launch_tb_slots(const int32_t* slot_off, const int32_t* slot_occ, int n_slots, const double2* fbar,
                     float2* grads, hipStream_t stream) {
    if (n_slots <= 0) return;
    hipLaunchKernelGGL(k_tb_slots, dim3((n_slots * 4 + 255) / 256), dim3(256), 0, stream, slot_off, slot_occ, n_slots,
                       fbar, grads);
}

}  // namespace qgm
