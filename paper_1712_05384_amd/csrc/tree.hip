// Device kernels of the bucket-elimination path (ordering 1, gfx950).
//
// Every bucket result is a batch-minor [2^r][B_eff] complex64 array in one
// arena: element (o, b) lives at (row + o) * B_eff + b, B_eff being the batch
// padded to a power of two (rows are scaled by a shift), so a wave that owns 64
// consecutive bitstrings reads and writes 512 contiguous bytes per tensor row
// whatever the bucket's axes.  The index arithmetic of a bucket (which input
// row belongs to result row o and value v of the summed variable) depends on
// o only, so it runs on the scalar unit; only the data and the per-bitstring
// factor variant sigma are per lane.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "tree_dev.hpp"

namespace qgm {

using namespace tree_dev;

// Factor tables (one launch; block i does 256 entries of table blocks[i].idx;
// block 0 also writes the constant 1): entry e = (c << sb) | sigma with
// c = (g << k) | w is the product over the bucket's factor groups (its own
// gate factors, Sec. III.B; then each absorbed bucket's factors summed over
// that bucket's variables) for those variable values, in FP64 rounded once to
// complex64.  A plan whose circuit reads no gate values runs this once, into
// its own device tables; otherwise every call runs it into the workspace.
__global__ void __launch_bounds__(256) k_tree_prologue(const TreeProBlock* __restrict__ blocks,
                                                       const TreeGTab* __restrict__ gtabs,
                                                       const TreeGroup* __restrict__ groups,
                                                       const TFactor* __restrict__ facs,
                                                       const double2* __restrict__ fixed,
                                                       const float2* __restrict__ slots, float2* __restrict__ gtab,
                                                       int64_t ones_g, const TFactor* __restrict__ phase, int n_phase,
                                                       int64_t phase_g) {
    __shared__ FactorLds L;
    if (blockIdx.x == 0 && threadIdx.x == 0) gtab[ones_g] = make_float2(1.f, 0.f);
    const TreeProBlock blk = blocks[blockIdx.x];
    if (blk.idx < 0) {   // phase factor i, entry 2a + c: its FP64 value (two-qubit factors: from the record)
        const int i = blk.sub * 256 + int(threadIdx.x);
        if (i >= 4 * n_phase) return;
        const TFactor f = phase[i >> 2];
        const double2 v = f.type == TF_MAT4 ? make_double2(0.0, 0.0)
                                            : factor_value(f, uint32_t(i >> 1) & 1u, uint32_t(i) & 1u, fixed, slots);
        reinterpret_cast<double2*>(gtab + phase_g)[i] = v;
        return;
    }
    const TreeGTab t = gtabs[blk.idx];
    const TreeGroup* __restrict__ gr = groups + t.group_off;
    const TFactor* __restrict__ tf = facs + gr[0].fac_off;   // the groups' factors are contiguous
    const int nf = stage_factors(L, tf, t.n_fac, fixed, slots);
    const int64_t e = int64_t(blk.sub) * 256 + threadIdx.x;
    if (e >= (int64_t(1) << (t.gb + t.k + t.sb))) return;
    const uint32_t sig = uint32_t(e) & ((1u << t.sb) - 1u);
    const uint32_t c = uint32_t(e) >> t.sb;
    double2 acc = make_double2(1.0, 0.0);
    for (int q = 0; q < t.n_groups; ++q) {
        const TreeGroup g = gr[q];
        const int f0 = g.fac_off - gr[0].fac_off, f1 = f0 + g.n_fac;
        double2 sum = make_double2(0.0, 0.0);
        for (uint32_t iv = 0; iv < (1u << g.k_int); ++iv) {
            const double2 v = factor_product(L, nf, tf, f0, f1, fixed, slots, c, sig, iv);
            sum.x += v.x;
            sum.y += v.y;
        }
        acc = cmuld(acc, sum);
    }
    gtab[t.g_off + e] = make_float2(float(acc.x), float(acc.y));
}

// What the tail kernel keeps in LDS for its work-group's 64 bitstrings: the
// results made in the tail (row r of lane l at rows[r * 64 + l]), the tail's
// factor tables and the constant 1.
struct TailView {
    float2* rows;
    const float2* g;      // the tail's factor tables (g_ent of a tail task counts from here)
    const float2* one;
};

// Where input t's row r lives for this lane: base + (r << sh) (a result in the
// arena: column b, rows B_eff apart, a power of two; a leaf table: its entries
// for the lane's output bits, rows 2^sb apart; a result kept in the tail's LDS:
// rows 64 apart; an input the bucket does not have: the constant 1 at row 0,
// whose row steps are all 0).
template <bool TL>
__device__ __forceinline__ void input_view(const TreeTask& tk, int t, const float2* __restrict__ ain,
                                           const float2* __restrict__ gtab, int64_t ones_g, uint64_t x, uint32_t b,
                                           uint32_t be_sh, const TailView& tv, const float2*& base, uint32_t& sh) {
    if (tk.in_row[t] < 0) {
        base = TL ? tv.one : gtab + ones_g;
        sh = 0;
    } else if (TL && tk.in_tab[t] == -2) {
        base = tv.rows + (b & 63u);
        sh = 6;
    } else if (tk.in_tab[t] >= 0) {
        const int tsb = tk.in_tsb[t];
        const uint64_t pk = uint64_t(tk.in_tsig[t]);
        uint32_t s = 0;
        for (int i = 0; i < tsb; ++i) s |= uint32_t((x >> ((pk >> (6 * i)) & 63u)) & 1ull) << i;
        base = gtab + tk.in_tab[t] + s;
        sh = uint32_t(tsb);
    } else {
        base = ain + b;
        sh = be_sh;
    }
}

// One wave unit of a bucket with inputs: the task's rows for the 64
// bitstrings b of one group,
//   R[o][b] = sum_{w < 2^K} G[g(o), w, sigma(b)] * prod_t T_t[idx_t(o) + off_t(w)][b],
// w running over the values of the bucket's K summed variables (one, or up to
// three for a merged chain).  No data-dependent branch: a bucket with fewer
// inputs than NIN multiplies a constant 1 (one address for all lanes, chosen
// per wave), and the task of a result with fewer rows than a unit wraps onto
// valid rows and stores into rows the arena reserves for it.  Inputs (ain) and
// results (aout) are views of one arena whose rows a level never both reads and
// writes, so all loads of a unit can be in flight at once.  In the tail kernel
// (TL) an input or the result may instead be rows kept in LDS (TailView).
template <int NIN, int K, bool TL>
__device__ __forceinline__ void tree_unit(const TreeTask& tk, const float2* __restrict__ ain,
                                          float2* __restrict__ aout, const float2* __restrict__ gtab, int64_t ones_g,
                                          int64_t sig, uint64_t x, uint32_t b, int64_t be, const TailView& tv) {
    constexpr int W = 1 << K;
    constexpr int WC = W < 8 ? W : 8;          // summed-variable values per load batch
    static_assert(WC == W, "one load batch holds every summed value (the repeat copies index within it)");
    constexpr int OB = tree_unit_rows(NIN, K);
    // Input t's row r for this lane is base[t] + (r << sh[t]) (input_view).  Rows
    // (32-bit), the factor-table entry of the unit's rows and the row offset of
    // each summed value w in each input are scalar; a power-of-two row pitch
    // makes the row scaling one shift instead of a 64-bit multiply per load.
    const uint32_t be_sh = uint32_t(__builtin_ctzll(uint64_t(be)));
    const float2* base[NIN];
    uint32_t sh[NIN];
#pragma unroll
    for (int t = 0; t < NIN; ++t) input_view<TL>(tk, t, ain, gtab, ones_g, x, b, be_sh, tv, base[t], sh[t]);
    int32_t row[OB][NIN], off[NIN][W];
    int64_t gent[OB];
#pragma unroll
    for (int t = 0; t < NIN; ++t) {
        row[0][t] = tk.in_row[t] < 0 ? 0 : tk.in_row[t];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            int32_t o = 0;
#pragma unroll
            for (int i = 0; i < K; ++i)
                if ((w >> i) & 1) o += tk.in_vs[t][i];
            off[t][w] = o;
        }
    }
    gent[0] = tk.g_ent;
#pragma unroll
    for (int oi = 1; oi < OB; ++oi) {
        const int j = __builtin_ctz(uint32_t(oi));
#pragma unroll
        for (int t = 0; t < NIN; ++t) row[oi][t] = row[oi - 1][t] + tk.in_inc[t][j];
        gent[oi] = gent[oi - 1] + (int64_t(tk.g_inc[j]) << tk.gshift);
    }
    // An entry repeats an earlier one when the input (or the table) does not vary
    // along the bit that distinguishes them: row i repeats row i - lowbit(i) if
    // input t's stride along result bit ctz(i) is 0, and summed value w repeats
    // w - lowbit(w) if t does not carry summed variable ctz(w).  The repeats
    // (uniform, per task) are not loaded: all other loads are issued first,
    // then the repeats are copied in registers.
    uint32_t in_om[NIN], in_wm[NIN];
#pragma unroll
    for (int t = 0; t < NIN; ++t) {
        in_om[t] = uint32_t(tk.in_omask[t]);
        uint32_t wm = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (tk.in_vs[t][i] != 0) wm |= 1u << i;
        in_wm[t] = wm;
    }
    const uint32_t g_om = uint32_t(tk.g_omask);
    // which entries (i, t, w) are loaded: bit w of lm[i][t] (all repeats cleared),
    // one mask per row and input, read through an empty asm so that each load
    // tests one bit instead of the compiler re-deriving both conditions per load
    uint32_t lm[OB][NIN];
#pragma unroll
    for (int t = 0; t < NIN; ++t) {
        uint32_t wl = 1u;
#pragma unroll
        for (int w = 1; w < W; ++w)
            if ((in_wm[t] >> __builtin_ctz(uint32_t(w))) & 1u) wl |= 1u << w;
#pragma unroll
        for (int i = 0; i < OB; ++i) {
            const bool rep_i = i > 0 && !((in_om[t] >> __builtin_ctz(uint32_t(i))) & 1u);
            lm[i][t] = __builtin_amdgcn_readfirstlane(rep_i ? 0u : wl);
            asm volatile("" : "+s"(lm[i][t]));
        }
    }
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
#pragma unroll
                for (int w = 0; w < WC; ++w) {
                    const int wa = w0 + w;
                    if ((lm[i][t] >> wa) & 1u)
                        a[i][t][w] = base[t][int64_t(uint32_t(row[i][t] + off[t][wa])) << sh[t]];
                }
            }
#pragma unroll
        for (int i = 0; i < OB; ++i) {
            const bool rep_i = i > 0 && !((g_om >> __builtin_ctz(uint32_t(i))) & 1u);
            if (!rep_i) {
#pragma unroll
                for (int w = 0; w < WC; ++w) q[i][w] = (TL ? tv.g : gtab)[gent[i] + (int64_t(w0 + w) << tk.sb) + sig];
            }
        }
        // the repeats, in ascending order (each copies an entry already final).  The
        // masks are re-read through an empty asm so that the compiler cannot fold a
        // copy into the load it replaces (which would wait on each load in turn)
        uint32_t om2[NIN], wm2[NIN];
        uint32_t g_om2 = __builtin_amdgcn_readfirstlane(g_om);   // uniform per task
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            om2[t] = __builtin_amdgcn_readfirstlane(in_om[t]);
            wm2[t] = __builtin_amdgcn_readfirstlane(in_wm[t]);
            asm volatile("" : "+s"(om2[t]), "+s"(wm2[t]));
        }
        asm volatile("" : "+s"(g_om2));
#pragma unroll
        for (int i = 0; i < OB; ++i) {
#pragma unroll
            for (int t = 0; t < NIN; ++t) {
                const bool rep_i = i > 0 && !((om2[t] >> __builtin_ctz(uint32_t(i))) & 1u);
#pragma unroll
                for (int w = 0; w < WC; ++w) {
                    const int wa = w0 + w;
                    const bool rep_w = w > 0 && !((wm2[t] >> __builtin_ctz(uint32_t(wa))) & 1u);
                    if (rep_i) a[i][t][w] = a[i > 0 ? i - (i & -i) : 0][t][w];
                    else if (rep_w) a[i][t][w] = a[i][t][w > 0 ? w - (wa & -wa) : 0];
                }
            }
            const bool rep_g = i > 0 && !((g_om2 >> __builtin_ctz(uint32_t(i))) & 1u);
            if (rep_g) {
#pragma unroll
                for (int w = 0; w < WC; ++w) q[i][w] = q[i > 0 ? i - (i & -i) : 0][w];
            }
        }
#pragma unroll
        for (int i = 0; i < OB; ++i)
#pragma unroll
            for (int w = 0; w < WC; ++w) {
                float2 pw = q[i][w];
#pragma unroll
                for (int t = 0; t + 1 < NIN; ++t) pw = cmulf(pw, a[i][t][w]);
                // the last factor goes straight into the sum: four fused multiply-adds
                const float2 l = a[i][NIN - 1][w];
                acc[i].x = fmaf(pw.x, l.x, acc[i].x);
                acc[i].x = fmaf(-pw.y, l.y, acc[i].x);
                acc[i].y = fmaf(pw.x, l.y, acc[i].y);
                acc[i].y = fmaf(pw.y, l.x, acc[i].y);
            }
    }
    if (TL) {
        float2* out = tv.rows + int64_t(tk.out_row) * 64 + (b & 63u);
#pragma unroll
        for (int i = 0; i < OB; ++i) out[i * 64] = acc[i];
        return;
    }
    float2* __restrict__ out = aout + int64_t(tk.out_row) * be + b;
#pragma unroll
    for (int i = 0; i < OB; ++i) out[int64_t(i) * be] = acc[i];
}

// A tile unit: a bucket whose unit bits 0 and 1 vary only input 0 (A), bit 2
// only input 1 (B), and neither a third input C (NC) nor the factor table:
//   R[i + 4 j] = sum_w G[w, sigma] C[w] A[i][w] B[j][w]   (i < 4, j < 2),
// with A, B the rows of inputs 0, 1 at those unit rows and summed value w.  It
// loads 4 + 2 (+ 1) input rows and one table row per w for 8 result rows (the
// general unit would hold every (row, input, w) entry and cover 2-4 rows).
template <int K, bool TL, bool NC>
__device__ __forceinline__ void tile_unit(const TreeTask& tk, const float2* __restrict__ ain,
                                          float2* __restrict__ aout, const float2* __restrict__ gtab, int64_t ones_g,
                                          int64_t sig, uint64_t x, uint32_t b, int64_t be, const TailView& tv) {
    constexpr int W = 1 << K;
    const uint32_t be_sh = uint32_t(__builtin_ctzll(uint64_t(be)));
    const float2 *base_a, *base_b, *base_c = nullptr;
    uint32_t sh_a, sh_b, sh_c = 0;
    input_view<TL>(tk, 0, ain, gtab, ones_g, x, b, be_sh, tv, base_a, sh_a);
    input_view<TL>(tk, 1, ain, gtab, ones_g, x, b, be_sh, tv, base_b, sh_b);
    if (NC) input_view<TL>(tk, 2, ain, gtab, ones_g, x, b, be_sh, tv, base_c, sh_c);
    // unit row o = o-1 + increment of bit ctz(o): rows 0..3 of A, rows 0 and 4 of B
    int32_t ra[4], rb[2];
    ra[0] = tk.in_row[0];
    ra[1] = ra[0] + tk.in_inc[0][0];
    ra[2] = ra[1] + tk.in_inc[0][1];
    ra[3] = ra[2] + tk.in_inc[0][0];
    rb[0] = tk.in_row[1];
    rb[1] = rb[0] + 2 * tk.in_inc[1][0] + tk.in_inc[1][1] + tk.in_inc[1][2];
    const int32_t rc = NC ? tk.in_row[2] : 0;
    int32_t oa[W], ob[W], oc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        oa[w] = ob[w] = oc[w] = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((w >> i) & 1) {
                oa[w] += tk.in_vs[0][i];
                ob[w] += tk.in_vs[1][i];
                if (NC) oc[w] += tk.in_vs[2][i];
            }
    }
    float2 A[4][W], Bv[2][W], Q[W], Cv[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
#pragma unroll
        for (int i = 0; i < 4; ++i) A[i][w] = base_a[int64_t(uint32_t(ra[i] + oa[w])) << sh_a];
#pragma unroll
        for (int j = 0; j < 2; ++j) Bv[j][w] = base_b[int64_t(uint32_t(rb[j] + ob[w])) << sh_b];
        if (NC) Cv[w] = base_c[int64_t(uint32_t(rc + oc[w])) << sh_c];
        Q[w] = (TL ? tv.g : gtab)[tk.g_ent + (int64_t(w) << tk.sb) + sig];
    }
    if (NC) {
#pragma unroll
        for (int w = 0; w < W; ++w) Q[w] = cmulf(Q[w], Cv[w]);
    }
    float2 acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = make_float2(0.f, 0.f);
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float2 qa = cmulf(Q[w], A[i][w]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const float2 l = Bv[j][w];
                float2& c = acc[i + 4 * j];
                c.x = fmaf(qa.x, l.x, c.x);
                c.x = fmaf(-qa.y, l.y, c.x);
                c.y = fmaf(qa.x, l.y, c.y);
                c.y = fmaf(qa.y, l.x, c.y);
            }
        }
    if (TL) {
        float2* out = tv.rows + int64_t(tk.out_row) * 64 + (b & 63u);
#pragma unroll
        for (int o = 0; o < 8; ++o) out[o * 64] = acc[o];
        return;
    }
    float2* __restrict__ out = aout + int64_t(tk.out_row) * be + b;
#pragma unroll
    for (int o = 0; o < 8; ++o) out[int64_t(o) * be] = acc[o];
}

// A large tile unit (tile 3: two inputs; 4: a third input C): 32 result rows,
// unit bits 0, 1, 3 varying input A only (8 rows of A) and bits 2, 4 input B
// only (4 rows of B), none of them input C or the factor table.  The summed
// values are streamed: per value w one table entry, 8 rows of A, 4 of B (and
// 1 of C) are loaded and the 32 results accumulated, so each loaded row serves
// 4 or 8 results (the 8-row tile loads 7 rows per 8 result rows and value,
// this one 13 per 32).  The task's in_inc[0][0..2] and in_inc[1][0..1] hold
// the row strides of those bits in A and B.
template <int K, bool TL, bool NC>
__device__ __forceinline__ void tile32_unit(const TreeTask& tk, const float2* __restrict__ ain,
                                            float2* __restrict__ aout, const float2* __restrict__ gtab,
                                            int64_t ones_g, int64_t sig, uint64_t x, uint32_t b, int64_t be,
                                            const TailView& tv) {
    constexpr int W = 1 << K;
    const uint32_t be_sh = uint32_t(__builtin_ctzll(uint64_t(be)));
    const float2 *base_a, *base_b, *base_c = nullptr;
    uint32_t sh_a, sh_b, sh_c = 0;
    input_view<TL>(tk, 0, ain, gtab, ones_g, x, b, be_sh, tv, base_a, sh_a);
    input_view<TL>(tk, 1, ain, gtab, ones_g, x, b, be_sh, tv, base_b, sh_b);
    if (NC) input_view<TL>(tk, 2, ain, gtab, ones_g, x, b, be_sh, tv, base_c, sh_c);
    int32_t ra[8], rb[4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
        ra[i] = tk.in_row[0] + ((i & 1) ? tk.in_inc[0][0] : 0) + ((i & 2) ? tk.in_inc[0][1] : 0) +
                ((i & 4) ? tk.in_inc[0][2] : 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) rb[j] = tk.in_row[1] + ((j & 1) ? tk.in_inc[1][0] : 0) + ((j & 2) ? tk.in_inc[1][1] : 0);
    float2 acc[32];
#pragma unroll
    for (int o = 0; o < 32; ++o) acc[o] = make_float2(0.f, 0.f);
#pragma unroll 2
    for (int w = 0; w < W; ++w) {
        int32_t oa = 0, ob = 0, oc = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((w >> i) & 1) {
                oa += tk.in_vs[0][i];
                ob += tk.in_vs[1][i];
                if (NC) oc += tk.in_vs[2][i];
            }
        float2 q = (TL ? tv.g : gtab)[tk.g_ent + (int64_t(w) << tk.sb) + sig];
        float2 A[8], Bv[4];
#pragma unroll
        for (int i = 0; i < 8; ++i) A[i] = base_a[int64_t(uint32_t(ra[i] + oa)) << sh_a];
#pragma unroll
        for (int j = 0; j < 4; ++j) Bv[j] = base_b[int64_t(uint32_t(rb[j] + ob)) << sh_b];
        if (NC) q = cmulf(q, base_c[int64_t(uint32_t(tk.in_row[2] + oc)) << sh_c]);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float2 qa = cmulf(q, A[i]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 l = Bv[j];
                // unit row of (A value i, B value j): bits 0, 1, 3 from i, bits 2, 4 from j
                float2& c = acc[(i & 3) | ((j & 1) << 2) | ((i & 4) << 1) | ((j & 2) << 3)];
                c.x = fmaf(qa.x, l.x, c.x);
                c.x = fmaf(-qa.y, l.y, c.x);
                c.y = fmaf(qa.x, l.y, c.y);
                c.y = fmaf(qa.y, l.x, c.y);
            }
        }
    }
    if (TL) {
        float2* out = tv.rows + int64_t(tk.out_row) * 64 + (b & 63u);
#pragma unroll
        for (int o = 0; o < 32; ++o) out[o * 64] = acc[o];
        return;
    }
    float2* __restrict__ out = aout + int64_t(tk.out_row) * be + b;
#pragma unroll
    for (int o = 0; o < 32; ++o) out[int64_t(o) * be] = acc[o];
}

// A unit of task tk for bitstring group bg (x = the lane's bitstring).
template <int NIN, bool TL = false>
__device__ __forceinline__ void tree_task(const TreeTask& tk, uint64_t x, const float2* __restrict__ ain,
                                          float2* __restrict__ aout, const float2* __restrict__ gtab, int64_t ones_g,
                                          uint32_t b, int64_t be, const TailView& tv = TailView{}) {
    static_assert(kTreeMaxSum == 3, "tasks sum 0 (the product over the open qubits), 1, 2 or 3 variables");
    const int64_t sig = gather_sigma(x, tk.sig_q, tk.n_sig);
    if constexpr (NIN >= 2) {
        if (tk.tile == 1) {   // two or three summed variables
            if (tk.k == 2) tile_unit<2, TL, false>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            else tile_unit<3, TL, false>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            return;
        }
    }
    if constexpr (NIN == 2 || NIN == 3) {
        if (!TL && tk.tile == 3) {   // never in the tail (32-row units have too many tasks for it)
            if (tk.k == 2) tile32_unit<2, TL, false>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            else tile32_unit<3, TL, false>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            return;
        }
    }
    if constexpr (NIN >= 3) {
        if (tk.tile == 2) {
            if (tk.k == 2) tile_unit<2, TL, true>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            else tile_unit<3, TL, true>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            return;
        }
    }
    if constexpr (NIN == 3) {
        if (!TL && tk.tile == 4) {
            if (tk.k == 2) tile32_unit<2, TL, true>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            else tile32_unit<3, TL, true>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
            return;
        }
    }
    if (tk.k == 0) tree_unit<NIN, 0, TL>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
    else if (tk.k == 1) tree_unit<NIN, 1, TL>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
    else if (tk.k == 2) tree_unit<NIN, 2, TL>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
    else tree_unit<NIN, 3, TL>(tk, ain, aout, gtab, ones_g, sig, x, b, be, tv);
}

// One level of the elimination tree: wave unit u handles task u / n_bg for
// the 64 bitstrings of group u % n_bg.  The bitstring is loaded before the
// task record arrives, so the unit waits on two memory round trips (task and
// bitstring together, then inputs and factor table together) before its
// stores.
//
// With at least 8 groups (pin != 0) the units are dealt by complex: the blocks
// with blockIdx = x mod 8 take, task by task, the groups g = x mod 8 (work-groups
// go to the 8 accelerator complexes in turn, so a group's rows stay in one L2
// and the re-read rows of consecutive tasks hit there).  The split depends only
// on blockIdx: every unit runs once whatever the dispatch does.
template <int NIN>
__global__ void __launch_bounds__(256) k_tree_level(const TreeTask* __restrict__ tasks, uint32_t n_units,
                                                    const float2* __restrict__ ain, float2* __restrict__ aout,
                                                    const float2* __restrict__ gtab, int64_t ones_g,
                                                    const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                    uint32_t n_bg, int pin) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t be = int64_t(B_eff);
    if (pin) {
        const uint32_t q = blockIdx.x % uint32_t(kPersistXcds);
        const uint32_t nbx = (n_bg - q + kPersistXcds - 1) / kPersistXcds;   // groups q, q + 8, ... (n_bg >= 8)
        const uint32_t n_tasks = n_units / n_bg;
        const uint32_t n_q = n_tasks * nbx;
        const uint32_t stride = (gridDim.x / kPersistXcds) * 4u;
        for (uint32_t v = (blockIdx.x / kPersistXcds) * 4u + wave; v < n_q; v += stride) {
            const uint32_t ti = v / nbx;
            const uint32_t bg = q + kPersistXcds * (v - ti * nbx);
            const uint32_t b = bg * 64u + lane;
            const uint64_t x = int64_t(b) < B ? bits[b] : 0ull;
            const TreeTask tk = tasks[ti];
            tree_task<NIN>(tk, x, ain, aout, gtab, ones_g, b, be);
        }
        return;
    }
    for (uint32_t u = blockIdx.x * 4u + wave; u < n_units; u += gridDim.x * 4u) {
        const uint32_t ti = u / n_bg;
        const uint32_t bg = u - ti * n_bg;
        const uint32_t b = bg * 64u + lane;
        const uint64_t x = int64_t(b) < B ? bits[b] : 0ull;
        const TreeTask tk = tasks[ti];
        tree_task<NIN>(tk, x, ain, aout, gtab, ones_g, b, be);
    }
}

// Quad tiles: a work-group of 4 waves runs 4 consecutive 32-row tile tasks of
// one two-input bucket (result bits 5 and 6 vary input B only) for one group
// of 64 bitstrings.  The 8 rows of A and the factor-table entry of every
// summed value are the same for the four tasks, so the waves first load them
// once into LDS (a quarter each), then each wave runs its own task reading A
// and the table from LDS and its 4 rows of B from memory: per wave
// 9 * 2^K / 4 + 4 * 2^K row loads instead of 13 * 2^K.  Results as in
// tile32_unit (same rows, same order of the products).
constexpr int kQuadRows = 9 << kTreeMaxSum;   // 8 rows of A and one table row per summed value
// Results of a level's quad tiles beyond this many bytes are stored non-temporally: they exceed the
// last-level cache, so keeping them there would only evict the rows of A and B that other units re-read.
constexpr int64_t kQuadStreamBytes = int64_t(256) << 20;

template <int K, bool NT>
__device__ __forceinline__ void quad_unit(const TreeTask& tk, const float2* __restrict__ ain,
                                          float2* __restrict__ aout, const float2* __restrict__ gtab, int64_t ones_g,
                                          int64_t sig, uint64_t x, uint32_t b, int64_t be, uint32_t lane,
                                          uint32_t wave, float2 (*sA)[64]) {
    constexpr int W = 1 << K;
    const uint32_t be_sh = uint32_t(__builtin_ctzll(uint64_t(be)));
    const float2 *base_a, *base_b;
    uint32_t sh_a, sh_b;
    input_view<false>(tk, 0, ain, gtab, ones_g, x, b, be_sh, TailView{}, base_a, sh_a);
    input_view<false>(tk, 1, ain, gtab, ones_g, x, b, be_sh, TailView{}, base_b, sh_b);
    // LDS row r < 8W: row i = r >> K of A at summed value w = r & (W - 1); row 8W + w: the table entry
    constexpr int PER = 9 * W / 4;
    float2 v[PER];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const int r = int(wave) + 4 * s;
        const int w = r & (W - 1);
        if (r < 8 * W) {
            const int i = r >> K;
            int32_t ra = tk.in_row[0] + ((i & 1) ? tk.in_inc[0][0] : 0) + ((i & 2) ? tk.in_inc[0][1] : 0) +
                         ((i & 4) ? tk.in_inc[0][2] : 0);
#pragma unroll
            for (int c = 0; c < K; ++c)
                if ((w >> c) & 1) ra += tk.in_vs[0][c];
            v[s] = base_a[int64_t(uint32_t(ra)) << sh_a];
        } else {
            v[s] = gtab[tk.g_ent + (int64_t(w) << tk.sb) + sig];
        }
    }
#pragma unroll
    for (int s = 0; s < PER; ++s) sA[int(wave) + 4 * s][lane] = v[s];
    __syncthreads();
    int32_t rb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) rb[j] = tk.in_row[1] + ((j & 1) ? tk.in_inc[1][0] : 0) + ((j & 2) ? tk.in_inc[1][1] : 0);
    float2 acc[32];
#pragma unroll
    for (int o = 0; o < 32; ++o) acc[o] = make_float2(0.f, 0.f);
#pragma unroll 2
    for (int w = 0; w < W; ++w) {
        int32_t ob = 0;
#pragma unroll
        for (int c = 0; c < K; ++c)
            if ((w >> c) & 1) ob += tk.in_vs[1][c];
        float2 Bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) Bv[j] = base_b[int64_t(uint32_t(rb[j] + ob)) << sh_b];
        const float2 q = sA[8 * W + w][lane];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float2 qa = cmulf(q, sA[(i << K) + w][lane]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 l = Bv[j];
                float2& c = acc[(i & 3) | ((j & 1) << 2) | ((i & 4) << 1) | ((j & 2) << 3)];
                c.x = fmaf(qa.x, l.x, c.x);
                c.x = fmaf(-qa.y, l.y, c.x);
                c.y = fmaf(qa.x, l.y, c.y);
                c.y = fmaf(qa.y, l.x, c.y);
            }
        }
    }
    float2* __restrict__ out = aout + int64_t(tk.out_row) * be + b;
#pragma unroll
    for (int o = 0; o < 32; ++o) {
        if constexpr (NT) {
            typedef float f2v __attribute__((ext_vector_type(2)));
            const f2v v2 = {acc[o].x, acc[o].y};
            __builtin_nontemporal_store(v2, reinterpret_cast<f2v*>(out + int64_t(o) * be));
        } else {
            out[int64_t(o) * be] = acc[o];
        }
    }
    __syncthreads();   // the next block overwrites the LDS rows
}

// Quad tiles with two bitstrings per lane (batch pitch of 128 or more): a
// work-group of 8 waves runs the 4 tasks of a block for 128 consecutive
// bitstrings; wave (t, h) computes the 16 rows of task t whose unit bit 3
// (A's third bit) is h, for bitstrings 2l and 2l + 1 of lane l.  Every row
// load and store then moves 16 bytes per lane: the address path of the
// vector memory unit takes about the same time per instruction for 16 bytes
// as for 8, so a row costs half the instructions of the one-bitstring form.
// The rows of A and the table entries shared by the 4 tasks are staged in
// LDS, 4 summed values at a time.  Same products in the same order as
// tile32_unit and quad_unit, per bitstring.
struct Q2Lds {
    float4 a[8 * 4][64];    // row i of A at summed value w0 + c: [i * 4 + c][lane], bitstrings 2l, 2l + 1
    float2 q[4][128];       // table entry at summed value w0 + c for bitstring column j
};

// Two consecutive bitstrings' entries of an arena input at row `row`: one 16-byte load.
__device__ __forceinline__ float4 q2_load(int32_t row, const float2* __restrict__ ain, uint32_t b0, uint32_t be_sh) {
    return *reinterpret_cast<const float4*>(ain + ((int64_t(uint32_t(row)) << be_sh) + b0));
}

template <int K>
__device__ __forceinline__ void quad2_unit(const TreeTask& tk, const float2* __restrict__ ain,
                                           float2* __restrict__ aout, const float2* __restrict__ gtab,
                                           const uint64_t* __restrict__ bits, int64_t B, uint32_t c0, int64_t be,
                                           uint32_t lane, uint32_t wave, Q2Lds& S) {
    constexpr int W = 1 << K;
    constexpr int CW = W < 4 ? W : 4;   // summed values staged at a time
    const uint32_t be_sh = uint32_t(__builtin_ctzll(uint64_t(be)));
    const uint32_t tid = wave * 64u + lane;
    const uint32_t h = wave >> 2;
    const uint32_t b0 = c0 + 2u * lane;
    const uint64_t x0 = int64_t(b0) < B ? bits[b0] : 0ull, x1 = int64_t(b0) + 1 < B ? bits[b0 + 1] : 0ull;
    // the table column this thread stages, and its bitstring's output bits
    const uint32_t jc = tid & 127u;
    const uint64_t xc = int64_t(c0 + jc) < B ? bits[c0 + jc] : 0ull;
    const int64_t sig_c = gather_sigma(xc, tk.sig_q, tk.n_sig);
    int32_t rb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) rb[j] = tk.in_row[1] + ((j & 1) ? tk.in_inc[1][0] : 0) + ((j & 2) ? tk.in_inc[1][1] : 0);
    float2 acc[16][2];
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o][0] = acc[o][1] = make_float2(0.f, 0.f);
#pragma unroll
    for (int w0 = 0; w0 < W; w0 += CW) {
        // stage rows i of A at values w0 .. w0 + CW - 1 (wave takes rows r = wave + 8 s) and the table entries
        constexpr int PER = 8 * CW / 8;
        float4 v[PER];
#pragma unroll
        for (int s2 = 0; s2 < PER; ++s2) {
            const int r = int(wave) + 8 * s2;
            const int i = r / CW, w = w0 + r % CW;
            int32_t ra = tk.in_row[0] + ((i & 1) ? tk.in_inc[0][0] : 0) + ((i & 2) ? tk.in_inc[0][1] : 0) +
                         ((i & 4) ? tk.in_inc[0][2] : 0);
#pragma unroll
            for (int c = 0; c < K; ++c)
                if ((w >> c) & 1) ra += tk.in_vs[0][c];
            v[s2] = q2_load(ra, ain, b0, be_sh);
        }
        float2 qv[CW * 128 / 512 > 0 ? CW * 128 / 512 : 1];
        constexpr int QPER = CW * 128 / 512;   // table entries per thread (1 for CW = 4)
#pragma unroll
        for (int s2 = 0; s2 < QPER; ++s2) {
            const int w = w0 + int(tid >> 7) + 4 * s2;
            qv[s2] = gtab[tk.g_ent + (int64_t(w) << tk.sb) + sig_c];
        }
        if (QPER == 0 && tid < uint32_t(CW) * 128u) qv[0] = gtab[tk.g_ent + (int64_t(w0 + int(tid >> 7)) << tk.sb) + sig_c];
#pragma unroll
        for (int s2 = 0; s2 < PER; ++s2) S.a[int(wave) + 8 * s2][lane] = v[s2];
#pragma unroll
        for (int s2 = 0; s2 < QPER; ++s2) S.q[int(tid >> 7) + 4 * s2][jc] = qv[s2];
        if (QPER == 0 && tid < uint32_t(CW) * 128u) S.q[tid >> 7][jc] = qv[0];
        __syncthreads();
#pragma unroll 1   // (unrolled, 153 VGPRs and 3 waves per SIMD: one work-group per compute unit)
        for (int c = 0; c < CW; ++c) {
            const int w = w0 + c;
            int32_t ob = 0;
#pragma unroll
            for (int cc = 0; cc < K; ++cc)
                if ((w >> cc) & 1) ob += tk.in_vs[1][cc];
            float4 Bv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) Bv[j] = q2_load(rb[j] + ob, ain, b0, be_sh);
            const float4 q = reinterpret_cast<const float4*>(S.q[c])[lane];
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
                const int i = ii | int(h << 2);
                const float4 A = S.a[i * CW + c][lane];
                const float2 qa0 = cmulf(make_float2(q.x, q.y), make_float2(A.x, A.y));
                const float2 qa1 = cmulf(make_float2(q.z, q.w), make_float2(A.z, A.w));
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float2& a0 = acc[ii | ((j & 1) << 2) | ((j & 2) << 2)][0];
                    float2& a1 = acc[ii | ((j & 1) << 2) | ((j & 2) << 2)][1];
                    a0.x = fmaf(qa0.x, Bv[j].x, a0.x);
                    a0.x = fmaf(-qa0.y, Bv[j].y, a0.x);
                    a0.y = fmaf(qa0.x, Bv[j].y, a0.y);
                    a0.y = fmaf(qa0.y, Bv[j].x, a0.y);
                    a1.x = fmaf(qa1.x, Bv[j].z, a1.x);
                    a1.x = fmaf(-qa1.y, Bv[j].w, a1.x);
                    a1.y = fmaf(qa1.x, Bv[j].w, a1.y);
                    a1.y = fmaf(qa1.y, Bv[j].z, a1.y);
                }
            }
        }
        __syncthreads();   // the next values (or the next block) overwrite the staged rows
    }
    // local row o = ii | j0 << 2 | j1 << 3 is unit row ii | j0 << 2 | h << 3 | j1 << 4
    float2* __restrict__ out = aout + int64_t(tk.out_row) * be + b0;
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        const int u = (o & 7) | int(h << 3) | ((o & 8) << 1);
        float4* dst = reinterpret_cast<float4*>(out + int64_t(u) * be);
        typedef float f4v __attribute__((ext_vector_type(4)));
        const f4v r4 = {acc[o][0].x, acc[o][0].y, acc[o][1].x, acc[o][1].y};
        __builtin_nontemporal_store(r4, reinterpret_cast<f4v*>(dst));
    }
}

// The quad tiles of one level with two bitstrings per lane (levels whose results exceed the last-level cache,
// both inputs of every quad bucket arena results; stores non-temporal): block (task block tb, column group
// g2) runs tasks 4 tb .. 4 tb + 3 for bitstring columns 128 g2 .. 128 g2 + 127 on the work-group's 8 waves.
// With at least 8 column groups the blocks are dealt by accelerator complex.  Every wave runs the same blocks.
__global__ void __launch_bounds__(512) k_tree_quad2(const TreeTask* __restrict__ tasks, uint32_t n_tb,
                                                    const float2* __restrict__ ain, float2* __restrict__ aout,
                                                    const float2* __restrict__ gtab,
                                                    const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                    uint32_t n_g2, int pin) {
    __shared__ Q2Lds S;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t be = int64_t(B_eff);
    auto block = [&](uint32_t tb, uint32_t g2) {
        const TreeTask tk = tasks[4u * tb + (wave & 3u)];   // (the 4 tasks of a block have the same K)
        if (tk.k == 2) quad2_unit<2>(tk, ain, aout, gtab, bits, B, g2 * 128u, be, lane, wave, S);
        else quad2_unit<3>(tk, ain, aout, gtab, bits, B, g2 * 128u, be, lane, wave, S);
    };
    if (pin) {
        const uint32_t q = blockIdx.x % uint32_t(kPersistXcds);
        const uint32_t nbx = (n_g2 - q + kPersistXcds - 1) / kPersistXcds;   // column groups q, q + 8, ...
        const uint32_t n_q = n_tb * nbx;
        const uint32_t stride = gridDim.x / kPersistXcds;
        for (uint32_t v = blockIdx.x / kPersistXcds; v < n_q; v += stride) {
            const uint32_t tb = v / nbx;
            block(tb, q + kPersistXcds * (v - tb * nbx));
        }
        return;
    }
    for (uint32_t v = blockIdx.x; v < n_tb * n_g2; v += gridDim.x) {
        const uint32_t tb = v / n_g2;
        block(tb, v - tb * n_g2);
    }
}

// The quad tiles of one level: block (task block tb, group bg) runs tasks
// 4 tb .. 4 tb + 3 on the work-group's 4 waves.  With at least 8 groups the
// blocks are dealt by accelerator complex as in k_tree_level.  Every wave of a
// work-group runs the same blocks (the barriers inside a block are reached by
// all of them); the four tasks of a block have the same K.
template <bool NT>
__global__ void __launch_bounds__(256) k_tree_quad(const TreeTask* __restrict__ tasks, uint32_t n_tb,
                                                   const float2* __restrict__ ain, float2* __restrict__ aout,
                                                   const float2* __restrict__ gtab, int64_t ones_g,
                                                   const uint64_t* __restrict__ bits, int64_t B, uint32_t B_eff,
                                                   uint32_t n_bg, int pin) {
    __shared__ float2 sA[kQuadRows][64];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t be = int64_t(B_eff);
    auto block = [&](uint32_t tb, uint32_t bg) {
        const uint32_t b = bg * 64u + lane;
        const uint64_t x = int64_t(b) < B ? bits[b] : 0ull;
        const TreeTask tk = tasks[4u * tb + wave];
        const int64_t sig = gather_sigma(x, tk.sig_q, tk.n_sig);
        if (tk.k == 2) quad_unit<2, NT>(tk, ain, aout, gtab, ones_g, sig, x, b, be, lane, wave, sA);
        else quad_unit<3, NT>(tk, ain, aout, gtab, ones_g, sig, x, b, be, lane, wave, sA);
    };
    if (pin) {
        const uint32_t q = blockIdx.x % uint32_t(kPersistXcds);
        const uint32_t nbx = (n_bg - q + kPersistXcds - 1) / kPersistXcds;   // groups q, q + 8, ... (n_bg >= 8)
        const uint32_t n_q = n_tb * nbx;
        const uint32_t stride = gridDim.x / kPersistXcds;
        for (uint32_t v = blockIdx.x / kPersistXcds; v < n_q; v += stride) {
            const uint32_t tb = v / nbx;
            block(tb, q + kPersistXcds * (v - tb * nbx));
        }
        return;
    }
    for (uint32_t v = blockIdx.x; v < n_tb * n_bg; v += gridDim.x) {
        const uint32_t tb = v / n_bg;
        block(tb, v - tb * n_bg);
    }
}

// Phase of the factors without free variables for bitstring x (FP64), from
// values staged in LDS by stage_phase.
struct PhaseLds {
    double2 v[kTreeMaxPhaseLds][4];
    int32_t q[kTreeMaxPhaseLds][2];   // bit of x feeding each variable (-1: fixed 0; -2: a two-qubit gate
                                      //   factor, evaluated from its record)
};

__device__ __forceinline__ int stage_phase(PhaseLds& P, const TFactor* __restrict__ phase, int n_phase,
                                           const double2* __restrict__ fixed, const float2* __restrict__ slots) {
    const int n_lds = n_phase < kTreeMaxPhaseLds ? n_phase : kTreeMaxPhaseLds;
    for (int i = threadIdx.x; i < n_lds * 4; i += blockDim.x) {
        const TFactor f = phase[i >> 2];
        if (f.type != TF_MAT4) P.v[i >> 2][i & 3] = factor_value(f, (i >> 1) & 1u, i & 1u, fixed, slots);
        if ((i & 3) == 0) {
            P.q[i >> 2][0] = f.type == TF_MAT4 ? -2 : (f.src0 == TS_SIG ? f.bit0 : -1);
            P.q[i >> 2][1] = f.src1 == TS_SIG ? f.bit1 : -1;
        }
    }
    return n_lds;
}

// Product of the factors without free variables for bitstring x (FP64).
__device__ __forceinline__ double2 phase_product(const PhaseLds& P, int n_lds, const TFactor* __restrict__ phase,
                                                 int n_phase, const double2* __restrict__ fixed,
                                                 const float2* __restrict__ slots, uint64_t x) {
    double2 acc = make_double2(1.0, 0.0);
    for (int i = 0; i < n_lds; ++i) {
        if (P.q[i][0] == -2) {
            acc = cmuld(acc, phase_factor(phase[i], x, fixed, slots));
            continue;
        }
        const uint32_t a = P.q[i][0] >= 0 ? uint32_t((x >> P.q[i][0]) & 1ull) : 0u;
        const uint32_t c = P.q[i][1] >= 0 ? uint32_t((x >> P.q[i][1]) & 1ull) : 0u;
        acc = cmuld(acc, P.v[i][a * 2 + c]);
    }
    for (int i = n_lds; i < n_phase; ++i) acc = cmuld(acc, phase_factor(phase[i], x, fixed, slots));   // beyond LDS
    return acc;
}

// Amplitude = phase x product of the rank-0 results (FP64), written as complex64 or complex128.
__device__ __forceinline__ void write_amplitude(const PhaseLds& P, int n_lds, const TFactor* __restrict__ phase,
                                                int n_phase, const double2* __restrict__ fixed,
                                                const float2* __restrict__ slots, const int64_t* __restrict__ final_rows,
                                                int n_final, const float2* __restrict__ arena, uint64_t x, uint32_t b,
                                                uint32_t B_eff, void* __restrict__ out, int c128) {
    double2 acc = phase_product(P, n_lds, phase, n_phase, fixed, slots, x);
    for (int i = 0; i < n_final; ++i) {
        const float2 r = arena[final_rows[i] * int64_t(B_eff) + b];
        acc = cmuld(acc, make_double2(r.x, r.y));
    }
    if (c128) static_cast<double2*>(out)[b] = acc;
    else static_cast<float2*>(out)[b] = make_float2(float(acc.x), float(acc.y));
}

// The last levels of the tree, whose buckets have few rows, in one launch:
// work-group g owns the 64 bitstrings of group g and runs every task of
// every tail level for them, its four waves taking the tasks of a level in
// turn, with a block barrier between levels (a level reads only results of
// earlier levels).  One burst of loads at the start copies to LDS what the
// tail reads more than once or late: the task and level records, the tail's
// factor tables, the FP64 values of the phase factors and the list of rank-0
// results.  The results made here stay in LDS, so after the first level
// (whose inputs are arena rows) a level waits only on LDS.  The phase product
// is split over waves 1-3 (factor i to wave 1 + i mod 3), each taking its
// share in the first level where it has no task; wave 0 then multiplies the
// three partial products and the rank-0 results in FP64.
constexpr int kTreeTailPhase = 64;   // phase factors whose values the tail stages in LDS

struct TailLds {
    TreeTask task[kTreeTailMaxTasks];
    TreeTailLevel lv[kTreeTailMaxLevels];
    int32_t fin[kTreeTailMaxFinal];
    float2 g[kTreeTailGEntries];
    float2 one;
    uint4 junk;                              // written by threads of the staging that have no element
    double2 part[3][64];
    double2 pv[kTreeTailPhase][4];           // FP64 values of the first kTreeTailPhase phase factors
    int32_t pq[kTreeTailPhase][2];           // the bits of x they read (-1 none, -2 from the record)
    float2 rows[kTreeTailLdsRows * 64];
};

// A task record kept in LDS, read into scalar registers (the address is uniform).
__device__ __forceinline__ TreeTask task_from_lds(const TreeTask* p) {
    TreeTask tk;
    const int32_t* src = reinterpret_cast<const int32_t*>(p);
    int32_t* dst = reinterpret_cast<int32_t*>(&tk);
#pragma unroll
    for (int i = 0; i < int(sizeof(TreeTask) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return tk;
}

constexpr int kTailTaskWords = (kTreeTailMaxTasks * int(sizeof(TreeTask)) / 16 + 255) / 256;
constexpr int kTailGWords = (kTreeTailGEntries / 2 + 255) / 256;          // 16-byte words of the tables
constexpr int kTailPhaseWords = (kTreeTailPhase * 4 + 255) / 256;          // double2 phase values

__global__ void __launch_bounds__(256) k_tree_tail(const TreeTailArgs a) {
    __shared__ TailLds T;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t be = int64_t(a.B_eff);
    const uint32_t b = blockIdx.x * 64u + lane;
    const int n_lds = a.n_phase < kTreeTailPhase ? a.n_phase : kTreeTailPhase;
    const uint64_t x = int64_t(b) < a.B ? a.bits[b] : 0ull;
    {   // every load of the staging in flight at once, then the LDS writes, all unconditional so that the
        // code is one straight run: indices are clamped into each array (every array holds at least one
        // element) and a thread without an element writes to a junk word
        const int tid = int(threadIdx.x);
        const int n_tw = a.n_tasks * int(sizeof(TreeTask) / 16);
        const int n_gw = (a.tail_g_entries + 1) / 2;
        const int n_pw = 4 * n_lds;
        const uint4* __restrict__ tsrc = reinterpret_cast<const uint4*>(a.tasks);
        const float4* __restrict__ gsrc = reinterpret_cast<const float4*>(a.gtab + a.tail_g0);   // tail_g0 is even
        const double2* __restrict__ psrc = reinterpret_cast<const double2*>(a.gtab + a.phase_g);
        auto clamp = [](int i, int n) { return i < n ? i : (n > 0 ? n - 1 : 0); };
        uint4 tv[kTailTaskWords];
        float4 gv[kTailGWords];
        double2 pv[kTailPhaseWords];
#pragma unroll
        for (int k = 0; k < kTailTaskWords; ++k) tv[k] = tsrc[clamp(tid + 256 * k, n_tw)];
#pragma unroll
        for (int k = 0; k < kTailGWords; ++k) gv[k] = gsrc[clamp(tid + 256 * k, n_gw)];
#pragma unroll
        for (int k = 0; k < kTailPhaseWords; ++k) pv[k] = psrc[clamp(tid + 256 * k, n_pw)];
        const TreeTailLevel lv = a.levels[clamp(tid, a.n_levels)];
        const int32_t fin = a.final_lds[clamp(tid, a.n_final)];
        const int32_t q0 = a.phase_q[2 * clamp(tid, n_lds)];
        const int32_t q1 = a.phase_q[2 * clamp(tid, n_lds) + 1];
        uint4* junk = &T.junk;
#pragma unroll
        for (int k = 0; k < kTailTaskWords; ++k) {
            const int i = tid + 256 * k;
            *(i < n_tw ? reinterpret_cast<uint4*>(T.task) + i : junk) = tv[k];
        }
#pragma unroll
        for (int k = 0; k < kTailGWords; ++k) {
            const int i = tid + 256 * k;
            *(i < n_gw ? reinterpret_cast<float4*>(T.g) + i : reinterpret_cast<float4*>(junk)) = gv[k];
        }
#pragma unroll
        for (int k = 0; k < kTailPhaseWords; ++k) {
            const int i = tid + 256 * k;
            *(i < n_pw ? &T.pv[i >> 2][i & 3] : reinterpret_cast<double2*>(junk)) = pv[k];
        }
        *(tid < a.n_levels ? &T.lv[tid] : reinterpret_cast<TreeTailLevel*>(junk)) = lv;
        *(tid < a.n_final ? &T.fin[tid] : reinterpret_cast<int32_t*>(junk)) = fin;
        *(tid < n_lds ? &T.pq[tid][0] : reinterpret_cast<int32_t*>(junk)) = q0;
        *(tid < n_lds ? &T.pq[tid][1] : reinterpret_cast<int32_t*>(junk) + 1) = q1;
        if (tid == 0) T.one = make_float2(1.f, 0.f);
    }
    __syncthreads();
    const TailView view{T.rows, T.g, &T.one};
    // this wave's share of the phase product (waves 1-3), into LDS
    auto phase_part = [&]() {
        double2 acc = make_double2(1.0, 0.0);
        for (int i = int(wave) - 1; i < a.n_phase; i += 3) {
            if (i >= n_lds || T.pq[i][0] == -2) {
                acc = cmuld(acc, phase_factor(a.phase[i], x, a.fixed, a.slots));
                continue;
            }
            const uint32_t ba = T.pq[i][0] >= 0 ? uint32_t((x >> T.pq[i][0]) & 1ull) : 0u;
            const uint32_t bc = T.pq[i][1] >= 0 ? uint32_t((x >> T.pq[i][1]) & 1ull) : 0u;
            acc = cmuld(acc, T.pv[i][ba * 2 + bc]);
        }
        T.part[wave - 1][lane] = acc;
    };
    bool part_done = wave == 0;
    for (int l = 0; l < a.n_levels; ++l) {
        const int task_off = __builtin_amdgcn_readfirstlane(T.lv[l].task_off);
        const int n_tasks = __builtin_amdgcn_readfirstlane(T.lv[l].n_tasks);
        const int nin = __builtin_amdgcn_readfirstlane(T.lv[l].nin);
        for (int t = int(wave); t < n_tasks; t += 4) {
            const TreeTask tk = task_from_lds(&T.task[task_off + t]);
            if (nin <= 1) tree_task<1, true>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be, view);
            else if (nin == 2) tree_task<2, true>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be, view);
            else if (nin == 3) tree_task<3, true>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be, view);
            else tree_task<4, true>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be, view);
        }
        if (!part_done && int(wave) >= n_tasks) {
            phase_part();
            part_done = true;
        }
        __syncthreads();
    }
    if (!part_done) phase_part();
    __syncthreads();
    if (wave == 0 && int64_t(b) < a.B) {
        double2 acc = cmuld(cmuld(T.part[0][lane], T.part[1][lane]), T.part[2][lane]);
        for (int i = 0; i < a.n_final; ++i) {
            const int32_t f = T.fin[i];
            const float2 r = f < 0 ? T.rows[(-1 - f) * 64 + int(lane)] : a.arena[int64_t(f) * be + b];
            acc = cmuld(acc, make_double2(r.x, r.y));
        }
        if (a.c128) static_cast<double2*>(a.out)[b] = acc;
        else static_cast<float2*>(a.out)[b] = make_float2(float(acc.x), float(acc.y));
    }
}

// The amplitudes when the tree has no tail levels.
__global__ void __launch_bounds__(256) k_tree_final(const int64_t* __restrict__ final_rows, int n_final,
                                                    const TFactor* __restrict__ phase, int n_phase,
                                                    const double2* __restrict__ fixed, const float2* __restrict__ slots,
                                                    const float2* __restrict__ arena, const uint64_t* __restrict__ bits,
                                                    int64_t B, uint32_t B_eff, void* __restrict__ out, int c128) {
    __shared__ PhaseLds P;
    const int n_lds = stage_phase(P, phase, n_phase, fixed, slots);
    __syncthreads();
    const uint32_t b = blockIdx.x * 256u + threadIdx.x;
    if (int64_t(b) >= B) return;
    write_amplitude(P, n_lds, phase, n_phase, fixed, slots, final_rows, n_final, arena, bits[b], b, B_eff, out, c128);
}

// ---- persistent launch: every level and the amplitude product at once ----
//
// Wave unit (task, bitstring group g) needs only the results of its inputs'
// tasks for the same group, so a launch can run all levels without a kernel
// boundary if each unit waits for exactly those.  Group g is pinned to the
// accelerator complex (XCD) g mod 8: a work-group reads the complex it runs on
// from its XCC_ID register and serves that complex's groups, its rank among
// the complex's work-groups being blockIdx / 8 (work-groups are dealt to the
// complexes in turn; a rank met twice aborts the launch), so a result row of
// group g is written and read through one L2.  Completion is signalled by one flag per (group, task), set with an
// agent-scope atomic store after the unit's stores are complete (s_waitcnt
// vmcnt(0): acknowledged by that L2), and polled with agent-scope atomic loads.
// Every result has its own rows for the whole launch (keep-all layout), so no
// L1 line read by a consumer can predate its producer's store.  Each XCD's
// waves take the units of its groups in increasing (task, group) order with a
// fixed stride; a unit waits only on units of lower index, and the grid fits
// the GPU at once, so the lowest unfinished unit can always proceed.  A wait
// that exceeds the launch's spin limit (2^20 polls unless the plan sets
// another) sets the abort word and the plan's failure record; later waits
// return at once and the amplitudes of the launch are written as NaN, so every
// wave still ends (amplitudes start as NaN, so one that is never written reads
// NaN).

__device__ __forceinline__ int32_t ld_flag(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until flags f[0, n) are all set (64 per poll, one per lane).  Giving
// up sets the launch's abort word and the plan's failure record.
__device__ void persist_wait(const int32_t* f, int n, int32_t* abort_word, int32_t* status, int spin_limit,
                             uint32_t lane) {
    for (int i0 = 0; i0 < n; i0 += 64) {
        const bool mine = i0 + int(lane) < n;
        for (int spin = 0;; ++spin) {
            const int32_t v = mine ? ld_flag(f + i0 + lane) : 1;
            if (__all(v != 0)) break;
            if (ld_flag(abort_word) != 0) return;
            if (spin >= spin_limit) {
                if (lane == 0) {
                    st_flag(abort_word, 1);
                    st_flag(status, 1);
                }
                return;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
}

template <int MAXC>
__global__ void __launch_bounds__(256) k_tree_persist(const TreePersist a) {
    __shared__ PhaseLds P;
    const int n_lds = stage_phase(P, a.phase, a.n_phase, a.fixed, a.slots);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t* abort_word = a.flags;
    const uint32_t xcc = __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11));   // HW_REG_XCC_ID[3:0]
    const uint32_t q = xcc % uint32_t(kPersistXcds);
    const uint32_t rank = blockIdx.x / kPersistXcds;
    if (threadIdx.x == 0) {
        // a complex outside 0..7, or a (complex, rank) pair met twice, breaks the pinning: abort (units still run)
        const int32_t seen = __hip_atomic_exchange(a.flags + kPersistSeen0 + q * kPersistMaxRanks + rank, 1,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (xcc >= uint32_t(kPersistXcds) || seen != 0) {
            st_flag(abort_word, 2);
            st_flag(a.status, 2);
        }
    }
    const uint32_t n_bg = a.B_eff / 64u;
    if (q >= n_bg) return;
    const uint32_t nbx = (n_bg - q + kPersistXcds - 1) / kPersistXcds;   // groups q, q + 8, ...
    const uint32_t n_waves = (gridDim.x / kPersistXcds) * 4u;
    const uint32_t w = rank * 4u + wave;
    const int64_t n_units = int64_t(a.n_tasks + 1) * nbx;
    const int64_t be = int64_t(a.B_eff);
    for (int64_t u = w; u < n_units; u += n_waves) {
        const int32_t ti = int32_t(u / nbx);
        const uint32_t bg = q + kPersistXcds * uint32_t(u - int64_t(ti) * nbx);
        const uint32_t b = bg * 64u + lane;
        const uint64_t x = int64_t(b) < a.B ? a.bits[b] : 0ull;
        int32_t* fl = a.flags + kPersistFlags0 + int64_t(bg) * a.flag_stride - a.task0;   // indexed by task number
        if (ti < a.n_tasks) {
            // the dependency lists are read from the record in memory (uniform index: scalar loads), not
            // from the register copy, which a run-time index would move to scratch
            const TreeTask* __restrict__ tp = a.tasks + ti;
            const int n_in = tp->n_in;
            for (int t = 0; t < n_in; ++t)
                persist_wait(fl + tp->dep_off[t], tp->dep_n[t], abort_word, a.status, a.spin_limit, lane);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // no input load moves above the polls
            const TreeTask tk = *tp;
            // the variant the task's rows were laid out for (the launch carries those up to the plan's largest)
            if (MAXC <= 1 || tk.nin_class == 1) tree_task<1>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be);
            else if (MAXC <= 2 || tk.nin_class == 2) tree_task<2>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be);
            else if (MAXC <= 3 || tk.nin_class == 3) tree_task<3>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be);
            else if (MAXC <= 4 || tk.nin_class == 4) tree_task<4>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be);
            else tree_task<kTreeMaxIn>(tk, x, a.arena, a.arena, a.gtab, a.ones_g, b, be);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");   // no result store moves below the flag
            __builtin_amdgcn_s_waitcnt(0);   // the unit's result stores are complete in L2
            if (lane == 0) st_flag(fl + a.task0 + ti, 1);
        } else {
            for (int f = 0; f < a.n_final_dep; ++f)
                persist_wait(fl + a.final_dep[2 * f], a.final_dep[2 * f + 1], abort_word, a.status, a.spin_limit,
                             lane);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (int64_t(b) < a.B) {
                if (ld_flag(abort_word) != 0) {
                    const double nan = __builtin_nan("");
                    if (a.c128) static_cast<double2*>(a.out)[b] = make_double2(nan, nan);
                    else static_cast<float2*>(a.out)[b] = make_float2(float(nan), float(nan));
                } else {
                    write_amplitude(P, n_lds, a.phase, a.n_phase, a.fixed, a.slots, a.final_rows, a.n_final, a.arena,
                                    x, b, a.B_eff, a.out, a.c128);
                }
            }
        }
    }
}

// Clears the flags of a persistent launch and sets its amplitudes to NaN.
__global__ void __launch_bounds__(256) k_persist_init(int32_t* __restrict__ flags, int64_t n_flags,
                                                      void* __restrict__ out, int64_t B, int c128) {
    const double nan = __builtin_nan("");
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n_flags + B; i += int64_t(gridDim.x) * 256) {
        if (i < n_flags) flags[i] = 0;
        else if (c128) static_cast<double2*>(out)[i - n_flags] = make_double2(nan, nan);
        else static_cast<float2*>(out)[i - n_flags] = make_float2(float(nan), float(nan));
    }
}

void launch_persist_init(int32_t* flags, int64_t n_flags, void* out, int64_t B, bool c128, hipStream_t stream) {
    const int64_t n = n_flags + B;
    if (n <= 0) return;
    const uint32_t grid = uint32_t(std::min<int64_t>((n + 255) / 256, 1024));
    hipLaunchKernelGGL(k_persist_init, dim3(grid), dim3(256), 0, stream, flags, n_flags, out, B, c128 ? 1 : 0);
}

// Grid: per XCD, as many work-groups as its compute units hold at once (the
// whole grid is resident), but no more than the XCD's units need.
template <int MAXC>
static hipError_t launch_persist_c(const TreePersist& a, hipStream_t stream) {
    static thread_local int cached_dev = -1, per_xcd = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev != cached_dev) {
        int n_cu = 0, occ = 0;
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_tree_persist<MAXC>),
                                                         256, 0);
        if (e != hipSuccess) return e;
        if (n_cu < kPersistXcds || occ < 1) return hipErrorInvalidConfiguration;
        per_xcd = std::min((n_cu / kPersistXcds) * occ, kPersistMaxRanks);
        cached_dev = dev;
    }
    const int64_t n_bg = a.B_eff / 64u;
    const int64_t nbx = (n_bg + kPersistXcds - 1) / kPersistXcds;
    const int64_t want = (int64_t(a.n_tasks + 1) * nbx + 3) / 4;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(per_xcd, want));
    hipLaunchKernelGGL(k_tree_persist<MAXC>, dim3(uint32_t(blocks * kPersistXcds)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_tree_persist(const TreePersist& a, hipStream_t stream) {
    switch (a.max_class) {
        case 1: return launch_persist_c<1>(a, stream);
        case 2: return launch_persist_c<2>(a, stream);
        case 3: return launch_persist_c<3>(a, stream);
        case 4: return launch_persist_c<4>(a, stream);
        default: return launch_persist_c<kTreeMaxIn>(a, stream);
    }
}

// Sets of amplitudes (open qubits): out[b][o] = phase x rank-0 results x R[row(o)] in
// FP64, R the result over the open qubits' variables (absent: 1), row(o) the bits
// of o outside zero_mask packed in order (the result's axes follow the output
// bits), and 0 when o has a bit of zero_mask set (an open qubit without
// non-diagonal gates ends in 0).  Block: 256 bitstrings x one chunk of kOpenChunk
// output indices.
constexpr int kOpenChunk = 64;
__global__ void __launch_bounds__(256) k_tree_final_open(const int64_t* __restrict__ final_rows, int n_final,
                                                         const TFactor* __restrict__ phase, int n_phase,
                                                         const double2* __restrict__ fixed,
                                                         const float2* __restrict__ slots,
                                                         const float2* __restrict__ arena, int64_t open_row,
                                                         int n_open, uint32_t zero_mask,
                                                         const uint64_t* __restrict__ bits, int64_t B,
                                                         uint32_t B_eff, void* __restrict__ out, int c128) {
    __shared__ PhaseLds P;
    const int n_lds = stage_phase(P, phase, n_phase, fixed, slots);
    __syncthreads();
    const uint32_t b = blockIdx.x * 256u + threadIdx.x;
    if (int64_t(b) >= B) return;
    const uint64_t x = bits[b];
    double2 acc = phase_product(P, n_lds, phase, n_phase, fixed, slots, x);
    for (int i = 0; i < n_final; ++i) {
        const float2 r = arena[final_rows[i] * int64_t(B_eff) + b];
        acc = cmuld(acc, make_double2(r.x, r.y));
    }
    const uint64_t n_out = uint64_t(1) << n_open;
    const uint64_t o0 = uint64_t(blockIdx.y) * kOpenChunk;
    for (uint64_t o = o0; o < o0 + kOpenChunk && o < n_out; ++o) {
        double2 v = make_double2(0.0, 0.0);
        if ((o & zero_mask) == 0) {
            v = acc;
            if (open_row >= 0) {
                uint64_t row = 0;
                int j = 0;
                for (int i = 0; i < n_open; ++i) {
                    if ((zero_mask >> i) & 1u) continue;
                    row |= ((o >> i) & 1ull) << j;
                    ++j;
                }
                const float2 r = arena[(open_row + int64_t(row)) * int64_t(B_eff) + b];
                v = cmuld(v, make_double2(r.x, r.y));
            }
        }
        const uint64_t k = uint64_t(b) * n_out + o;
        if (c128) static_cast<double2*>(out)[k] = v;
        else static_cast<float2*>(out)[k] = make_float2(float(v.x), float(v.y));
    }
}

void launch_tree_final_open(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase,
                            const double2* fixed, const float2* slots, const float2* arena, int64_t open_row,
                            int n_open, uint32_t zero_mask, const uint64_t* bits, int64_t B, uint32_t B_eff,
                            void* out, bool c128, hipStream_t stream) {
    const uint32_t gx = uint32_t((B + 255) / 256);
    const uint32_t gy = uint32_t(((int64_t(1) << n_open) + kOpenChunk - 1) / kOpenChunk);
    hipLaunchKernelGGL(k_tree_final_open, dim3(gx, gy), dim3(256), 0, stream, final_rows, n_final, phase, n_phase,
                       fixed, slots, arena, open_row, n_open, zero_mask, bits, B, B_eff, out, c128 ? 1 : 0);
}

// Leaf tables (plans without gate values, once): block (entry chunk, leaf).
// R[o][s] = sum over the leaf's summed values w of its factor table
// G[((o << k) | w) << sb | s], in FP64, rounded once.
__global__ void __launch_bounds__(256) k_tree_leaf_tables(const TreeLeaf* __restrict__ leaves, int depth,
                                                          float2* __restrict__ gtab) {
    const TreeLeaf& L = leaves[blockIdx.y];
    if (L.depth != depth) return;
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= (int64_t(1) << (L.r + L.sb))) return;
    const int64_t o = e >> L.sb, sg = e & ((int64_t(1) << L.sb) - 1);
    int64_t g = o;
    if (L.n_in > 0) {
        g = 0;
        for (int j = 0; j < L.gb; ++j) g |= ((o >> L.gpos[j]) & 1) << j;
    }
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t w = 0; w < (int64_t(1) << L.k); ++w) {
        const float2 v = gtab[L.g_off + ((((g << L.k) | w) << L.sb) | sg)];
        double2 term = make_double2(v.x, v.y);
        for (int t = 0; t < L.n_in; ++t) {   // a composed leaf: its inputs' entries (FP64 products)
            int64_t idx = 0;
            for (int a = 0; a < L.in_na[t]; ++a) {
                const int src = L.in_src[t][a];
                idx |= (src >= 16 ? (w >> (src - 16)) & 1 : (o >> src) & 1) << a;
            }
            int64_t s = 0;
            for (int b = 0; b < L.in_sb[t]; ++b) s |= ((sg >> L.in_spos[t][b]) & 1) << b;
            const float2 x = gtab[L.in_off[t] + ((idx << L.in_sb[t]) | s)];
            term = cmuld(term, make_double2(x.x, x.y));
        }
        acc.x += term.x;
        acc.y += term.y;
    }
    gtab[L.leaf_off + e] = make_float2(float(acc.x), float(acc.y));
}

void launch_tree_leaf_tables(const TreeLeaf* leaves, int n_leaves, int64_t max_entries, int max_depth, float2* gtab,
                             hipStream_t stream) {
    if (n_leaves <= 0) return;
    for (int d = 0; d <= max_depth; ++d)   // a composed leaf reads leaves of smaller depth
        hipLaunchKernelGGL(k_tree_leaf_tables, dim3(uint32_t((max_entries + 255) / 256), uint32_t(n_leaves)),
                           dim3(256), 0, stream, leaves, d, gtab);
}

void launch_tree_prologue(const TreeProBlock* blocks, int n_blocks, const TreeGTab* gtabs, const TreeGroup* groups,
                          const TFactor* facs, const double2* fixed, const float2* slots, float2* gtab,
                          int64_t ones_g, const TFactor* phase, int n_phase, int64_t phase_g, hipStream_t stream) {
    if (n_blocks <= 0) return;   // a plan without buckets reads no table
    hipLaunchKernelGGL(k_tree_prologue, dim3(uint32_t(n_blocks)), dim3(256), 0, stream, blocks, gtabs, groups, facs,
                       fixed, slots, gtab, ones_g, phase, n_phase, phase_g);
}

template <int NIN>
static void launch_level_n(hipStream_t stream, const TreeTask* tasks, int64_t n_tasks, const float2* ain,
                           float2* aout, const float2* gtab, int64_t ones_g, const uint64_t* bits, int64_t B,
                           uint32_t B_eff, uint32_t n_bg) {
    // launches of at most 2^31 wave units (tasks of one level are independent)
    const int64_t per = std::max<int64_t>(1, (int64_t(1) << 31) / int64_t(n_bg));
    for (int64_t t0 = 0; t0 < n_tasks; t0 += per) {
        const int64_t nt = std::min<int64_t>(per, n_tasks - t0);
        const uint32_t n_units = uint32_t(nt * n_bg);
        uint32_t grid = uint32_t(std::min<int64_t>((int64_t(n_units) + 3) / 4, kStepMaxGrid));
        const int pin = n_bg >= uint32_t(kPersistXcds) ? 1 : 0;
        if (pin) grid = std::max<uint32_t>(grid / kPersistXcds, 1) * kPersistXcds;   // a multiple of 8 blocks
        hipLaunchKernelGGL(k_tree_level<NIN>, dim3(grid), dim3(256), 0, stream, tasks + t0, n_units, ain, aout, gtab,
                           ones_g, bits, B, B_eff, n_bg, pin);
    }
}

void launch_tree_level(int nin, const TreeTask* tasks, int32_t n_tasks, const float2* ain, float2* aout,
                       const float2* gtab, int64_t ones_g, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       uint32_t n_groups, hipStream_t stream, int32_t n_quad, bool quad_arena) {
    const uint32_t n_bg = n_groups;
    if (n_tasks <= 0 || n_bg == 0) return;
    // the level's quad tiles first, then its other tasks; results beyond the last-level cache: two bitstrings
    // per lane (half the load and store instructions; a smaller level runs faster with twice the work-groups)
    // and non-temporal stores
    const bool big = int64_t(n_quad) * 32 * int64_t(B_eff) * int64_t(sizeof(float2)) > kQuadStreamBytes;
    if (n_quad > 0 && B_eff >= 128 && big && quad_arena) {
        const uint32_t n_g2 = (n_bg + 1) / 2;   // column groups of 128 (within the pitch, a power of two >= 128)
        const int64_t per = std::max<int64_t>(1, (int64_t(1) << 31) / int64_t(n_g2));
        for (int64_t tb0 = 0; tb0 < n_quad / 4; tb0 += per) {
            const int64_t ntb = std::min<int64_t>(per, n_quad / 4 - tb0);
            const int pin = n_g2 >= uint32_t(kPersistXcds) ? 1 : 0;
            uint32_t grid = uint32_t(std::min<int64_t>(ntb * int64_t(n_g2), kStepMaxGrid));
            if (pin) grid = std::max<uint32_t>(grid / kPersistXcds, 1) * kPersistXcds;
            hipLaunchKernelGGL(k_tree_quad2, dim3(grid), dim3(512), 0, stream, tasks + 4 * tb0, uint32_t(ntb), ain,
                               aout, gtab, bits, B, B_eff, n_g2, pin);
        }
        tasks += n_quad;
        n_tasks -= n_quad;
        n_quad = 0;
        if (n_tasks <= 0) return;
    }
    if (n_quad > 0) {
        const bool nt = big;
        const int64_t per = std::max<int64_t>(1, (int64_t(1) << 31) / int64_t(n_bg));   // blocks per launch
        for (int64_t tb0 = 0; tb0 < n_quad / 4; tb0 += per) {
            const int64_t ntb = std::min<int64_t>(per, n_quad / 4 - tb0);
            const int pin = n_bg >= uint32_t(kPersistXcds) ? 1 : 0;
            uint32_t grid = uint32_t(std::min<int64_t>(ntb * int64_t(n_bg), kStepMaxGrid));
            if (pin) grid = std::max<uint32_t>(grid / kPersistXcds, 1) * kPersistXcds;
            if (nt)
                hipLaunchKernelGGL(k_tree_quad<true>, dim3(grid), dim3(256), 0, stream, tasks + 4 * tb0, uint32_t(ntb),
                                   ain, aout, gtab, ones_g, bits, B, B_eff, n_bg, pin);
            else
                hipLaunchKernelGGL(k_tree_quad<false>, dim3(grid), dim3(256), 0, stream, tasks + 4 * tb0,
                                   uint32_t(ntb), ain, aout, gtab, ones_g, bits, B, B_eff, n_bg, pin);
        }
        tasks += n_quad;
        n_tasks -= n_quad;
        if (n_tasks <= 0) return;
    }
    switch (launch_inputs(nin)) {
        case 1: launch_level_n<1>(stream, tasks, n_tasks, ain, aout, gtab, ones_g, bits, B, B_eff, n_bg); break;
        case 2: launch_level_n<2>(stream, tasks, n_tasks, ain, aout, gtab, ones_g, bits, B, B_eff, n_bg); break;
        case 3: launch_level_n<3>(stream, tasks, n_tasks, ain, aout, gtab, ones_g, bits, B, B_eff, n_bg); break;
        case 4: launch_level_n<4>(stream, tasks, n_tasks, ain, aout, gtab, ones_g, bits, B, B_eff, n_bg); break;
        default: launch_level_n<kTreeMaxIn>(stream, tasks, n_tasks, ain, aout, gtab, ones_g, bits, B, B_eff, n_bg);
    }
}

void launch_tree_tail(const TreeTailArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(k_tree_tail, dim3(uint32_t((a.B + 63) / 64)), dim3(256), 0, stream, a);
}

void launch_tree_final(const int64_t* final_rows, int n_final, const TFactor* phase, int n_phase, const double2* fixed,
                       const float2* slots, const float2* arena, const uint64_t* bits, int64_t B, uint32_t B_eff,
                       void* out, bool c128, hipStream_t stream) {
    const uint32_t grid = uint32_t((B + 255) / 256);
    hipLaunchKernelGGL(k_tree_final, dim3(grid), dim3(256), 0, stream, final_rows, n_final, phase, n_phase, fixed,
                       slots, arena, bits, B, B_eff, out, c128 ? 1 : 0);
}

// Slicing (Sec. V outlook): the batch columns of one chunk of slices.  Column
// b * 2^chunk_bits + j carries bitstring b with slice (slice0 + j) in the
// bits above the n qubits, so the kernels fix sliced variable i by bit n + i
// exactly as they fix an output variable by its qubit's bit.
__global__ void __launch_bounds__(256) k_slice_cols(const uint64_t* __restrict__ bits, int64_t B, int n,
                                                    int chunk_bits, uint64_t slice0, uint64_t* __restrict__ cols) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= (B << chunk_bits)) return;
    const int64_t b = c >> chunk_bits;
    const uint64_t j = uint64_t(c) & ((uint64_t(1) << chunk_bits) - 1);
    cols[c] = (bits[b] & ((uint64_t(1) << n) - 1)) | ((slice0 + j) << n);   // n < 64 when a plan slices
}

// Sum over the slices of one chunk, in slice order, in FP64: v = (first ? 0 :
// acc) + sum_j part[b * 2^chunk_bits + j][o]; the last chunk writes the
// amplitude (complex64 or complex128), the others the running sum.
__global__ void __launch_bounds__(256) k_slice_sum(const double2* __restrict__ part, int64_t B, int chunk_bits,
                                                   int n_open, double2* __restrict__ acc, int first, int last,
                                                   void* __restrict__ out, int c128) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t n_out = int64_t(1) << n_open;
    if (e >= B * n_out) return;
    const int64_t b = e >> n_open, o = e & (n_out - 1);
    double2 v = first ? make_double2(0.0, 0.0) : acc[e];
    for (int64_t j = 0; j < (int64_t(1) << chunk_bits); ++j) {
        const double2 x = part[(((b << chunk_bits) + j) << n_open) + o];
        v.x += x.x;
        v.y += x.y;
    }
    if (!last) acc[e] = v;
    else if (c128) static_cast<double2*>(out)[e] = v;
    else static_cast<float2*>(out)[e] = make_float2(float(v.x), float(v.y));
}

void launch_slice_cols(const uint64_t* bits, int64_t B, int n, int chunk_bits, uint64_t slice0, uint64_t* cols,
                       hipStream_t stream) {
    const int64_t m = B << chunk_bits;
    hipLaunchKernelGGL(k_slice_cols, dim3(uint32_t((m + 255) / 256)), dim3(256), 0, stream, bits, B, n, chunk_bits,
                       slice0, cols);
}

void launch_slice_sum(const double2* part, int64_t B, int chunk_bits, int n_open, double2* acc, bool first, bool last,
                      void* out, bool c128, hipStream_t stream) {
    const int64_t m = B << n_open;
    hipLaunchKernelGGL(k_slice_sum, dim3(uint32_t((m + 255) / 256)), dim3(256), 0, stream, part, B, chunk_bits, n_open,
                       acc, first ? 1 : 0, last ? 1 : 0, out, c128 ? 1 : 0);
}

}  // namespace qgm
