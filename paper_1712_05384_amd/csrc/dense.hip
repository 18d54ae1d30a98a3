// Dense elimination step on the matrix cores (FP32 MFMA, or BF16x3 split
// precision with FP32 accumulation, gfx950).
//
// Same contraction as k_step, F'[row, n] = sum_k F[row (+) k] G_sigma(b)[v, k, n],
// for steps whose K and N are both large (2^3..2^5): there the VALU kernel is
// bound by the complex multiply-adds and the G reads, not by HBM.
//
// Per bitstring b the step is a small GEMM C_b[m, n] = sum_k A_b[m, k] G[k, n]
// whose operand G depends on b only through the variant sigma(b).  Complex
// numbers use the real 2x2 embedding: with A_r[m][2k+c'] the interleaved
// (re, im) of A and
//   Gemb[2k][2n] = Re G, Gemb[2k][2n+1] = Im G, Gemb[2k+1][2n] = -Im G, Gemb[2k+1][2n+1] = Re G,
// C_r = A_r Gemb is the interleaved C, so the data stay complex64 in memory and
// the algorithmic flop count 8*M*K*N is unchanged.
//
// Work-group tile: 16 consecutive bitstrings x 16 frontier rows that share the
// V bits.  Each thread owns one bitstring and K (row, k) pairs of the tile; the
// next tile's A is prefetched into registers (all loads issued together) while
// the current tile is multiplied, and lands in LDS as [b][row][2K+2 floats]
// with a b pitch of 16*(2K+2)+2 floats: the 16 lanes that write one row hit
// distinct banks, and the row pitch spreads a half-wave's MFMA operand reads.
// Global accesses are 128-byte contiguous (16 b of one row).  Each wave takes
// the bitstrings of one variant sigma (the 16 are sorted by sigma), so its G
// fragments stay in VGPRs across tiles and are loaded again only when sigma or
// the V bits change; per bitstring it issues (2K/4) x (2N/16)
// v_mfma_f32_16x16x4_f32 and writes C back over A in LDS, from where the tile
// is stored with the same 128-byte accesses.
//
// BF16x3: the same tile, with every FP32 operand split into bf16 hi + lo and
// three v_mfma_f32_16x16x16_bf16 (hi*hi + hi*lo + lo*hi) per 16-deep k-step,
// accumulated in FP32: 3 * (2K/16) * (2N/16) instructions per bitstring.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qgm {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// BF16x3 split of an FP32 value: hi = bf16(x) rounded to nearest even, lo =
// bf16(x - hi); a*b is then hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo*lo term,
// ~2^-16 relative, is dropped) with FP32 accumulation.
__device__ __forceinline__ void split_bf16(float x, short& hi, short& lo) {
    uint32_t u = __float_as_uint(x);
    uint32_t h = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    hi = short(h >> 16);
    const float r = x - __uint_as_float(h);
    uint32_t v = __float_as_uint(r);
    lo = short((v + 0x7fffu + ((v >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ uint32_t deposit_bits(uint32_t x, const int32_t* pos, int nbits) {
    uint32_t r = 0;
    for (int i = 0; i < nbits; ++i) r |= ((x >> i) & 1u) << pos[i];
    return r;
}

template <int KB, int NB, bool B3>
__global__ void __launch_bounds__(256, 2) k_dense(DenseParams dp, const float2* __restrict__ fin,
                                                  float2* __restrict__ fout, const uint16_t* __restrict__ vids,
                                                  const float2* __restrict__ gtab, uint32_t B_eff,
                                                  uint32_t n_tiles) {
    constexpr int K = 1 << KB, N = 1 << NB;
    constexpr int KS = (2 * K) / 4;       // MFMA k-steps over the real K
    constexpr int NBLK = (2 * N) / 16;    // 16-column blocks over the real N
    constexpr int RS = 2 * (K > N ? K : N) + 2;   // floats per row
    constexpr int BS = 16 * RS + 2;               // floats per bitstring block
    // Cross-tile prefetch of A keeps 2K floats per thread live during the MFMAs;
    // it is used when that fits beside the G fragments (2K/4 * 2N/16 floats)
    // under the two-work-groups-per-CU register budget.  Otherwise the second
    // work-group on the CU overlaps one tile's loads with the other's MFMAs.
    constexpr bool PREFETCH = (KS * NBLK + 2 * K) <= 96;
    constexpr int KS3 = (2 * K) / 16;     // BF16x3: 16x16x16 k-steps over the real K
    __shared__ float tile[16 * BS];
    __shared__ uint32_t sigs[16], pin[16], pout[16];
    __shared__ int order[16];
    __shared__ int sig_start[kDenseMaxVariants + 1];
    __shared__ uint32_t koff[K];

    const StepParams& sp = dp.sp;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int bl = tid & 15, pr = tid >> 4;
    const float2* __restrict__ G = gtab + sp.g_off;
    // per-kernel constants: K offsets, and the input / output offsets of the 16 tile rows
    if (tid < K) koff[tid] = deposit_bits(uint32_t(tid), sp.kpos, KB);
    if (tid < 16) {
        const uint32_t r = deposit_bits(uint32_t(tid), dp.inner_pos, 4);
        uint32_t ri = r;
        for (int i = 0; i < KB; ++i) {
            const uint32_t p = uint32_t(sp.kpos[i]);
            ri = ((ri >> p) << (p + 1)) | (ri & ((1u << p) - 1u));
        }
        pin[tid] = ri;
        pout[tid] = r;
    }
    __syncthreads();
    const uint32_t nbb = B_eff / 16;
    auto tile_base = [&](uint32_t T, uint32_t& base_row, uint32_t& base_in, uint32_t& b0) {
        const uint32_t bb = T % nbb;
        base_row = deposit_bits(T / nbb, dp.outer_pos, dp.n_outer);
        uint32_t ri = base_row;
        for (int i = 0; i < KB; ++i) {
            const uint32_t p = uint32_t(sp.kpos[i]);
            ri = ((ri >> p) << (p + 1)) | (ri & ((1u << p) - 1u));
        }
        base_in = ri;
        b0 = bb * 16;
    };
    // the thread's share of a tile: pairs p = pr + 16 j (j < K) of (row, k), one bitstring bl
    float2 pre[K];
    uint32_t pre_sig = 0;
    auto prefetch = [&](uint32_t T) {
        uint32_t base_row, base_in, b0;
        tile_base(T, base_row, base_in, b0);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int p = pr + 16 * j;
            const int i = p >> KB, k = p & (K - 1);
            if (sp.input_is_one) pre[j] = make_float2(k == 0 ? 1.f : 0.f, 0.f);
            else pre[j] = fin[size_t(base_in + pin[i] + koff[k]) * B_eff + b0 + bl];
        }
        if (tid < 16) pre_sig = vids[b0 + tid];
    };
    uint32_t T = blockIdx.x;
    if (PREFETCH && T < n_tiles) prefetch(T);
    uint32_t cur_sig = 0xffffffffu, cur_v = 0xffffffffu;
    const int n_var = 1 << sp.sb;
    // waves per variant (n_var < 4) or variants per wave (n_var >= 4)
    const int wpv = n_var < 4 ? 4 / n_var : 1;
    float gf[B3 ? 1 : KS][NBLK];
    v4s gh[B3 ? KS3 : 1][NBLK], gl3[B3 ? KS3 : 1][NBLK];
    for (; T < n_tiles; T += gridDim.x) {
        uint32_t base_row, base_in, b0;
        tile_base(T, base_row, base_in, b0);
        uint32_t v = 0;
        for (int i = 0; i < sp.vb; ++i) v |= ((base_row >> sp.vpos[i]) & 1u) << i;
        if (!PREFETCH) prefetch(T);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int p = pr + 16 * j;
            const int i = p >> KB, k = p & (K - 1);
            *reinterpret_cast<float2*>(&tile[bl * BS + i * RS + 2 * k]) = pre[j];
        }
        if (tid < 16) sigs[tid] = pre_sig;
        __syncthreads();
        if (tid < 16) {   // stable order of the 16 bitstrings by sigma
            const uint32_t s = sigs[tid];
            int rank = 0;
            for (int j = 0; j < 16; ++j) rank += (sigs[j] < s) || (sigs[j] == s && j < tid);
            order[rank] = tid;
        }
        if (tid <= n_var) {   // first sorted position of each variant
            int c = 0;
            for (int j = 0; j < 16; ++j) c += sigs[j] < uint32_t(tid);
            sig_start[tid] = c;
        }
        __syncthreads();
        if (PREFETCH && T + gridDim.x < n_tiles) prefetch(T + gridDim.x);   // in flight during the MFMAs
        // wave w multiplies the bitstrings of variant w mod n_var (sharing them with the
        // other waves of that variant), and of w + 4, w + 8, ... when there are more
        // than 4 variants; G fragments stay in VGPRs while (sigma, V) is unchanged
        for (int sig = wave % n_var; sig < n_var; sig += 4) {
            const int lo = sig_start[sig], hi = sig_start[sig + 1];
            if (lo == hi) continue;
            if (uint32_t(sig) != cur_sig || v != cur_v) {
                cur_sig = uint32_t(sig);
                cur_v = v;
                if constexpr (!B3) {
#pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const int kr = 4 * s + (lane >> 4);
                        const int k = kr >> 1, cp = kr & 1;
#pragma unroll
                        for (int nb = 0; nb < NBLK; ++nb) {
                            const int nr = 16 * nb + (lane & 15);
                            const int n = nr >> 1, c = nr & 1;
                            const float2 g = G[(((v * K + uint32_t(k)) * N + uint32_t(n)) << sp.sb) + uint32_t(sig)];
                            gf[s][nb] = cp == 0 ? (c == 0 ? g.x : g.y) : (c == 0 ? -g.y : g.x);
                        }
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < KS3; ++s) {
#pragma unroll
                        for (int nb = 0; nb < NBLK; ++nb) {
                            const int nr = 16 * nb + (lane & 15);
                            const int n = nr >> 1, c = nr & 1;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const int kr = 16 * s + 4 * (lane >> 4) + j;
                                const int k = kr >> 1, cp = kr & 1;
                                const float2 g =
                                    G[(((v * K + uint32_t(k)) * N + uint32_t(n)) << sp.sb) + uint32_t(sig)];
                                const float x = cp == 0 ? (c == 0 ? g.x : g.y) : (c == 0 ? -g.y : g.x);
                                short h, l;
                                split_bf16(x, h, l);
                                gh[s][nb][j] = h;
                                gl3[s][nb][j] = l;
                            }
                        }
                    }
                }
            }
            for (int q = lo + wave / n_var % wpv; q < hi; q += wpv) {
                const int b_l = order[q];
                v4f acc[NBLK];
#pragma unroll
                for (int nb = 0; nb < NBLK; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
                if constexpr (!B3) {
                    const float* arow = &tile[b_l * BS + (lane & 15) * RS + (lane >> 4)];
#pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const float a = arow[4 * s];
#pragma unroll
                        for (int nb = 0; nb < NBLK; ++nb)
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, gf[s][nb], acc[nb], 0, 0, 0);
                    }
                } else {
                    const float* arow = &tile[b_l * BS + (lane & 15) * RS + 4 * (lane >> 4)];
#pragma unroll
                    for (int s = 0; s < KS3; ++s) {
                        const float2 x01 = *reinterpret_cast<const float2*>(arow + 16 * s);
                        const float2 x23 = *reinterpret_cast<const float2*>(arow + 16 * s + 2);
                        v4s ah, al;
                        short h, l;
                        split_bf16(x01.x, h, l); ah[0] = h; al[0] = l;
                        split_bf16(x01.y, h, l); ah[1] = h; al[1] = l;
                        split_bf16(x23.x, h, l); ah[2] = h; al[2] = l;
                        split_bf16(x23.y, h, l); ah[3] = h; al[3] = l;
#pragma unroll
                        for (int nb = 0; nb < NBLK; ++nb) {
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, gh[s][nb], acc[nb], 0, 0, 0);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, gl3[s][nb], acc[nb], 0, 0, 0);
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, gh[s][nb], acc[nb], 0, 0, 0);
                        }
                    }
                }
#pragma unroll
                for (int nb = 0; nb < NBLK; ++nb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 4 * (lane >> 4) + r;
                        tile[b_l * BS + i * RS + 16 * nb + (lane & 15)] = acc[nb][r];
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int p = pr + 16 * j;
            const int i = p >> NB, n = p & (N - 1);
            const float2 c = *reinterpret_cast<const float2*>(&tile[bl * BS + i * RS + 2 * n]);
            fout[size_t(base_row + pout[i] + (uint32_t(n) << sp.row_bits)) * B_eff + b0 + bl] = c;
        }
        __syncthreads();
    }
}

template <int KB, int NB>
static void launch_dense_t(const DenseParams& dp, const float2* fin, float2* fout, const uint16_t* vids,
                           const float2* gtab, uint32_t B_eff, hipStream_t stream) {
    const uint32_t n_tiles = (1u << dp.n_outer) * (B_eff / 16);
    uint32_t grid = n_tiles < kDenseMaxGrid ? n_tiles : kDenseMaxGrid;
    if (dp.bf16x3)
        hipLaunchKernelGGL((k_dense<KB, NB, true>), dim3(grid), dim3(256), 0, stream, dp, fin, fout, vids, gtab, B_eff,
                           n_tiles);
    else
        hipLaunchKernelGGL((k_dense<KB, NB, false>), dim3(grid), dim3(256), 0, stream, dp, fin, fout, vids, gtab, B_eff,
                           n_tiles);
}

template <int KB>
static void launch_dense_nb(int nb, const DenseParams& dp, const float2* fin, float2* fout, const uint16_t* vids,
                            const float2* gtab, uint32_t B_eff, hipStream_t stream) {
    switch (nb) {
        case 3: launch_dense_t<KB, 3>(dp, fin, fout, vids, gtab, B_eff, stream); break;
        case 4: launch_dense_t<KB, 4>(dp, fin, fout, vids, gtab, B_eff, stream); break;
        default: launch_dense_t<KB, 5>(dp, fin, fout, vids, gtab, B_eff, stream); break;
    }
}

void launch_dense(const DenseParams& dp, const float2* fin, float2* fout, const uint16_t* vids, const float2* gtab,
                  uint32_t B_eff, hipStream_t stream) {
    switch (dp.sp.kb) {
        case 3: launch_dense_nb<3>(dp.sp.nb, dp, fin, fout, vids, gtab, B_eff, stream); break;
        case 4: launch_dense_nb<4>(dp.sp.nb, dp, fin, fout, vids, gtab, B_eff, stream); break;
        default: launch_dense_nb<5>(dp.sp.nb, dp, fin, fout, vids, gtab, B_eff, stream); break;
    }
}

}  // namespace qgm
