// Device helpers shared by the bucket-elimination kernels (forward and
// adjoint): complex arithmetic, gate-factor values, factor staging in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace qgm {
namespace tree_dev {

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

// Value of a two-qubit gate factor (TF_MAT4) at argument index
// a4 = 8 a0 + 4 a1 + 2 c0 + c1: M[2 a0 + a1][2 c0 + c1], rows in consecutive slots.
__device__ __forceinline__ double2 factor_value4(const TFactor& f, uint32_t a4, const float2* __restrict__ slots) {
    const float2 m = slots[size_t(f.mat - kFixedMats) * 4 + a4];
    return make_double2(m.x, m.y);
}

// Value of any factor for argument index a4 (its variables' values, first
// variable most significant: 2 bits, or 4 for TF_MAT4).
__device__ __forceinline__ double2 factor_value_any(const TFactor& f, uint32_t a4, const double2* __restrict__ fixed,
                                                    const float2* __restrict__ slots) {
    if (f.type == TF_MAT4) return factor_value4(f, a4, slots);
    return factor_value(f, (a4 >> 1) & 1u, a4 & 1u, fixed, slots);
}

// A factor without free variables for bitstring x, from its record.
__device__ __forceinline__ double2 phase_factor(const TFactor& f, uint64_t x, const double2* __restrict__ fixed,
                                                const float2* __restrict__ slots) {
    auto bit = [&](int32_t src, int32_t b) { return src == TS_SIG ? uint32_t((x >> b) & 1ull) : 0u; };
    uint32_t a4 = bit(f.src0, f.bit0) * 2u + bit(f.src1, f.bit1);
    if (f.type == TF_MAT4) a4 = a4 * 4u + bit(f.src2, f.bit2) * 2u + bit(f.src3, f.bit3);
    return factor_value_any(f, a4, fixed, slots);
}

constexpr int kTreeMaxPrologueFactors = 64;
constexpr int kTreeMaxPhaseLds = 512;

// The values of up to kTreeMaxPrologueFactors factors (4, or 16 for a
// two-qubit gate), and the sources of their variables, staged in LDS by the
// whole block.
struct FactorLds {
    double2 v[kTreeMaxPrologueFactors][16];
    int32_t s[kTreeMaxPrologueFactors][8];
    int32_t four[kTreeMaxPrologueFactors];
};

__device__ __forceinline__ int stage_factors(FactorLds& L, const TFactor* __restrict__ facs, int n_fac,
                                             const double2* __restrict__ fixed, const float2* __restrict__ slots) {
    const int nf = n_fac < kTreeMaxPrologueFactors ? n_fac : kTreeMaxPrologueFactors;
    for (int i = threadIdx.x; i < nf * 16; i += blockDim.x) {
        const TFactor f = facs[i >> 4];
        const uint32_t a4 = uint32_t(i & 15);
        if (f.type == TF_MAT4 || a4 < 4u) L.v[i >> 4][a4] = factor_value_any(f, a4, fixed, slots);
        if (a4 == 0) {
            L.s[i >> 4][0] = f.src0;
            L.s[i >> 4][1] = f.bit0;
            L.s[i >> 4][2] = f.src1;
            L.s[i >> 4][3] = f.bit1;
            L.s[i >> 4][4] = f.src2;
            L.s[i >> 4][5] = f.bit2;
            L.s[i >> 4][6] = f.src3;
            L.s[i >> 4][7] = f.bit3;
            L.four[i >> 4] = f.type == TF_MAT4 ? 1 : 0;
        }
    }
    __syncthreads();
    return nf;
}

// Product of factors [f0, f1) of a table for index c, output bits sig and a
// group's own summed value iv (FP64).
__device__ __forceinline__ double2 factor_product(const FactorLds& L, int nf, const TFactor* __restrict__ facs,
                                                  int f0, int f1, const double2* __restrict__ fixed,
                                                  const float2* __restrict__ slots, uint32_t c, uint32_t sig,
                                                  uint32_t iv) {
    auto val = [&](int32_t src, int32_t bit) -> uint32_t {
        switch (src) {
            case TS_G: return (c >> bit) & 1u;
            case TS_SIG: return (sig >> bit) & 1u;
            case TS_INT: return (iv >> bit) & 1u;
            default: return 0u;
        }
    };
    double2 acc = make_double2(1.0, 0.0);
    for (int i = f0; i < f1; ++i) {
        if (i < nf) {
            uint32_t a4 = val(L.s[i][0], L.s[i][1]) * 2u + val(L.s[i][2], L.s[i][3]);
            if (L.four[i]) a4 = a4 * 4u + val(L.s[i][4], L.s[i][5]) * 2u + val(L.s[i][6], L.s[i][7]);
            acc = cmuld(acc, L.v[i][a4]);
        } else {   // beyond the LDS copy: read the record directly
            const TFactor f = facs[i];
            uint32_t a4 = val(f.src0, f.bit0) * 2u + val(f.src1, f.bit1);
            if (f.type == TF_MAT4) a4 = a4 * 4u + val(f.src2, f.bit2) * 2u + val(f.src3, f.bit3);
            acc = cmuld(acc, factor_value_any(f, a4, fixed, slots));
        }
    }
    return acc;
}

__device__ __forceinline__ uint32_t gather_sigma(uint64_t x, const int32_t* q, int n) {
    uint32_t sig = 0;
#pragma unroll
    for (int i = 0; i < kTreeMaxSig; ++i)
        if (i < n) sig |= uint32_t((x >> q[i]) & 1ull) << i;
    return sig;
}

}  // namespace tree_dev
}  // namespace qgm
