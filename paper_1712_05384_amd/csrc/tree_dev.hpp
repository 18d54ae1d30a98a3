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


constexpr int kTreeMaxPrologueFactors = 64;
constexpr int kTreeMaxPhaseLds = 512;

// The four values of up to kTreeMaxPrologueFactors factors, and the sources
// of their variables, staged in LDS by the whole block.
struct FactorLds {
    double2 v[kTreeMaxPrologueFactors][4];
    int32_t s[kTreeMaxPrologueFactors][4];
};

__device__ __forceinline__ int stage_factors(FactorLds& L, const TFactor* __restrict__ facs, int n_fac,
                                             const double2* __restrict__ fixed, const float2* __restrict__ slots) {
    const int nf = n_fac < kTreeMaxPrologueFactors ? n_fac : kTreeMaxPrologueFactors;
    for (int i = threadIdx.x; i < nf * 4; i += blockDim.x) {
        const TFactor f = facs[i >> 2];
        L.v[i >> 2][i & 3] = factor_value(f, (i >> 1) & 1u, i & 1u, fixed, slots);
        if ((i & 3) == 0) {
            L.s[i >> 2][0] = f.src0;
            L.s[i >> 2][1] = f.bit0;
            L.s[i >> 2][2] = f.src1;
            L.s[i >> 2][3] = f.bit1;
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
            acc = cmuld(acc, L.v[i][val(L.s[i][0], L.s[i][1]) * 2u + val(L.s[i][2], L.s[i][3])]);
        } else {   // beyond the LDS copy: read the record directly
            const TFactor f = facs[i];
            acc = cmuld(acc, factor_value(f, val(f.src0, f.bit0), val(f.src1, f.bit1), fixed, slots));
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
