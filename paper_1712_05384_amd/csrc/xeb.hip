// Cross-entropy benchmarking and sampling from a set of amplitudes (gfx950).
//
// Statistics (App. B): from a batch of amplitudes A(x_j), p_j = |A(x_j)|^2 in
// FP64, the sums over the batch of log p_j, p_j and p_j log p_j and the number
// of zero p_j; from them the cross entropy of the batch taken as a sample of
// the device's output, Eq. (cee), the fidelity estimate of Eq. (ae) with the
// Porter-Thomas values of H_0 and H(p_U), and the entropy estimated from a
// uniformly chosen set (App. C).  Each block sums a contiguous share of the
// batch in a fixed order, one block adds the partial sums in block order: the
// result does not depend on the launch timing.
//
// Sampling from a set (App. C): bitstring j of a uniformly chosen set is drawn
// with probability p_j / sum_k p_k.  The cumulative sums are an FP64 inclusive
// scan (fixed order, as above); draw i takes the caller's uniform u_i in [0, 1)
// and returns the first j whose cumulative sum exceeds u_i times the total.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace qgm {

namespace {

constexpr int kXebThreads = 256;
constexpr int kXebBatch = 8;   // loads a thread issues before it adds them (the order of the adds is kept)
constexpr int kXebMaxBlocks = 1024;                      // blocks of the partial sums and of the scan
constexpr int kXebRun = kXebMaxBlocks / kXebThreads;     // block values per thread of the one-block kernels

__device__ __forceinline__ double prob(const void* amps, int c128, int64_t j) {
    if (c128) {
        const double2 a = static_cast<const double2*>(amps)[j];
        return a.x * a.x + a.y * a.y;
    }
    const float2 a = static_cast<const float2*>(amps)[j];
    const double x = a.x, y = a.y;
    return x * x + y * y;
}

// Natural logarithm of a positive, finite p: p = m 2^e with m in [1/sqrt 2,
// sqrt 2), log p = e log 2 + 2 atanh(s) with s = (m - 1) / (m + 1), |s| <= 0.172,
// and atanh(s) / s = sum_k s^(2k) / (2k + 1) to k = 11 (the omitted terms are
// below 1e-18 relative).  About a third of the instructions of the library's
// double-double logarithm; within a few ulp of it.
__device__ __forceinline__ double log_pos(double p) {
    int e;
    double m = frexp(p, &e);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double q = 1.0 / 23.0;
#pragma unroll
    for (int k = 10; k >= 0; --k) q = fma(q, z, 1.0 / double(2 * k + 1));
    return double(e) * 0.69314718055994530942 + 2.0 * s * q;
}

// Block-wide sum in a fixed order (per-thread values, then a tree over the block).
__device__ double block_sum(double v, double* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kXebThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// Four block-wide sums at once, each in the order of block_sum (the same tree):
// one barrier per tree step for the four.
__device__ void block_sum4(double v[4], double4* lds) {
    lds[threadIdx.x] = make_double4(v[0], v[1], v[2], v[3]);
    __syncthreads();
    for (int s = kXebThreads / 2; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) {
            const double4 a = lds[threadIdx.x], b = lds[threadIdx.x + s];
            lds[threadIdx.x] = make_double4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
        }
        __syncthreads();
    }
    const double4 r = lds[0];
    v[0] = r.x;
    v[1] = r.y;
    v[2] = r.z;
    v[3] = r.w;
    __syncthreads();
}

}  // namespace

// Normalisation of sets of amplitudes (Sec. III.A): block b writes
// sum_o |A(x_b, o)|^2 over the 2^n_open entries of bitstring b, in FP64 and in
// a fixed order (strided per thread, then the block tree).  With every qubit
// open the one set is the whole output distribution, whose sum is 1.
__global__ void __launch_bounds__(kXebThreads) k_prob_sums(const void* __restrict__ amps, int c128, int64_t n_out,
                                                           double* __restrict__ out) {
    __shared__ double lds[kXebThreads];
    const int64_t j0 = int64_t(blockIdx.x) * n_out;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n_out; j += int64_t(kXebThreads) * kXebBatch) {
        double pb[kXebBatch];   // kXebBatch loads in flight, then their adds in order
#pragma unroll
        for (int u = 0; u < kXebBatch; ++u) {
            const int64_t ju = j + int64_t(u) * kXebThreads;
            pb[u] = ju < n_out ? prob(amps, c128, j0 + ju) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kXebBatch; ++u)
            if (j + int64_t(u) * kXebThreads < n_out) s += pb[u];
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Block i sums p over the batch entries [i * chunk, (i + 1) * chunk).  Each
// thread takes the entries j0 + t, j0 + t + 256, ... in that order; it issues
// kXebPartBatch loads before it adds any of them (one memory round trip per
// batch instead of one per entry: a whole 4096-entry chunk in one).
constexpr int kXebPartBatch = 16;
__global__ void __launch_bounds__(kXebThreads) k_xeb_partial(const void* __restrict__ amps, int c128, int64_t B,
                                                             int64_t chunk, double* __restrict__ part) {
    __shared__ double4 lds4[kXebThreads];
    const int64_t j0 = int64_t(blockIdx.x) * chunk, j1 = j0 + chunk < B ? j0 + chunk : B;
    double slog = 0.0, sp = 0.0, splog = 0.0, nzero = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += int64_t(kXebThreads) * kXebPartBatch) {
        double pb[kXebPartBatch];
#pragma unroll
        for (int u = 0; u < kXebPartBatch; ++u) {
            const int64_t ju = j + int64_t(u) * kXebThreads;
            pb[u] = ju < j1 ? prob(amps, c128, ju) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kXebPartBatch; ++u) {
            if (j + int64_t(u) * kXebThreads >= j1) continue;   // beyond the chunk
            const double p = pb[u];
            if (p > 0.0) {
                const double l = log_pos(p);
                slog += l;
                sp += p;
                splog += p * l;
            } else {
                nzero += 1.0;
            }
        }
    }
    double v[4] = {slog, sp, splog, nzero};
    block_sum4(v, lds4);
    if (threadIdx.x == 0) {
        double* o = part + size_t(blockIdx.x) * 4;
        o[0] = v[0];
        o[1] = v[1];
        o[2] = v[2];
        o[3] = v[3];
    }
}

// One block: the sums over the partials (block order), then the estimators.
// out: [0] sum log p, [1] sum p, [2] sum p log p, [3] zeros, [4] cross entropy
// -mean log p over the nonzero entries (Eq. (cee)), [5] fidelity of Eq. (ae)
// with H_0 = n log 2 + gamma and H(p_U) = n log 2 - 1 + gamma, [6] entropy
// estimated from a uniform set, -(2^n / t) sum p log p (App. C), [7] sum p
// times 2^n / t (1 for a uniform set of a normalised state, up to O(1/sqrt t)).
__global__ void __launch_bounds__(kXebThreads) k_xeb_final(const double* __restrict__ part, int n_part, int64_t B,
                                                           int n_qubits, double* __restrict__ out) {
    __shared__ double4 lds4[kXebThreads];
    // each thread adds a contiguous run of at most kXebRun partials (all loaded before the adds), then
    // the tree adds the threads in order
    const int per = (n_part + kXebThreads - 1) / kXebThreads;
    const int i0 = int(threadIdx.x) * per;
    double pv[kXebRun][4];
#pragma unroll
    for (int u = 0; u < kXebRun; ++u)
#pragma unroll
        for (int k = 0; k < 4; ++k) pv[u][k] = u < per && i0 + u < n_part ? part[size_t(i0 + u) * 4 + k] : 0.0;
    double s[4];
    for (int k = 0; k < 4; ++k) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < kXebRun; ++u)
            if (u < per && i0 + u < n_part) v += pv[u][k];
        s[k] = v;
    }
    block_sum4(s, lds4);
    if (threadIdx.x == 0) {
        const double euler_gamma = 0.57721566490153286061;
        const double log_n = double(n_qubits) * 0.69314718055994530942;
        const double m = double(B) - s[3];
        const double ce = m > 0.0 ? -s[0] / m : __builtin_nan("");
        const double h0 = log_n + euler_gamma, hu = log_n - 1.0 + euler_gamma;
        const double scale = exp2(double(n_qubits)) / double(B);
        out[0] = s[0];
        out[1] = s[1];
        out[2] = s[2];
        out[3] = s[3];
        out[4] = ce;
        out[5] = (h0 - ce) / (h0 - hu);
        out[6] = -scale * s[2];
        out[7] = scale * s[1];
    }
}

// Inclusive scan of the per-thread values v over the block (a fixed
// Kogge-Stone tree, so the result does not depend on timing); returns the sum
// of the values of the threads before this one, and the block total in *total.
__device__ double block_exclusive_scan(double v, double* lds, double* total) {
    const int t = int(threadIdx.x);
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kXebThreads; off <<= 1) {
        const double add = t >= off ? lds[t - off] : 0.0;
        __syncthreads();
        if (t >= off) lds[t] += add;
        __syncthreads();
    }
    const double excl = t > 0 ? lds[t - 1] : 0.0;
    *total = lds[kXebThreads - 1];
    __syncthreads();
    return excl;
}

// Inclusive FP64 scan of p: block i scans its chunk in tiles of kScanTile
// entries, writing local sums (from 0 at the chunk's start) and its total.  A
// tile is read with coalesced loads into LDS; thread t adds its run of kScanRun
// consecutive entries in order, the runs are combined by the block scan, and
// the sums leave through LDS with coalesced stores.  LDS rows of kScanRun + 1
// doubles keep the run reads of a wave on distinct banks.
constexpr int kScanRun = 16;
constexpr int kScanTile = kXebThreads * kScanRun;

__device__ __forceinline__ int scan_slot(int e) { return (e / kScanRun) * (kScanRun + 1) + e % kScanRun; }

__global__ void __launch_bounds__(kXebThreads) k_scan_local(const void* __restrict__ amps, int c128, int64_t B,
                                                            int64_t chunk, double* __restrict__ cum,
                                                            double* __restrict__ totals) {
    __shared__ double tile[kXebThreads * (kScanRun + 1)];
    __shared__ double lds[kXebThreads];
    const int t = int(threadIdx.x);
    const int64_t j0 = int64_t(blockIdx.x) * chunk, j1 = j0 + chunk < B ? j0 + chunk : B;
    double carry = 0.0;
    for (int64_t q0 = j0; q0 < j1; q0 += kScanTile) {
        const int n = j1 - q0 < kScanTile ? int(j1 - q0) : kScanTile;
        double pb[kScanRun];
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) {
            const int e = t + u * kXebThreads;
            pb[u] = e < n ? prob(amps, c128, q0 + e) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) tile[scan_slot(t + u * kXebThreads)] = pb[u];
        __syncthreads();
        double v[kScanRun];
        double run = 0.0;
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) v[u] = tile[t * (kScanRun + 1) + u];
#pragma unroll
        for (int u = 0; u < kScanRun; ++u)
            if (t * kScanRun + u < n) run += v[u];
        double total;
        double acc = carry + block_exclusive_scan(run, lds, &total);
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) {
            acc += v[u];
            tile[t * (kScanRun + 1) + u] = acc;   // (entries beyond the tile: never stored below)
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kScanRun; ++u) {
            const int e = t + u * kXebThreads;
            if (e < n) cum[q0 + e] = tile[scan_slot(e)];
        }
        carry += total;
        __syncthreads();
    }
    if (t == 0) totals[blockIdx.x] = carry;
}

// Replaces the block totals by their exclusive prefix sums (one block: thread t
// takes a run of at most kXebMaxBlocks / 256 consecutive totals, the runs by
// the block scan) and writes the grand total after them.

__global__ void __launch_bounds__(kXebThreads) k_scan_offsets(double* __restrict__ totals, int n_blocks) {
    __shared__ double lds[kXebThreads];
    const int per = (n_blocks + kXebThreads - 1) / kXebThreads;   // at most kXebRun
    const int i0 = int(threadIdx.x) * per;
    double v[kXebRun];
    double run = 0.0;
#pragma unroll
    for (int u = 0; u < kXebRun; ++u) v[u] = u < per && i0 + u < n_blocks ? totals[i0 + u] : 0.0;
#pragma unroll
    for (int u = 0; u < kXebRun; ++u)
        if (u < per && i0 + u < n_blocks) run += v[u];
    double total;
    double acc = block_exclusive_scan(run, lds, &total);
#pragma unroll
    for (int u = 0; u < kXebRun; ++u)
        if (u < per && i0 + u < n_blocks) {
            totals[i0 + u] = acc;
            acc += v[u];
        }
    if (threadIdx.x == 0) totals[n_blocks] = total;
}

__global__ void __launch_bounds__(kXebThreads) k_scan_add(double* __restrict__ cum, int64_t B, int64_t chunk,
                                                          const double* __restrict__ totals) {
    const int64_t j = int64_t(blockIdx.x) * kXebThreads + threadIdx.x;
    if (j < B) cum[j] += totals[j / chunk];
}

// One draw per thread and grid-stride step: the first j with cum[j] > u * total
// (the last entry if none), found in two binary searches: over the last sums
// of the scan blocks (copied to LDS by each work-group) for the block that
// holds it, then inside that block: about half of the memory round trips of a
// search over the whole array, and the same index where cum does not decrease
// (it can fall by rounding only from a block's last sum to the next block's
// first, where both indices are within rounding of the target).
constexpr int64_t kSampleMaxBlocks = 1024;   // (8192, one draw per thread: 118 instead of 101 us for 2^20 draws)

__global__ void __launch_bounds__(kXebThreads) k_sample(const double* __restrict__ cum, int64_t B, int64_t chunk,
                                                        const double* __restrict__ totals, int n_blocks,
                                                        const double* __restrict__ u, int64_t m,
                                                        int64_t* __restrict__ idx) {
    __shared__ double last[kXebMaxBlocks];
    for (int b = int(threadIdx.x); b < n_blocks; b += kXebThreads) {
        const int64_t e = (int64_t(b) + 1) * chunk < B ? (int64_t(b) + 1) * chunk : B;
        last[b] = cum[e - 1];
    }
    __syncthreads();
    const double total = totals[n_blocks];
    for (int64_t i = int64_t(blockIdx.x) * kXebThreads + threadIdx.x; i < m;
         i += int64_t(gridDim.x) * kXebThreads) {
        const double target = u[i] * total;
        int lb = 0, hb = n_blocks - 1;
        while (lb < hb) {
            const int mid = lb + (hb - lb) / 2;
            if (last[mid] > target) hb = mid;
            else lb = mid + 1;
        }
        int64_t lo = int64_t(lb) * chunk;
        int64_t hi = (int64_t(lb) + 1) * chunk < B ? (int64_t(lb) + 1) * chunk - 1 : B - 1;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (cum[mid] > target) hi = mid;
            else lo = mid + 1;
        }
        idx[i] = lo;
    }
}

// Work split shared by the launchers and the workspace query.
static int64_t xeb_chunk(int64_t B) {
    const int64_t blocks = B < kXebMaxBlocks * kXebThreads ? (B + kXebThreads - 1) / kXebThreads : kXebMaxBlocks;
    return (B + blocks - 1) / blocks;
}

uint64_t xeb_workspace_bytes(int64_t B) {
    const int64_t chunk = xeb_chunk(B > 0 ? B : 1);
    const int64_t blocks = (B + chunk - 1) / chunk + 1;
    return uint64_t(8 * (B + 4 * blocks + blocks + 1) + 256);
}

void launch_prob_sums(const void* amps, int c128, int64_t B, int64_t n_out, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_prob_sums, dim3(uint32_t(B)), dim3(kXebThreads), 0, stream, amps, c128, n_out, out);
}

void launch_xeb(const void* amps, bool c128, int64_t B, int n_qubits, double* out, double* ws, hipStream_t stream) {
    const int64_t chunk = xeb_chunk(B);
    const int n_part = int((B + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_xeb_partial, dim3(n_part), dim3(kXebThreads), 0, stream, amps, c128 ? 1 : 0, B, chunk, ws);
    hipLaunchKernelGGL(k_xeb_final, dim3(1), dim3(kXebThreads), 0, stream, ws, n_part, B, n_qubits, out);
}

void launch_sample_set(const void* amps, bool c128, int64_t B, const double* u, int64_t m, int64_t* idx, double* ws,
                       hipStream_t stream) {
    const int64_t chunk = xeb_chunk(B);
    const int n_blocks = int((B + chunk - 1) / chunk);
    double* cum = ws;
    double* totals = ws + B;
    hipLaunchKernelGGL(k_scan_local, dim3(n_blocks), dim3(kXebThreads), 0, stream, amps, c128 ? 1 : 0, B, chunk, cum,
                       totals);
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(kXebThreads), 0, stream, totals, n_blocks);
    hipLaunchKernelGGL(k_scan_add, dim3(uint32_t((B + kXebThreads - 1) / kXebThreads)), dim3(kXebThreads), 0, stream,
                       cum, B, chunk, static_cast<const double*>(totals));
    if (m > 0)
        hipLaunchKernelGGL(k_sample, dim3(uint32_t(std::min<int64_t>((m + kXebThreads - 1) / kXebThreads, kSampleMaxBlocks))),
                           dim3(kXebThreads), 0, stream, static_cast<const double*>(cum), B, chunk,
                           static_cast<const double*>(totals), n_blocks, u, m, idx);
}

}  // namespace qgm
