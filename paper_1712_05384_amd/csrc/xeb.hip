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

#include "kernels.hpp"

namespace qgm {

namespace {

constexpr int kXebThreads = 256;

__device__ __forceinline__ double prob(const void* amps, int c128, int64_t j) {
    if (c128) {
        const double2 a = static_cast<const double2*>(amps)[j];
        return a.x * a.x + a.y * a.y;
    }
    const float2 a = static_cast<const float2*>(amps)[j];
    const double x = a.x, y = a.y;
    return x * x + y * y;
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
    for (int64_t j = threadIdx.x; j < n_out; j += kXebThreads) s += prob(amps, c128, j0 + j);
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Block i sums p over the batch entries [i * chunk, (i + 1) * chunk).
__global__ void __launch_bounds__(kXebThreads) k_xeb_partial(const void* __restrict__ amps, int c128, int64_t B,
                                                             int64_t chunk, double* __restrict__ part) {
    __shared__ double lds[kXebThreads];
    const int64_t j0 = int64_t(blockIdx.x) * chunk, j1 = j0 + chunk < B ? j0 + chunk : B;
    double slog = 0.0, sp = 0.0, splog = 0.0, nzero = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kXebThreads) {
        const double p = prob(amps, c128, j);
        if (p > 0.0) {
            const double l = log(p);
            slog += l;
            sp += p;
            splog += p * l;
        } else {
            nzero += 1.0;
        }
    }
    slog = block_sum(slog, lds);
    sp = block_sum(sp, lds);
    splog = block_sum(splog, lds);
    nzero = block_sum(nzero, lds);
    if (threadIdx.x == 0) {
        double* o = part + size_t(blockIdx.x) * 4;
        o[0] = slog;
        o[1] = sp;
        o[2] = splog;
        o[3] = nzero;
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
    __shared__ double lds[kXebThreads];
    double s[4];
    for (int k = 0; k < 4; ++k) {
        // each thread adds a contiguous run of partials, then the tree adds the threads in order
        const int per = (n_part + kXebThreads - 1) / kXebThreads;
        double v = 0.0;
        for (int i = int(threadIdx.x) * per; i < (int(threadIdx.x) + 1) * per && i < n_part; ++i) v += part[size_t(i) * 4 + k];
        s[k] = block_sum(v, lds);
    }
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

// Inclusive FP64 scan of p: block i scans its chunk (one thread per run of
// entries, then the run totals in order), writing local sums and its total.
__global__ void __launch_bounds__(kXebThreads) k_scan_local(const void* __restrict__ amps, int c128, int64_t B,
                                                            int64_t chunk, double* __restrict__ cum,
                                                            double* __restrict__ totals) {
    __shared__ double lds[kXebThreads];
    const int64_t j0 = int64_t(blockIdx.x) * chunk, j1 = j0 + chunk < B ? j0 + chunk : B;
    const int64_t per = (chunk + kXebThreads - 1) / kXebThreads;
    const int64_t r0 = j0 + int64_t(threadIdx.x) * per, r1 = r0 + per < j1 ? r0 + per : j1;
    double run = 0.0;
    for (int64_t j = r0; j < r1; ++j) run += prob(amps, c128, j);
    lds[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {   // exclusive offsets of the runs, in order
        double acc = 0.0;
        for (int i = 0; i < kXebThreads; ++i) {
            const double v = lds[i];
            lds[i] = acc;
            acc += v;
        }
        totals[blockIdx.x] = acc;
    }
    __syncthreads();
    double acc = lds[threadIdx.x];
    for (int64_t j = r0; j < r1; ++j) {
        acc += prob(amps, c128, j);
        cum[j] = acc;
    }
}

// Adds the exclusive prefix of the block totals (one block, in order) to every entry.
__global__ void __launch_bounds__(kXebThreads) k_scan_offsets(double* __restrict__ totals, int n_blocks) {
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int i = 0; i < n_blocks; ++i) {
            const double v = totals[i];
            totals[i] = acc;
            acc += v;
        }
        totals[n_blocks] = acc;
    }
}

__global__ void __launch_bounds__(kXebThreads) k_scan_add(double* __restrict__ cum, int64_t B, int64_t chunk,
                                                          const double* __restrict__ totals) {
    const int64_t j = int64_t(blockIdx.x) * kXebThreads + threadIdx.x;
    if (j < B) cum[j] += totals[j / chunk];
}

__global__ void __launch_bounds__(kXebThreads) k_sample(const double* __restrict__ cum, int64_t B,
                                                        const double* __restrict__ totals, int n_blocks,
                                                        const double* __restrict__ u, int64_t m,
                                                        int64_t* __restrict__ idx) {
    const int64_t i = int64_t(blockIdx.x) * kXebThreads + threadIdx.x;
    if (i >= m) return;
    const double target = u[i] * totals[n_blocks];
    int64_t lo = 0, hi = B - 1;   // first j with cum[j] > target (the last entry if none)
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cum[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    idx[i] = lo;
}

// Work split shared by the launchers and the workspace query.
static int64_t xeb_chunk(int64_t B) {
    const int64_t blocks = B < 1024 * kXebThreads ? (B + kXebThreads - 1) / kXebThreads : 1024;
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
        hipLaunchKernelGGL(k_sample, dim3(uint32_t((m + kXebThreads - 1) / kXebThreads)), dim3(kXebThreads), 0, stream,
                           static_cast<const double*>(cum), B, static_cast<const double*>(totals), n_blocks, u, m, idx);
}

}  // namespace qgm
