// LDS-resident bucket elimination (qgm_amplitudes with tree_exec 3, gfx950).
//
// Work-group b evaluates App. A's buckets for bitstring b alone: every result
// of the elimination tree lives in the work-group's LDS, so the launch reads
// from HBM only the bitstring, the table entries at its output bits (the
// deltas of Eq. (psi_x) select them) and its job records, and writes one
// amplitude.  The waves share each level's jobs (64 result rows of one bucket,
// one row per lane, or 128 or 256 with two or four rows per lane): lane l
// multiplies the factor-table entry of its row and summed value w by its
// input rows, sums over w, and stores the row; a block barrier separates
// levels, as a level reads only results of earlier levels.  A job record
// holds the lane offsets of its first row (per input and for the table, two
// 8-entry tables by three-bit groups of the lane) and the strides of result
// bits 6 and 7; the records are copied to LDS with the tables when they fit,
// so after the first burst of loads the levels touch no memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.hpp"
#include "tree_dev.hpp"

namespace qgm {

using namespace tree_dev;

namespace {

// 16 bytes of a job record (LDS or memory; the address is wave-uniform).
__device__ __forceinline__ uint4 rec16(const char* __restrict__ rp, int byte) {
    return *reinterpret_cast<const uint4*>(rp + byte);
}
__device__ __forceinline__ uint32_t half(uint4 v, int i) {   // 16-bit field i of a 16-byte word
    const uint32_t d = (i >> 1) == 0 ? v.x : (i >> 1) == 1 ? v.y : (i >> 1) == 2 ? v.z : v.w;
    return (i & 1) ? d >> 16 : d & 0xFFFFu;
}

// Lane offset of slot s: the record's entry for the lane's bits 0-2 (which
// includes the slot's base) plus its entry for bits 3-5; lo and hi are the
// record addresses of the lane's entries of slot 0 (2 (l & 7) and
// 16 + 2 (l >> 3) bytes past the tables), so each entry is one 16-bit load.
__device__ __forceinline__ uint32_t lane_off(const char* __restrict__ lo, const char* __restrict__ hi, int s) {
    return uint32_t(*reinterpret_cast<const uint16_t*>(lo + 32 * s)) +
           uint32_t(*reinterpret_cast<const uint16_t*>(hi + 32 * s));
}

// One job: rows out_row + 64 m + lane of its bucket's result for m < M (lanes
// < the record's count; row m's slot offsets add the record's strides of
// result bits 6 and 7 for the bits of m); h is the record's first 16 bytes, rp
// the record, L the work-group's LDS.
template <int NIN, int K, int M>
__device__ __forceinline__ void lds_job(uint4 h, uint32_t lanes, const char* __restrict__ rp, char* __restrict__ L,
                                        const uint32_t (&lb)[2], uint32_t lane) {
    constexpr int W = 1 << K;
    constexpr int NR = NIN > 0 ? NIN : 1;
    const uint4 tw = rec16(rp, 16);
    uint4 iw[NR];
#pragma unroll
    for (int t = 0; t < NIN; ++t) iw[t] = rec16(rp, 32 + 16 * t);
    uint32_t row[M][NR], tb[M];
    const char* __restrict__ lo = rp + 96 + lb[0];
    const char* __restrict__ hi = rp + 96 + lb[1];
#pragma unroll
    for (int t = 0; t < NIN; ++t) row[0][t] = lane_off(lo, hi, t);
    tb[0] = lane_off(lo, hi, kLdsMaxIn);
    if constexpr (M >= 2) {
        const uint4 s6 = rec16(rp, 256);
#pragma unroll
        for (int t = 0; t < NIN; ++t) row[1][t] = row[0][t] + half(s6, t);
        tb[1] = tb[0] + half(s6, kLdsMaxIn);
    }
    if constexpr (M == 4) {
        const uint4 s7 = rec16(rp, 272);
#pragma unroll
        for (int m = 2; m < 4; ++m) {
#pragma unroll
            for (int t = 0; t < NIN; ++t) row[m][t] = row[m - 2][t] + half(s7, t);
            tb[m] = tb[m - 2] + half(s7, kLdsMaxIn);
        }
    }
    // every load of a job with at most kLdsBatchLoads loads per row (half as many with four rows) is issued
    // before the first product: the values pass through empty asm statements, so the compiler cannot
    // interleave the loads with the arithmetic (one LDS round trip per job instead of one per summed value).
    // A larger job takes its rows one after the other (each row's store precedes the next row's loads, which
    // may read the same LDS), so its registers stay those of one row.
    constexpr bool BATCH = lds_batched(NIN, K, M == 4 ? 2 : M - 1);
    constexpr int MB = BATCH ? M : 1;
#pragma unroll
    for (int m0 = 0; m0 < M; m0 += MB) {
        float2 q[MB][W], v[MB][NR][W];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
#pragma unroll
            for (int w = 0; w < W; ++w) q[m][w] = *reinterpret_cast<const float2*>(L + tb[m0 + m] + half(tw, w));
#pragma unroll
            for (int t = 0; t < NIN; ++t)
#pragma unroll
                for (int w = 0; w < W; ++w)
                    v[m][t][w] = *reinterpret_cast<const float2*>(L + row[m0 + m][t] + half(iw[t], w));
        }
        if constexpr (BATCH) {
#pragma unroll
            for (int m = 0; m < MB; ++m) {
#pragma unroll
                for (int w = 0; w < W; ++w) asm volatile("" : "+v"(q[m][w].x), "+v"(q[m][w].y));
#pragma unroll
                for (int t = 0; t < NIN; ++t)
#pragma unroll
                    for (int w = 0; w < W; ++w) asm volatile("" : "+v"(v[m][t][w].x), "+v"(v[m][t][w].y));
            }
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                if constexpr (NIN == 0) {
                    acc.x += q[m][w].x;
                    acc.y += q[m][w].y;
                } else {
                    float2 pw = q[m][w];
#pragma unroll
                    for (int t = 0; t + 1 < NIN; ++t) pw = cmulf(pw, v[m][t][w]);
                    const float2 l = v[m][NIN - 1][w];   // the last factor enters the sum as fused multiply-adds
                    acc.x = fmaf(pw.x, l.x, acc.x);
                    acc.x = fmaf(-pw.y, l.y, acc.x);
                    acc.y = fmaf(pw.x, l.y, acc.y);
                    acc.y = fmaf(pw.y, l.x, acc.y);
                }
            }
            if (lane < lanes) *reinterpret_cast<float2*>(L + (h.x >> 16) + 512 * (m0 + m) + 8 * lane) = acc;
        }
    }
}

template <int NIN, int K>
__device__ __forceinline__ void lds_job_m(int rl, uint4 h, uint32_t lanes, const char* __restrict__ rp,
                                          char* __restrict__ L, const uint32_t (&lb)[2], uint32_t lane) {
    // rows per lane up to the planner's limit for this shape (the other cases are never recorded)
    constexpr int R = lds_max_rl(NIN, K);
    if (R >= 2 && rl == 2) lds_job<NIN, K, R >= 2 ? 4 : 1>(h, lanes, rp, L, lb, lane);
    else if (R >= 1 && rl >= 1) lds_job<NIN, K, R >= 1 ? 2 : 1>(h, lanes, rp, L, lb, lane);
    else lds_job<NIN, K, 1>(h, lanes, rp, L, lb, lane);
}

template <int NIN>
__device__ __forceinline__ void lds_job_k(int k, int rl, uint4 h, uint32_t lanes, const char* __restrict__ rp,
                                          char* __restrict__ L, const uint32_t (&lb)[2], uint32_t lane) {
    switch (k) {
        case 0: lds_job_m<NIN, 0>(rl, h, lanes, rp, L, lb, lane); break;
        case 1: lds_job_m<NIN, 1>(rl, h, lanes, rp, L, lb, lane); break;
        case 2: lds_job_m<NIN, 2>(rl, h, lanes, rp, L, lb, lane); break;
        default: lds_job_m<NIN, 3>(rl, h, lanes, rp, L, lb, lane); break;
    }
}

// The FP64 product of the factors without free variables for bitstring x, on
// one wave, in a fixed order: lane partial products (factor i on lane i mod 64)
// from lane_phase, then a butterfly (phase_butterfly) whose lane-0 result is
// written to *phase_v.  The first 64 factors' values (pv0..pv3 at the bits pq)
// come from the launch's first burst of loads; a two-qubit gate's factor is
// evaluated from its record.
__device__ __forceinline__ double2 lane_phase(const LdsArgs& a, uint64_t x, uint32_t lane, int2 pq, double2 pv0,
                                              double2 pv1, double2 pv2, double2 pv3) {
    double2 ph = make_double2(1.0, 0.0);
    if (int(lane) < a.n_phase) {
        const uint32_t e = (pq.x >= 0 ? uint32_t((x >> pq.x) & 1ull) * 2u : 0u) +
                           (pq.y >= 0 ? uint32_t((x >> pq.y) & 1ull) : 0u);
        ph = e == 0 ? pv0 : e == 1 ? pv1 : e == 2 ? pv2 : pv3;
        if (pq.x == -2) ph = phase_factor(a.phase[lane], x, a.fixed, a.slots);
    }
    for (int i = int(lane) + 64; i < a.n_phase; i += 64) {   // more than 64 phase factors
        const int2 q = reinterpret_cast<const int2*>(a.phq)[i];
        const uint32_t e = (q.x >= 0 ? uint32_t((x >> q.x) & 1ull) * 2u : 0u) +
                           (q.y >= 0 ? uint32_t((x >> q.y) & 1ull) : 0u);
        ph = cmuld(ph, q.x == -2 ? phase_factor(a.phase[i], x, a.fixed, a.slots) : a.pv[4 * i + e]);
    }
    return ph;
}

__device__ __forceinline__ void phase_butterfly(double2 ph, uint32_t lane, double2* phase_v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const double2 o = make_double2(__shfl_xor(ph.x, m, 64), __shfl_xor(ph.y, m, 64));
        ph = cmuld(ph, o);
    }
    if (lane == 0) *phase_v = ph;
}

}  // namespace

// The launch: work-group b evaluates bitstring b with NT threads; RL: the job
// records are in LDS (copied with the tables), else read from memory.  LDS (all
// of it dynamic, so record offsets are absolute): the output bits of each table
// slice, the FP64 phase, then the data (results, table slices, job records).
template <int NT, bool RL>
__global__ void __launch_bounds__(NT) k_tree_lds(const LdsArgs a) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) char L[];
    uint32_t* sig = reinterpret_cast<uint32_t*>(L);
    double2* phase_v = reinterpret_cast<double2*>(L + 4 * kLdsMaxStages);
    float2* data = reinterpret_cast<float2*>(L + kLdsHeader);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b = blockIdx.x;
    const uint64_t x = a.bits[b];
    // Everything the levels read from memory, in one burst of loads issued before any is waited for: the
    // table entries' descriptors and the job records (independent of the bitstring; records as 16-byte
    // words), the stage records, the phase factors' values.  Indices are clamped to valid entries (the
    // arrays are never empty), so no load is conditional.
    constexpr int R = 4;
    const int n_e = a.n_entries;
    uint32_t en[R];
#pragma unroll
    for (int i = 0; i < R; ++i) en[i] = a.zent[uint32_t(min(i * NT + int(tid), max(n_e - 1, 0)))];
    const int n_rw = RL ? a.n_jobs * (kLdsRecordBytes / 16) : 0;
    const uint4* __restrict__ rsrc = reinterpret_cast<const uint4*>(a.recs);
    uint4* rdst = reinterpret_cast<uint4*>(L + kLdsHeader + 8 * a.recs0);
    uint4 rw[R];
#pragma unroll
    for (int i = 0; i < R; ++i) rw[i] = rsrc[min(i * NT + int(tid), max(n_rw - 1, 0))];
#pragma unroll
    for (int i = 0; i < R; ++i) asm volatile("" : "+v"(rw[i].x), "+v"(rw[i].y), "+v"(rw[i].z), "+v"(rw[i].w));
    // the stage record of stage tid (n_sig, then the 12 qubits)
    static_assert(sizeof(LdsStage) == 64 && kTreeMaxSig == 12, "stage records are four 16-byte words");
    const int4* sp = reinterpret_cast<const int4*>(a.stages + min(int(tid), max(a.n_stages - 1, 0)));
    const int4 sh0 = sp[0], sq0 = sp[1], sq1 = sp[2], sq2 = sp[3];
    // the phase factor of lane tid of the last wave: the bits its variables read and its 4 FP64 values (its
    // product is formed in the last level)
    const int ip = min(int(lane), max(a.n_phase - 1, 0));
    const int2 pq = reinterpret_cast<const int2*>(a.phq)[ip];
    const double2 pv0 = a.pv[4 * ip], pv1 = a.pv[4 * ip + 1], pv2 = a.pv[4 * ip + 2], pv3 = a.pv[4 * ip + 3];
    // now the values
    const double2 ph = wave == NW - 1 ? lane_phase(a, x, lane, pq, pv0, pv1, pv2, pv3) : make_double2(1.0, 0.0);
    if (int(tid) < a.n_stages) {
        const int q[12] = {sq0.x, sq0.y, sq0.z, sq0.w, sq1.x, sq1.y, sq1.z, sq1.w, sq2.x, sq2.y, sq2.z, sq2.w};
        uint32_t g = 0;
#pragma unroll
        for (int i = 0; i < 12; ++i)
            if (i < sh0.x) g |= uint32_t((x >> q[i]) & 1ull) << i;
        sig[tid] = a.staged ? g * uint32_t(sh0.y) : g;   // the slice's offset in its staged block, or sigma
    }
    for (int s2 = int(tid) + NT; s2 < a.n_stages; s2 += NT) {   // more stages than threads
        const LdsStage& st = a.stages[s2];
        sig[s2] = gather_sigma(x, st.sig_q, st.n_sig) * (a.staged ? uint32_t(st.n) : 1u);
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
        if (i * NT + int(tid) < n_rw) rdst[i * NT + int(tid)] = rw[i];
    for (int i = R * NT + int(tid); i < n_rw; i += NT) rdst[i] = rsrc[i];   // more record words than one round
    __syncthreads();
    // the table slices from the staged copy (consecutive entries of a slice are consecutive there): R entries
    // per thread per round, every load issued before any store
    for (int e0 = 0; e0 < n_e;) {
        uint32_t sg[R];
#pragma unroll
        for (int i = 0; i < R; ++i) sg[i] = sig[en[i] >> 24];
        float2 v[R];
#pragma unroll
        for (int i = 0; i < R; ++i)   // staged index < 2^24: a 32-bit byte offset from the copy's base
            v[i] = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(a.ztab) +
                                                    (((en[i] & 0xFFFFFFu) + sg[i]) << 3));
        const int e1 = e0 + R * NT;
        if (e1 < n_e) {
#pragma unroll
            for (int i = 0; i < R; ++i) en[i] = a.zent[uint32_t(min(e1 + i * NT + int(tid), n_e - 1))];
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int e = e0 + i * NT + int(tid);
            if (e < n_e) data[a.tables0 + e] = v[i];
        }
        e0 = e1;
    }
    // the byte offsets of the lane's entries in a record's lane-offset tables (bits 0-2, bits 3-5)
    const uint32_t lb[2] = {2u * (lane & 7u), 16u + 2u * (lane >> 3)};
    const char* __restrict__ recs = RL ? L + kLdsHeader + 8 * a.recs0 : reinterpret_cast<const char*>(a.recs);
    __syncthreads();
    for (int lv = 0; lv < a.n_levels; ++lv) {
        const int j1 = a.level_job_off[lv + 1];
        for (int j = a.level_job_off[lv] + int(wave); j < j1; j += NW) {
            const char* __restrict__ rp = recs + j * kLdsRecordBytes;
            const uint4 h = rec16(rp, 0);
            const uint32_t hd = __builtin_amdgcn_readfirstlane(h.x & 0xFFFFu);
            const uint32_t lanes = ((hd >> 5) & 63u) + 1u;
            const int k = int((hd >> 3) & 3u);
            const int rl = int((hd >> 11) & 3u);
            switch (hd & 7u) {
                case 0: lds_job_k<0>(k, rl, h, lanes, rp, L, lb, lane); break;
                case 1: lds_job_k<1>(k, rl, h, lanes, rp, L, lb, lane); break;
                case 2: lds_job_k<2>(k, rl, h, lanes, rp, L, lb, lane); break;
                case 3: lds_job_k<3>(k, rl, h, lanes, rp, L, lb, lane); break;
                default: lds_job_k<4>(k, rl, h, lanes, rp, L, lb, lane); break;
            }
        }
        // the phase product on the last wave during the last level (it usually has no job there)
        if (lv == a.n_levels - 1 && wave == NW - 1) phase_butterfly(ph, lane, phase_v);
        __syncthreads();
    }
    if (a.n_levels == 0) {
        if (wave == NW - 1) phase_butterfly(ph, lane, phase_v);
        __syncthreads();
    }
    if (tid == 0) {
        double2 acc = *phase_v;
        for (int f = 0; f < a.n_final; ++f) {
            const float2 r = *reinterpret_cast<const float2*>(L + a.finals[f]);
            acc = cmuld(acc, make_double2(r.x, r.y));
        }
        if (a.c128) static_cast<double2*>(a.out)[b] = acc;
        else static_cast<float2*>(a.out)[b] = make_float2(float(acc.x), float(acc.y));
    }
}

__global__ void __launch_bounds__(256) k_lds_stage(const LdsStage* __restrict__ stages,
                                                   const LdsEntry* __restrict__ entries,
                                                   const float2* __restrict__ gtab, float2* __restrict__ z) {
    const LdsStage st = stages[blockIdx.y];
    const int64_t m = int64_t(st.n) << st.n_sig;
    const int lg = __ffs(st.n) - 1;   // n is a power of two
    for (int64_t idx = int64_t(blockIdx.x) * 256 + threadIdx.x; idx < m; idx += int64_t(gridDim.x) * 256) {
        const int64_t sg = idx >> lg, i = idx & (st.n - 1);
        z[st.zoff + idx] = gtab[int64_t(entries[st.e0 + i].src) + sg];
    }
}

void launch_lds_stage(const LdsStage* stages, int n_stages, const LdsEntry* entries, const float2* gtab, float2* z,
                      int64_t max_m, hipStream_t stream) {
    if (n_stages <= 0 || max_m <= 0) return;
    const uint32_t gx = uint32_t(std::min<int64_t>((max_m + 255) / 256, 64));
    hipLaunchKernelGGL(k_lds_stage, dim3(gx, uint32_t(n_stages)), dim3(256), 0, stream, stages, entries, gtab, z);
}

namespace {

// The launch's kernel for a work-group size and record placement.
const void* lds_kernel(int threads, bool rl) {
    constexpr int S = kLdsSmallThreads, G = kLdsLargeThreads;
    if (threads == G) return rl ? reinterpret_cast<const void*>(&k_tree_lds<G, true>)
                                : reinterpret_cast<const void*>(&k_tree_lds<G, false>);
    return rl ? reinterpret_cast<const void*>(&k_tree_lds<S, true>) : reinterpret_cast<const void*>(&k_tree_lds<S, false>);
}

// Work-groups of the launch that one compute unit holds at once (registers and
// LDS, the runtime's occupancy figure) times the device's compute units, per
// device, kernel and LDS size; 0 if the runtime does not say.
int64_t lds_resident_groups(int threads, bool rl, size_t sh) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    static std::mutex mu;
    static std::map<std::tuple<int, int, bool, size_t>, int64_t> cache;
    const auto key = std::make_tuple(dev, threads, rl, sh);
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lds_kernel(threads, rl), threads, sh) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 0;
    }
    return cache[key] = int64_t(per_cu) * cus;
}

}  // namespace

// Job records in LDS (one LDS round trip per job instead of a memory one)
// while every work-group of the call is resident at once; in memory when the
// batch takes more than one round of work-groups and the LDS they free lets a
// compute unit hold more work-groups (5x5 depth 25: 11.4 vs 11.8 us at 1024
// bitstrings with the records in LDS, 390 vs 413 us at 65536 with them in
// memory).
void launch_tree_lds(const LdsArgs& a0, hipStream_t stream) {
    if (a0.B <= 0) return;
    LdsArgs a = a0;
    if (a0.recs0 >= 0) {
        const size_t with = size_t(kLdsHeader) + size_t(a0.lds_size) * sizeof(float2);
        const size_t without = size_t(kLdsHeader) + size_t(a0.recs0) * sizeof(float2);
        const int64_t g_with = lds_resident_groups(a0.threads, true, with);
        if (g_with > 0 && int64_t(a0.B) > g_with && lds_resident_groups(a0.threads, false, without) > g_with) {
            a.recs0 = -1;            // the kernel reads the records from the plan's tables
            a.lds_size = a0.recs0;   // (the LDS data ends where the records would start)
        }
    }
    const size_t sh = size_t(kLdsHeader) + size_t(a.lds_size) * sizeof(float2);
    const dim3 g(uint32_t(a.B));
    constexpr int S = kLdsSmallThreads, G = kLdsLargeThreads;
    const bool rl = a.recs0 >= 0;
    if (a.threads == G && rl) hipLaunchKernelGGL((k_tree_lds<G, true>), g, dim3(G), sh, stream, a);
    else if (a.threads == G) hipLaunchKernelGGL((k_tree_lds<G, false>), g, dim3(G), sh, stream, a);
    else if (rl) hipLaunchKernelGGL((k_tree_lds<S, true>), g, dim3(S), sh, stream, a);
    else hipLaunchKernelGGL((k_tree_lds<S, false>), g, dim3(S), sh, stream, a);
}

}  // namespace qgm
