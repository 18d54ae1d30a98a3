// The LDS-resident program of a bucket plan (qgm_amplitudes, tree_exec 3).
//
// App. A's buckets are evaluated for one bitstring at a time by one
// work-group: every result of the elimination tree lives in LDS (rows packed
// by lifetime, as the HBM arena of the level launches), and the factor tables
// and leaf tables, which depend on the bitstring only through its output bits
// (the deltas of Eq. (psi_x)), are copied to LDS at those bits before the first
// level.  A job is 64, 128 or 256 consecutive result rows of one bucket (1, 2
// or 4 rows per lane, chosen per level so that a level's jobs take one pass
// of the waves where they can); its record holds, per input and for the
// table, the lane offsets of its first row by three-bit groups of the lane
// (two 16-bit loads and an add give a lane's offset) and the strides of
// result bits 6 and 7.  The records are copied to LDS with the tables when
// they fit, so a job reads no memory.
//
// Layout in LDS: a tensor's variables in decreasing order of elimination (the
// variable eliminated last is axis 0), a factor table indexed (w << gb) | g
// with g over its variables in that same order.  A bucket's result variables
// are eliminated after its summed ones, so in every input they come first and
// in the result's order: the low result axes (the lanes) are the low axes of
// each input and of the table, and the 64 lanes of a job touch consecutive
// entries (or share one), which keeps LDS reads free of bank conflicts.
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "tree.hpp"

namespace qgm {

namespace {

// Index of variable v in axes (-1: absent).
int axis_of(const std::vector<int>& axes, int v) {
    for (size_t i = 0; i < axes.size(); ++i)
        if (axes[i] == v) return int(i);
    return -1;
}

// The index in layout `from` of the entry whose index in layout `to` is i
// (both orders of the same variables).
int64_t relayout(int64_t i, const std::vector<int>& to, const std::vector<int>& from) {
    int64_t o = 0;
    for (size_t k = 0; k < to.size(); ++k)
        if ((i >> k) & 1) o |= int64_t(1) << axis_of(from, to[k]);
    return o;
}

// Orders the jobs [j0, j1) of one level for the kernel's fixed assignment (wave
// w takes the level's jobs w, w + W, w + 2W, ...): longest first, each to the
// least loaded wave that still takes a job in the assignment (waves 0 .. m - 1
// take one more than the rest when W does not divide the count), then the
// jobs in pass order.  The cost of a job is its loads per lane (rows per lane
// x (inputs + table) x summed values) plus a fixed part for the record and
// the lane offsets.
void order_level_jobs(LdsProgram& P, int32_t j0, int32_t j1, int W) {
    const int n = j1 - j0;
    if (n <= W) return;   // one pass: every job on a wave of its own
    auto cost = [&](int32_t j) {
        const LdsJob& jb = P.jobs[size_t(j)];
        return 16 + (1 << jb.rl) * (jb.nin + 1) * (1 << jb.k);
    };
    std::vector<int32_t> idx;
    for (int32_t j = j0; j < j1; ++j) idx.push_back(j);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
    const int full = n / W, extra = n % W;
    std::vector<std::vector<int32_t>> wave(static_cast<size_t>(W));
    std::vector<int64_t> load(static_cast<size_t>(W), 0);
    for (int32_t j : idx) {
        int best = -1;
        for (int w = 0; w < W; ++w) {
            const int cap = full + (w < extra ? 1 : 0);
            if (int(wave[size_t(w)].size()) < cap && (best < 0 || load[size_t(w)] < load[size_t(best)])) best = w;
        }
        wave[size_t(best)].push_back(j);
        load[size_t(best)] += cost(j);
    }
    std::vector<LdsJob> jobs;
    std::vector<int32_t> bucket;
    for (int pass = 0; pass <= full; ++pass)
        for (int w = 0; w < W; ++w)
            if (pass < int(wave[size_t(w)].size())) {
                jobs.push_back(P.jobs[size_t(wave[size_t(w)][size_t(pass)])]);
                bucket.push_back(P.job_bucket[size_t(wave[size_t(w)][size_t(pass)])]);
            }
    for (int i = 0; i < n; ++i) {
        P.jobs[size_t(j0 + i)] = jobs[size_t(i)];
        P.job_bucket[size_t(j0 + i)] = bucket[size_t(i)];
    }
}

}  // namespace

void build_lds_program(TreePlan& t) {
    LdsProgram P;
    auto fail = [&](const std::string& why) {
        P = LdsProgram{};
        P.ok = false;
        P.why = why;
        t.lds = std::move(P);
    };
    if (t.n_open > 0) return fail("open qubits (sets of amplitudes) run on the level launches");
    const int T = int(t.tensor_axes.size());
    const int n_levels = int(t.levels.size());
    std::vector<int> maker(T, -1);
    for (size_t i = 0; i < t.steps.size(); ++i) maker[t.steps[i].out_tensor] = int(i);
    for (const TreeStep& st : t.steps) {
        if (st.table_leaf) continue;
        if (int(st.in_tensors.size()) > kLdsMaxIn) return fail("a bucket with more than 4 inputs");
        if (st.kg > 3) return fail("a bucket summing more than 3 variables");
    }
    // elimination position of every variable, and the LDS axis order of every tensor
    int max_var = 0;
    for (int v : t.order) max_var = std::max(max_var, v);
    std::vector<int> pos(size_t(max_var) + 1, -1);
    for (size_t i = 0; i < t.order.size(); ++i) pos[size_t(t.order[i])] = int(i);
    auto later_first = [&](std::vector<int> vars) {
        std::stable_sort(vars.begin(), vars.end(), [&](int a, int b) { return pos[size_t(a)] > pos[size_t(b)]; });
        return vars;
    };
    std::vector<std::vector<int>> lax(static_cast<size_t>(T));
    for (int i = 0; i < T; ++i) lax[size_t(i)] = later_first(t.tensor_axes[size_t(i)]);
    // results made by the levels: LDS rows packed by lifetime (a result is live from the level that makes it
    // to the last level that reads it, the rank-0 results to the end), largest first at the lowest free row
    P.tensor_lds.assign(T, -1);
    std::vector<int> idx;
    for (int i = 0; i < T; ++i)
        if (maker[i] >= 0 && !t.steps[size_t(maker[i])].table_leaf) idx.push_back(i);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return t.tensor_axes[a].size() > t.tensor_axes[b].size(); });
    auto made = [&](int i) { return t.tensor_made[i]; };
    auto used = [&](int i) { return t.tensor_used[i]; };
    std::vector<int> placed;
    int64_t rows = 0;
    for (int a : idx) {
        const int64_t size = int64_t(1) << t.tensor_axes[a].size();
        std::vector<std::pair<int64_t, int64_t>> busy;
        for (int b : placed)
            if (!(used(b) < made(a) || used(a) < made(b)))
                busy.push_back({P.tensor_lds[b], P.tensor_lds[b] + (int64_t(1) << t.tensor_axes[b].size())});
        std::sort(busy.begin(), busy.end());
        int64_t off = 0;
        for (auto& iv : busy) {
            if (off + size <= iv.first) break;
            off = std::max(off, iv.second);
        }
        if (off + size > kLdsMaxComplex) return fail("results exceed the LDS of a work-group");
        P.tensor_lds[a] = int32_t(off);
        rows = std::max(rows, off + size);
        placed.push_back(a);
    }
    // the tables copied at the bitstring's output bits, in their LDS layouts: each bucket's factor table
    // (LDS entry (w << gb) | g from table entry ((g << kg) | w) << sb | sigma, g in the planner's order),
    // each leaf table (LDS entry o from table entry (o << sb) | sigma, o in the planner's axis order)
    P.tables0 = int32_t(rows);
    int64_t e = 0;
    std::vector<int64_t> tab_lds(t.steps.size(), -1);
    std::vector<std::vector<int>> gax(t.steps.size());
    std::vector<char> read_by_job(static_cast<size_t>(T), 0);   // leaf tables some job reads (not only composed leaves)
    for (const TreeStep& st : t.steps)
        if (!st.table_leaf)
            for (int tin : st.in_tensors) read_by_job[size_t(tin)] = 1;
    for (size_t i = 0; i < t.steps.size(); ++i) {
        const TreeStep& st = t.steps[i];
        if (st.table_leaf && !read_by_job[size_t(st.out_tensor)]) continue;
        const int64_t n = st.table_leaf ? (int64_t(1) << st.out_axes.size()) : (int64_t(1) << (st.gb() + st.kg));
        if (P.tables0 + e + n > kLdsMaxComplex) return fail("factor tables exceed the LDS of a work-group");
        if (int(P.stages.size()) >= kLdsMaxStages) return fail("more than 256 tables");
        LdsStage sg{};
        sg.n_sig = st.sb();
        sg.n = int32_t(n);
        sg.e0 = int32_t(e);
        sg.zoff = int32_t(P.z_entries);
        P.z_entries += n << st.sb();
        if (P.z_entries >= (int64_t(1) << 24)) return fail("staged tables exceed 2^24 entries");
        for (int b = 0; b < st.sb(); ++b) sg.sig_q[b] = st.sig_q[size_t(b)];
        const uint32_t s = uint32_t(P.stages.size());
        P.stages.push_back(sg);
        P.stage_bucket.push_back(int(i));
        if (st.table_leaf) {
            const std::vector<int>& ta = t.tensor_axes[size_t(st.out_tensor)];
            for (int64_t c = 0; c < n; ++c)
                P.entries.push_back({uint32_t(st.leaf_off + (relayout(c, lax[size_t(st.out_tensor)], ta) << st.sb())), s});
            P.tensor_lds[st.out_tensor] = int32_t(P.tables0 + e);
        } else {
            gax[i] = later_first(st.gvars);
            const int gb = st.gb();
            for (int64_t c = 0; c < n; ++c) {
                const int64_t w = c >> gb, g = relayout(c & ((int64_t(1) << gb) - 1), gax[i], st.gvars);
                P.entries.push_back({uint32_t(st.g_off + (((g << st.kg) | w) << st.sb())), s});
            }
        }
        tab_lds[i] = P.tables0 + e;
        e += n;
    }
    P.lds_size = int32_t(P.tables0 + e);
    if (P.lds_size > kLdsMaxComplex) return fail("LDS of a work-group exceeded");
    // the device's entry list: the staged index of each entry and its stage (a slice is one contiguous read)
    for (size_t i = 0; i < P.entries.size(); ++i) {
        const LdsStage& sg = P.stages[P.entries[i].stage];
        P.zent.push_back(uint32_t(sg.zoff + (int64_t(i) - sg.e0)) | (P.entries[i].stage << 24));
        if (P.entries[i].src >= (1u << 24)) return fail("a table entry beyond 2^24");
        P.gent.push_back(P.entries[i].src | (P.entries[i].stage << 24));
    }
    auto bytes = [](int64_t entry) { return int32_t(kLdsHeader + 8 * entry); };
    // Rows per lane of each bucket (rl: 2^rl rows): 2 where a row's loads batch and the result has 128 rows
    // or more (the rows share the record and the lane offsets, their loads are independent); then, per level,
    // more rows per lane for the bucket with the most jobs while the level has more jobs than the work-group
    // has waves and a bucket can take more (a level whose jobs take one pass of the waves ends sooner than
    // one that takes two, although its longest job is longer).
    std::vector<int> rl(t.steps.size(), 0);
    auto rank = [&](int sid) { return int(lax[size_t(t.steps[size_t(sid)].out_tensor)].size()); };
    auto jobs_of = [&](int sid) { return std::max<int64_t>(1, (int64_t(1) << rank(sid)) >> (6 + rl[size_t(sid)])); };
    auto can_grow = [&](int sid) {
        const TreeStep& st = t.steps[size_t(sid)];
        const int nin = int(st.in_tensors.size());
        return rl[size_t(sid)] < lds_max_rl(nin, st.kg) && rank(sid) >= 7 + rl[size_t(sid)];
    };
    int64_t n_jobs = 0, max_jobs = 0;
    for (int L = 0; L < n_levels; ++L) {
        int64_t nj = 0;
        for (int sid : t.levels[size_t(L)]) {
            const TreeStep& st = t.steps[size_t(sid)];
            if (st.table_leaf) continue;
            if (rank(sid) >= 7 && lds_batched(int(st.in_tensors.size()), st.kg, 1)) rl[size_t(sid)] = 1;
            nj += jobs_of(sid);
        }
        n_jobs += nj;
        max_jobs = std::max(max_jobs, nj);
    }
    // 8 waves when levels have many jobs (fewer bitstrings fit a compute unit, each finishes sooner), else 4
    const double mean_jobs = n_levels > 0 ? double(n_jobs) / n_levels : 0.0;
    P.threads = mean_jobs >= 5.0 || max_jobs >= 12 ? kLdsLargeThreads : kLdsSmallThreads;
    const int64_t n_waves = P.threads / 64;
    for (int L = 0; L < n_levels; ++L) {
        for (;;) {
            int64_t nj = 0, best = -1;
            for (int sid : t.levels[size_t(L)]) {
                if (t.steps[size_t(sid)].table_leaf) continue;
                nj += jobs_of(sid);
                if (can_grow(sid) && (best < 0 || jobs_of(sid) > jobs_of(int(best)))) best = sid;
            }
            if (nj <= n_waves || best < 0) break;
            ++rl[size_t(best)];
        }
    }
    // jobs, level by level
    P.level_job_off.assign(1, 0);
    for (int L = 0; L < n_levels; ++L) {
        for (int sid : t.levels[size_t(L)]) {
            const TreeStep& st = t.steps[size_t(sid)];
            if (st.table_leaf) continue;
            const std::vector<int>& ra = lax[size_t(st.out_tensor)];
            const int r = int(ra.size());
            const int nin = int(st.in_tensors.size());
            // the entry stride of each result axis in every input (slot k < nin) and in the table (slot nin)
            std::vector<std::vector<int64_t>> ostr(size_t(nin) + 1, std::vector<int64_t>(size_t(r), 0));
            for (int k = 0; k <= nin; ++k) {
                const std::vector<int>& ax = k < nin ? lax[size_t(st.in_tensors[size_t(k)])] : gax[size_t(sid)];
                for (int j = 0; j < r; ++j) {
                    const int a = axis_of(ax, ra[size_t(j)]);
                    if (a >= 0) ostr[size_t(k)][size_t(j)] = int64_t(1) << a;
                }
            }
            const int64_t n_rows = int64_t(1) << r;
            const int jrl = rl[size_t(sid)];
            for (int64_t o0 = 0; o0 < n_rows; o0 += int64_t(64) << jrl) {
                LdsJob jb{};
                jb.nin = nin;
                jb.k = st.kg;
                jb.lanes = int32_t(std::min<int64_t>(64, n_rows));
                jb.rl = jrl;
                jb.out_row = bytes(P.tensor_lds[st.out_tensor] + o0);
                for (int k = 0; k <= nin; ++k) {
                    int64_t row = k < nin ? P.tensor_lds[st.in_tensors[size_t(k)]] : tab_lds[size_t(sid)];
                    if (row < 0) return fail("an input without LDS rows");
                    for (int j = 6 + jrl; j < r; ++j)
                        if ((o0 >> j) & 1) row += ostr[size_t(k)][size_t(j)];
                    const int slot = k < nin ? k : kLdsMaxIn;
                    jb.base[slot] = bytes(row);
                    for (int j = 0; j < std::min(r, 6); ++j) jb.str[slot][j] = int32_t(8 * ostr[size_t(k)][size_t(j)]);
                    for (int x = 0; x < jrl; ++x) jb.strx[x][slot] = int32_t(8 * ostr[size_t(k)][size_t(6 + x)]);
                }
                // the summed values: their offset in each input, and in the table (w << gb)
                for (int w = 0; w < (1 << st.kg); ++w) {
                    jb.tw[w] = int32_t(8 * (int64_t(w) << st.gb()));
                    for (int k = 0; k < nin; ++k) {
                        const std::vector<int>& ax = lax[size_t(st.in_tensors[size_t(k)])];
                        int64_t off = 0;
                        for (int v = 0; v < st.kg; ++v) {
                            const int a = axis_of(ax, st.vars[size_t(v)]);
                            if (((w >> v) & 1) && a >= 0) off += int64_t(1) << a;
                        }
                        jb.in_w[k][w] = int32_t(8 * off);
                    }
                }
                P.jobs.push_back(jb);
                P.job_bucket.push_back(sid);
            }
        }
        order_level_jobs(P, P.level_job_off.back(), int32_t(P.jobs.size()), int(n_waves));
        P.level_job_off.push_back(int32_t(P.jobs.size()));
    }
    for (int f : t.finals) {
        if (P.tensor_lds[f] < 0) return fail("a rank-0 result without LDS rows");
        P.finals.push_back(bytes(P.tensor_lds[f]));
    }
    // the device records; kept in LDS after the tables when they fit (then a job reads nothing from memory)
    P.recs.assign(P.jobs.size() * size_t(kLdsRecordHalves), 0);
    for (size_t j = 0; j < P.jobs.size(); ++j) {
        const LdsJob& jb = P.jobs[j];
        uint16_t* rc = &P.recs[j * size_t(kLdsRecordHalves)];
        rc[0] = uint16_t(jb.nin | (jb.k << 3) | ((jb.lanes - 1) << 5) | (jb.rl << 11));
        rc[1] = uint16_t(jb.out_row);
        for (int s2 = 0; s2 <= kLdsMaxIn; ++s2) rc[2 + s2] = uint16_t(jb.base[s2]);
        for (int w = 0; w < 8; ++w) rc[8 + w] = uint16_t(jb.tw[w]);
        for (int k = 0; k < kLdsMaxIn; ++k)
            for (int w = 0; w < 8; ++w) rc[16 + 8 * k + w] = uint16_t(jb.in_w[k][w]);
        for (int s2 = 0; s2 <= kLdsMaxIn; ++s2)
            for (int c = 0; c < 8; ++c) {
                int32_t lo = jb.base[s2], hi = 0;
                for (int i = 0; i < 3; ++i)
                    if ((c >> i) & 1) {
                        lo += jb.str[s2][i];
                        hi += jb.str[s2][3 + i];
                    }
                if (lo > 0xFFFF || hi > 0xFFFF) return fail("a lane offset beyond 64 KiB");
                rc[48 + 16 * s2 + c] = uint16_t(lo);
                rc[56 + 16 * s2 + c] = uint16_t(hi);
            }
        for (int x = 0; x < 2; ++x)
            for (int s2 = 0; s2 <= kLdsMaxIn; ++s2) rc[128 + 8 * x + s2] = uint16_t(jb.strx[x][s2]);
    }
    // records in LDS whenever they fit: a job then reads its record with one LDS round trip instead of a
    // memory one (measured faster at every batch on 5x5 depth 25, although fewer work-groups fit a CU)
    const int64_t rec_entries = int64_t(P.jobs.size()) * (kLdsRecordBytes / 8);
    const int32_t recs0 = (P.lds_size + 1) & ~1;   // 16-byte aligned (the header is 16-byte aligned)
    if (recs0 + rec_entries <= kLdsMaxComplex) {
        P.recs0 = recs0;
        P.lds_size = recs0 + int32_t(rec_entries);
    }
    P.ok = true;
    t.lds = std::move(P);
}

int64_t lds_bytes_per_amp(const LdsProgram& P) {
    if (!P.ok) return 0;
    int64_t b = int64_t(P.entries.size()) * 8;
    for (const LdsJob& j : P.jobs)
        b += int64_t(j.lanes) * (int64_t(1) << j.rl) * (((int64_t(1) << j.k) * (j.nin + 1) + 1) * 8);
    return b;
}

}  // namespace qgm
