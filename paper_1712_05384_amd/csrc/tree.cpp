// Bucket-elimination planner (ordering 1): greedy treewidth orders, bucket
// steps, elimination-tree levels and the arena of intermediate results.
#include "tree.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <map>
#include <set>

#include "plan.hpp"

namespace qgm {

namespace {

// splitmix64 (Steele, Lea, Flood 2014): seeds the randomised tie breaks.
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

enum { VK_FREE = 0, VK_ZERO = 1, VK_SIG = 2 };

struct RawFactor {
    int type, mat;
    int v[4];
    int nv;
    std::vector<int> free;   // free-variable indices (fi) it touches, distinct
};

struct Model {
    std::vector<int> kind;        // per variable id: VK_*
    std::vector<int> fi;          // per variable id: free index or -1
    std::vector<int> free_var;    // free index -> variable id
    std::vector<RawFactor> facs;  // factors with at least one free variable
    std::vector<TFactor> phase;
    std::vector<int> kept;        // free indices of the open qubits' last variables, output bit ascending
    int zero_mask = 0;            // output bits of open qubits without non-diagonal gates (amplitude 0 if set)
    std::vector<int> sig_bit;     // per VK_SIG variable: bit of the batch column's word that fixes it (the
                                  //   qubit for an output variable, n + j for sliced variable j)
};

TFactor fixed_factor(const Plan& p, const Model& m, const RawFactor& f) {
    TFactor t{};
    t.type = f.type;
    t.mat = f.mat;
    int* srcs[4][2] = {{&t.src0, &t.bit0}, {&t.src1, &t.bit1}, {&t.src2, &t.bit2}, {&t.src3, &t.bit3}};
    for (int i = 0; i < f.nv; ++i) {
        const int v = f.v[i];
        if (m.kind[v] == VK_SIG) { *srcs[i][0] = TS_SIG; *srcs[i][1] = m.sig_bit[v]; }
        else { *srcs[i][0] = TS_ZERO; *srcs[i][1] = 0; }
    }
    return t;
}

// Greedy elimination order on the graph of free variables.  crit 0 picks the
// variable of fewest alive neighbours (min-degree), crit 1 the one whose
// elimination adds the fewest fill edges (min-fill, ties by degree); ties
// left after that go to a per-variable priority (random or the index).
std::vector<int> greedy_order(int nF, const std::vector<uint8_t>& adj0, int crit, uint64_t seed) {
    std::vector<uint8_t> adj = adj0;
    std::vector<int> deg(nF, 0), alive(nF, 1), score(nF, 0);
    std::vector<uint64_t> prio(nF);
    SplitMix rng{seed};
    for (int i = 0; i < nF; ++i) prio[i] = seed ? rng.next() : uint64_t(i);
    for (int i = 0; i < nF; ++i)
        for (int j = 0; j < nF; ++j) deg[i] += adj[size_t(i) * nF + j];
    auto nbrs = [&](int u, std::vector<int>& out) {
        out.clear();
        const uint8_t* row = &adj[size_t(u) * nF];
        for (int j = 0; j < nF; ++j)
            if (row[j] && alive[j]) out.push_back(j);
    };
    std::vector<int> nb, nb2;
    auto fill_of = [&](int u) {
        nbrs(u, nb2);
        int f = 0;
        for (size_t a = 0; a < nb2.size(); ++a)
            for (size_t b = a + 1; b < nb2.size(); ++b) f += adj[size_t(nb2[a]) * nF + nb2[b]] ? 0 : 1;
        return f;
    };
    if (crit == 1)
        for (int i = 0; i < nF; ++i) score[i] = fill_of(i);
    std::vector<int> order;
    order.reserve(nF);
    std::vector<uint8_t> dirty(nF, 0);
    for (int it = 0; it < nF; ++it) {
        int best = -1;
        for (int u = 0; u < nF; ++u) {
            if (!alive[u]) continue;
            if (best < 0) { best = u; continue; }
            const int su = crit == 1 ? score[u] : deg[u], sb = crit == 1 ? score[best] : deg[best];
            if (su < sb || (su == sb && (deg[u] < deg[best] || (deg[u] == deg[best] && prio[u] < prio[best]))))
                best = u;
        }
        nbrs(best, nb);
        alive[best] = 0;
        order.push_back(best);
        for (int a : nb) deg[a] -= 1;
        for (size_t a = 0; a < nb.size(); ++a)
            for (size_t b = a + 1; b < nb.size(); ++b) {
                uint8_t& e = adj[size_t(nb[a]) * nF + nb[b]];
                if (!e) {
                    e = 1;
                    adj[size_t(nb[b]) * nF + nb[a]] = 1;
                    deg[nb[a]] += 1;
                    deg[nb[b]] += 1;
                }
            }
        if (crit == 1) {
            // fill counts change only within distance two of the eliminated variable
            std::vector<int> touched;
            for (int a : nb) {
                if (!dirty[a]) { dirty[a] = 1; touched.push_back(a); }
                nbrs(a, nb2);
                for (int c : nb2)
                    if (!dirty[c]) { dirty[c] = 1; touched.push_back(c); }
            }
            for (int u : touched) { score[u] = fill_of(u); dirty[u] = 0; }
        }
    }
    return order;
}

struct SimOut {
    bool ok = false;
    double bytes = 0, flops = 0;
    int levels = 0, max_rank = 0, max_in = 0;
    std::string why;
};

// A bucket step in free-variable indices, before merging and encoding.
struct RStep {
    std::vector<int> vars;   // summed variables (the bucket's variable first)
    std::vector<int> out;    // result axes, elimination position ascending
    std::vector<int> ins;    // input results
    std::vector<int> facs;   // gate factors (indices into Model::facs)
    std::vector<std::pair<std::vector<int>, std::vector<int>>> absorbed;   // (variables, factors) of folded buckets
    int out_tensor = -1;
    bool alive = true;
    bool open = false;       // multiplies the results over the open qubits' variables (sums nothing)
};

struct RTensor {
    std::vector<int> axes;
    int producer = -1;
};

// Factor-table variables (besides the summed ones) and output bits of a set of factors.
void table_vars(const Plan& p, const Model& m, const std::vector<int>& facs, const std::vector<int>& summed,
                std::set<int>& gset, std::vector<int>& sigq) {
    gset.clear();
    sigq.clear();
    for (int f : facs) {
        const RawFactor& rf = m.facs[f];
        for (int u : rf.free)
            if (std::find(summed.begin(), summed.end(), u) == summed.end()) gset.insert(u);
        for (int k = 0; k < rf.nv; ++k)
            if (m.kind[rf.v[k]] == VK_SIG) {
                const int q = m.sig_bit[rf.v[k]];
                if (std::find(sigq.begin(), sigq.end(), q) == sigq.end()) sigq.push_back(q);
            }
    }
}

// Table variables and output bits of a bucket with absorbed groups: every
// free variable of any factor that is neither summed by the bucket nor a
// group's own variable.
void group_table_vars(const Plan& p, const Model& m, const RStep& st, std::set<int>& gset, std::vector<int>& sigq) {
    std::vector<int> excl = st.vars;
    for (auto& a : st.absorbed) excl.insert(excl.end(), a.first.begin(), a.first.end());
    std::vector<int> facs = st.facs;
    for (auto& a : st.absorbed) facs.insert(facs.end(), a.second.begin(), a.second.end());
    table_vars(p, m, facs, excl, gset, sigq);
}

bool fits(int rank, int n_in, int gb, int k, int sb) {
    return rank <= kTreeMaxRank && n_in <= kTreeMaxIn && gb <= kTreeMaxGBits && sb <= kTreeMaxSig &&
           k <= kTreeMaxSum && gb + k + sb <= kTreeMaxGIndex;
}

// Runs bucket elimination over the structure for an order (free indices):
// bucket i multiplies the results and factors whose earliest variable is
// order[i] and sums that variable out.  With `steps`/`tens` set, also
// records the steps.
SimOut simulate(const Plan& p, const Model& m, const std::vector<int>& order, std::vector<RStep>* steps,
                std::vector<RTensor>* tens, bool check_limits = true) {
    SimOut r;
    const int nF = int(order.size());
    std::vector<int> pos(nF);
    for (int i = 0; i < nF; ++i) pos[order[i]] = i;
    std::vector<std::vector<int>> bfac(nF), bten(nF);
    for (int f = 0; f < int(m.facs.size()); ++f) {
        int e = nF;
        for (int u : m.facs[f].free) e = std::min(e, pos[u]);
        bfac[e].push_back(f);
    }
    std::vector<std::vector<int>> taxes;
    std::vector<int> tmade;
    std::set<int> gset;
    std::vector<int> sigq;
    const int n_elim = nF - int(m.kept.size());   // the kept variables close the order and are not summed
    for (int i = 0; i < n_elim; ++i) {
        const int v = order[i];
        std::set<int> A;
        int level = 0;
        for (int tid : bten[i]) {
            for (int u : taxes[tid]) A.insert(u);
            level = std::max(level, tmade[tid] + 1);
        }
        for (int f : bfac[i])
            for (int u : m.facs[f].free) A.insert(u);
        if (!A.count(v)) { r.why = "internal: variable missing from its bucket"; return r; }
        table_vars(p, m, bfac[i], {v}, gset, sigq);
        std::vector<int> out;
        for (int u : A) if (u != v) out.push_back(u);
        std::sort(out.begin(), out.end(), [&](int a, int b) { return pos[a] < pos[b]; });
        const int n_in = int(bten[i].size());
        if (check_limits && !fits(int(out.size()), n_in, int(gset.size()), 1, int(sigq.size()))) {
            char buf[200];
            snprintf(buf, sizeof buf, "bucket exceeds kernel limits (rank %d, inputs %d, table bits %d, output bits %d)",
                     int(out.size()), n_in, int(gset.size()), int(sigq.size()));
            r.why = buf;
            return r;
        }
        const double rows = double(int64_t(1) << out.size());
        double bytes = 8.0 * rows;
        for (int tid : bten[i]) bytes += 8.0 * double(int64_t(1) << taxes[tid].size());
        const int mult = n_in + (bfac[i].empty() ? 0 : 1);
        r.bytes += bytes;
        r.flops += 2.0 * rows * (6.0 * std::max(mult - 1, 0) + 2.0);
        r.levels = std::max(r.levels, level + 1);
        r.max_rank = std::max(r.max_rank, int(out.size()));
        r.max_in = std::max(r.max_in, n_in);
        const int tid = int(taxes.size());
        taxes.push_back(out);
        tmade.push_back(level);
        if (!out.empty()) bten[pos[out[0]]].push_back(tid);
        if (steps) {
            RStep st;
            st.vars = {v};
            st.out = out;
            st.ins = bten[i];
            st.facs = bfac[i];
            st.out_tensor = tid;
            RTensor rt;
            rt.axes = out;
            rt.producer = int(steps->size());
            tens->push_back(rt);
            steps->push_back(st);
        }
    }
    // open qubits: every result and factor left on the kept variables is multiplied into one
    // result over all of them (a chain of such buckets when more than kTreeMaxIn results remain)
    if (!m.kept.empty()) {
        std::vector<int> ins, facs;
        for (int i = n_elim; i < nF; ++i) {
            ins.insert(ins.end(), bten[i].begin(), bten[i].end());
            facs.insert(facs.end(), bfac[i].begin(), bfac[i].end());
        }
        while (true) {
            const bool last = int(ins.size()) <= kTreeMaxIn;
            std::vector<int> take(ins.begin(), ins.begin() + std::min<size_t>(ins.size(), kTreeMaxIn));
            std::vector<int> fac_here = last ? facs : std::vector<int>{};
            std::vector<int> out;
            int level = 0;
            if (last) {
                out = m.kept;
            } else {
                std::set<int> A;
                for (int tid : take) A.insert(taxes[tid].begin(), taxes[tid].end());
                for (int u : m.kept)
                    if (A.count(u)) out.push_back(u);
            }
            for (int tid : take) level = std::max(level, tmade[tid] + 1);
            table_vars(p, m, fac_here, {}, gset, sigq);
            if (check_limits && !fits(int(out.size()), int(take.size()), int(gset.size()), 0, int(sigq.size()))) {
                r.why = "the bucket over the open qubits exceeds the kernel limits";
                return r;
            }
            const double rows = double(int64_t(1) << out.size());
            double bytes = 8.0 * rows;
            for (int tid : take) bytes += 8.0 * double(int64_t(1) << taxes[tid].size());
            r.bytes += bytes;
            r.flops += rows * 6.0 * double(take.size());
            r.levels = std::max(r.levels, level + 1);
            r.max_rank = std::max(r.max_rank, int(out.size()));
            r.max_in = std::max(r.max_in, int(take.size()));
            const int tid = int(taxes.size());
            taxes.push_back(out);
            tmade.push_back(level);
            if (steps) {
                RStep st;
                st.out = out;
                st.ins = take;
                st.facs = fac_here;
                st.out_tensor = tid;
                st.open = true;
                RTensor rt;
                rt.axes = out;
                rt.producer = int(steps->size());
                tens->push_back(rt);
                steps->push_back(st);
            }
            if (last) break;
            ins.erase(ins.begin(), ins.begin() + long(take.size()));
            ins.insert(ins.begin(), tid);
        }
    }
    r.ok = true;
    return r;
}

// Merges chain links: a bucket whose only input is the result of one earlier
// bucket absorbs that bucket (both summed variables at once) when the merged
// index space grows by at most one bit, so the intermediate result is never
// written and the elimination tree loses a level.
void merge_chains(const Plan& p, const Model& m, std::vector<RStep>& steps, std::vector<RTensor>& tens) {
    std::set<int> gset;
    std::vector<int> sigq;
    for (size_t i = 0; i < steps.size(); ++i) {
        RStep& par = steps[i];
        if (par.ins.size() != 1 || par.open) continue;
        const int tid = par.ins[0];
        RStep& ch = steps[tens[tid].producer];
        if (ch.open) continue;
        std::vector<int> V = ch.vars;
        V.insert(V.end(), par.vars.begin(), par.vars.end());
        std::vector<int> facs = ch.facs;
        facs.insert(facs.end(), par.facs.begin(), par.facs.end());
        table_vars(p, m, facs, V, gset, sigq);
        if (!fits(int(par.out.size()), int(ch.ins.size()), int(gset.size()), int(V.size()), int(sigq.size()))) continue;
        const int64_t work_m = int64_t(1) << (par.out.size() + V.size());
        const int64_t work_c = int64_t(1) << (ch.out.size() + ch.vars.size());
        const int64_t work_p = int64_t(1) << (par.out.size() + par.vars.size());
        if (work_m > 2 * std::max(work_c, work_p)) continue;
        par.vars = V;
        par.facs = facs;
        par.ins = ch.ins;
        ch.alive = false;
        tens[tid].producer = -2;   // never materialised
    }
}

// Folds every bucket without inputs into the factor table of the bucket that
// reads its result: that bucket's table gets one more factor group, the sum
// over the folded bucket's variables of its factors' product.  The folded
// result is never materialised and level 0 of the tree (if every such bucket
// has a reader and the tables stay within the limits) needs no launch.
int absorb_leaves(const Plan& p, const Model& m, std::vector<RStep>& steps, std::vector<RTensor>& tens) {
    std::vector<int> reader(tens.size(), -1);
    for (size_t i = 0; i < steps.size(); ++i)
        if (steps[i].alive)
            for (int t : steps[i].ins) reader[t] = int(i);
    std::set<int> gset;
    std::vector<int> sigq;
    int n = 0;
    for (size_t i = 0; i < steps.size(); ++i) {
        RStep& lf = steps[i];
        if (!lf.alive || !lf.ins.empty() || !lf.absorbed.empty() || reader[lf.out_tensor] < 0) continue;
        RStep& par = steps[reader[lf.out_tensor]];
        if (par.absorbed.size() >= 15) continue;   // a table has at most 16 factor groups
        par.absorbed.push_back({lf.vars, lf.facs});
        group_table_vars(p, m, par, gset, sigq);
        const int n_in = int(par.ins.size()) - 1;
        if (!fits(int(par.out.size()), n_in, int(gset.size()), int(par.vars.size()), int(sigq.size()))) {
            par.absorbed.pop_back();
            continue;
        }
        par.ins.erase(std::find(par.ins.begin(), par.ins.end(), lf.out_tensor));
        lf.alive = false;
        tens[lf.out_tensor].producer = -2;   // never materialised
        ++n;
    }
    return n;
}

}  // namespace

// Turns the merged raw steps into the plan: compact result ids, levels,
// factor tables (index c = (g << kg) | w, kg = most summed variables of the
// level), arena rows, sigma rows and wave tasks.
// Axis order of a bucket's result: a wave unit covers the result rows that
// differ in the lowest kTreeOcBits axes, and an input that does not carry one
// of them is read once for the rows that differ in it.  So those positions go,
// greedily, to the axes that leave the fewest distinct input rows per unit,
//   sum over inputs t of 2^(|U & axes(t)| + |summed & axes(t)|),
// U the axes chosen so far (elimination order breaks ties and orders the rest).
// The order is free: every reader indexes a result through its axis strides.
// After them come the axes that the largest inputs do not carry (by the total
// rows of the inputs lacking the axis): consecutive tasks then re-read the same
// rows of those inputs while they are still in the L2.
static std::vector<int> unit_axis_order(const RStep& st, const std::vector<std::vector<int>>& out_of) {
    std::vector<int> rest = st.out, chosen;
    auto carries = [&](int in, int u) {
        const std::vector<int>& ax = out_of[in];
        return std::find(ax.begin(), ax.end(), u) != ax.end();
    };
    while (int(chosen.size()) < kTreeOcBits && !rest.empty()) {
        size_t best = 0;
        double best_cost = std::numeric_limits<double>::infinity();
        for (size_t c = 0; c < rest.size(); ++c) {
            double cost = 0;
            for (int in : st.ins) {
                int e = carries(in, rest[c]) ? 1 : 0;
                for (int u : chosen) e += carries(in, u) ? 1 : 0;
                for (int v : st.vars) e += carries(in, v) ? 1 : 0;
                cost += double(int64_t(1) << e);
            }
            if (cost < best_cost) { best_cost = cost; best = c; }
        }
        chosen.push_back(rest[best]);
        rest.erase(rest.begin() + long(best));
    }
    std::vector<double> lack(rest.size(), 0.0);
    for (size_t c = 0; c < rest.size(); ++c)
        for (int in : st.ins)
            if (!carries(in, rest[c])) lack[c] += double(int64_t(1) << out_of[in].size());
    std::vector<size_t> idx(rest.size());
    for (size_t c = 0; c < idx.size(); ++c) idx[c] = c;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return lack[x] > lack[y]; });
    for (size_t c : idx) chosen.push_back(rest[c]);
    return chosen;
}

// A bucket with two or three inputs summing at least two variables whose result
// has two bits carried by one input only (A) and one bit carried by another
// input only (B), none of them a factor-table variable: its result axes start
// with those three bits and a wave unit covers the 2 x 2 x 2 rows from 4 rows of
// A, 2 of B and (a third input C, which varies along none of them) 1 of C per
// summed value (the general unit holds every (row, input, value) entry and
// covers 2-4 rows).  Returns 1 (two inputs) or 2 (three), the axis order and
// the inputs in the order A, B, C.
static int tile_axis_order(const Plan& p, const Model& m, const RStep& st,
                           const std::vector<std::vector<int>>& out_of, std::vector<int>& order,
                           std::vector<int>& ins, char& quad) {
    quad = 0;
    const int n = int(st.ins.size());
    if (st.open || (n != 2 && n != 3) || st.vars.size() < 2) return 0;
    std::set<int> gset;
    std::vector<int> sigq;
    group_table_vars(p, m, st, gset, sigq);
    auto carries = [&](int in, int u) {
        const std::vector<int>& ax = out_of[in];
        return std::find(ax.begin(), ax.end(), u) != ax.end();
    };
    std::vector<std::vector<int>> only(n);
    for (int u : st.out) {
        if (gset.count(u)) continue;
        int holder = -1, count = 0;
        for (int k = 0; k < n; ++k)
            if (carries(st.ins[k], u)) { holder = k; ++count; }
        if (count == 1) only[holder].push_back(u);
    }
    int ka = -1, kb = -1;
    for (int a = 0; a < n && ka < 0; ++a)
        for (int b = 0; b < n; ++b)
            if (a != b && only[a].size() >= 2 && !only[b].empty()) { ka = a; kb = b; break; }
    if (ka < 0) return 0;
    // the 32-row tile when A has three bits alone and B two: unit bits a0 a1 b0 a2 b1 (bits 0-2 also make the
    // 8-row tile, which a level whose launch cannot hold the large unit falls back to)
    int big = 0;
    for (int a = 0; a < n && !big; ++a)
        for (int b = 0; b < n; ++b)
            if (a != b && only[a].size() >= 3 && only[b].size() >= 2) { ka = a; kb = b; big = 2; break; }
    order = {only[ka][0], only[ka][1], only[kb][0]};
    if (big) {
        order.push_back(only[ka][2]);
        order.push_back(only[kb][1]);
        // two inputs and two more bits of B alone: those next (result bits 5 and 6), so four consecutive
        // 32-row units read the same rows of A
        if (n == 2 && only[kb].size() >= 4) {
            order.push_back(only[kb][2]);
            order.push_back(only[kb][3]);
            quad = 1;
        }
    }
    ins = {st.ins[ka], st.ins[kb]};
    for (int k = 0; k < n; ++k)
        if (k != ka && k != kb) ins.push_back(st.ins[k]);
    std::vector<int> rest;
    for (int u : st.out)
        if (std::find(order.begin(), order.end(), u) == order.end()) rest.push_back(u);
    // the other axes as in the general order: those that most inputs lack (by size) lowest
    std::vector<double> lack(rest.size(), 0.0);
    for (size_t c = 0; c < rest.size(); ++c)
        for (int in : st.ins)
            if (!carries(in, rest[c])) lack[c] += double(int64_t(1) << out_of[in].size());
    std::vector<size_t> idx(rest.size());
    for (size_t c = 0; c < idx.size(); ++c) idx[c] = c;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return lack[x] > lack[y]; });
    for (size_t c : idx) order.push_back(rest[c]);
    return n - 1 + big;
}

static qgm_status finalize_tree(const Plan& p, const Model& m, const std::vector<int>& order,
                                const std::vector<RStep>& rs, const std::vector<RTensor>& rt, TreePlan& t,
                                std::string* err) {
    const int nF = int(order.size());
    std::vector<int> pos(nF);
    for (int i = 0; i < nF; ++i) pos[order[i]] = i;
    // result axes (free-variable indices) of every raw result, then their unit-friendly order
    std::vector<std::vector<int>> out_of(rt.size());
    for (const RStep& st : rs)
        if (st.alive) out_of[st.out_tensor] = st.out;
    std::vector<std::vector<int>> out_ord(rs.size());
    std::vector<int> tile_of(rs.size(), 0);
    std::vector<char> quad_of(rs.size(), 0);
    std::vector<std::vector<int>> tile_ins(rs.size());
    for (size_t i = 0; i < rs.size(); ++i) {   // a bucket over the open qubits keeps their order (output index bits)
        if (!rs[i].alive) continue;
        if (rs[i].open) out_ord[i] = rs[i].out;
        else if (p.opts.no_tile == 0 &&
                 (tile_of[i] = tile_axis_order(p, m, rs[i], out_of, out_ord[i], tile_ins[i], quad_of[i])) != 0) {}
        else out_ord[i] = unit_axis_order(rs[i], out_of);
    }
    std::vector<int> tmap(rt.size(), -1);
    t.tensor_axes.clear();
    for (size_t i = 0; i < rs.size(); ++i) {
        const RStep& st = rs[i];
        if (!st.alive) continue;
        tmap[st.out_tensor] = int(t.tensor_axes.size());
        std::vector<int> ax;
        for (int u : out_ord[i]) ax.push_back(m.free_var[u]);
        t.tensor_axes.push_back(ax);
    }
    const int T = int(t.tensor_axes.size());
    t.tensor_made.assign(T, 0);
    t.steps.clear();
    t.finals.clear();
    std::set<int> gset;
    std::vector<int> sigq;
    std::vector<std::vector<std::pair<std::vector<int>, std::vector<int>>>> step_groups;   // (own vars, factors)
    std::vector<int> step_of_tensor(static_cast<size_t>(T), -1);                             // step making each result
    double bytes = 0, flops = 0;
    for (size_t si = 0; si < rs.size(); ++si) {
        const RStep& st = rs[si];
        if (!st.alive) continue;
        TreeStep ts;
        for (int u : st.vars) ts.vars.push_back(m.free_var[u]);
        ts.out_tensor = tmap[st.out_tensor];
        for (int u : out_ord[si]) ts.out_axes.push_back(m.free_var[u]);
        int level = 0;
        for (int in : (tile_of[si] ? tile_ins[si] : st.ins)) {   // a tile's inputs in the order A, B, C
            const int ti = tmap[in];
            if (ti < 0) { *err = "internal: merged result still read"; return QGM_E_INTERNAL; }
            ts.in_tensors.push_back(ti);
            level = std::max(level, t.tensor_made[ti] + 1);
        }
        ts.level = level;
        ts.tile = tile_of[si];
        ts.quad = quad_of[si] != 0;
        t.tensor_made[ts.out_tensor] = level;
        group_table_vars(p, m, st, gset, sigq);
        std::vector<int> g(gset.begin(), gset.end());
        std::sort(g.begin(), g.end(), [&](int a, int b) { return pos[a] < pos[b]; });
        for (int u : g) ts.gvars.push_back(m.free_var[u]);
        ts.sig_q = sigq;
        // a bucket without inputs whose table over (result, output bits) is small: with fixed gates it is
        // built once with the plan and read per lane; its axes follow its table variables
        if (p.n_slots == 0 && !st.open && ts.in_tensors.empty() && !ts.out_axes.empty() &&
            ts.gvars.size() == ts.out_axes.size() && int(ts.out_axes.size() + sigq.size()) <= kTreeLeafTableBits) {
            ts.table_leaf = true;
            ts.level = -1;
            t.tensor_made[ts.out_tensor] = -1;
            ts.out_axes = ts.gvars;
            t.tensor_axes[ts.out_tensor] = ts.gvars;
            ++t.n_table_leaves;
        }
        // a bucket whose inputs are all leaf tables (Sec. V: its result depends on the bitstring only through
        // the output bits its subtree reads): with few result and output bits, a leaf table too, built once for
        // every value of those bits; its output bits are its own, then its inputs' others
        if (p.n_slots == 0 && !st.open && !ts.table_leaf && !ts.in_tensors.empty() && !ts.out_axes.empty() &&
            p.opts.no_compose == 0 && int(ts.in_tensors.size()) <= kTreeMaxIn && ts.kg <= kTreeMaxSum &&
            ts.out_axes.size() <= 16) {
            bool leaves = true;
            std::vector<int> sig_all = sigq;
            int depth = 0;
            for (int ti : ts.in_tensors) {
                const int ms = step_of_tensor[size_t(ti)];
                if (ms < 0 || !t.steps[size_t(ms)].table_leaf || t.tensor_axes[size_t(ti)].size() > 16) {
                    leaves = false;
                    break;
                }
                depth = std::max(depth, t.steps[size_t(ms)].leaf_depth + 1);
                for (int q : t.steps[size_t(ms)].sig_q)
                    if (std::find(sig_all.begin(), sig_all.end(), q) == sig_all.end()) sig_all.push_back(q);
            }
            const int sb_all = int(sig_all.size());
            if (leaves && sb_all <= kTreeComposeSig && int(ts.out_axes.size()) + sb_all <= kTreeComposeBits &&
                int(ts.gvars.size()) + ts.kg + sb_all <= kTreeMaxGIndex) {
                ts.table_leaf = true;
                ts.composed = true;
                ts.tile = 0;   // (no unit runs it; its axes keep the order chosen for its consumers)
                ts.quad = false;
                ts.leaf_depth = depth;
                ts.level = -1;
                t.tensor_made[ts.out_tensor] = -1;
                ts.sig_q = sig_all;
                ++t.n_table_leaves;
            }
        }
        step_groups.push_back({{std::vector<int>{}, st.facs}});
        for (auto& a : st.absorbed) step_groups.back().push_back(a);
        if (ts.out_axes.empty()) t.finals.push_back(ts.out_tensor);
        if (st.open) t.open_tensor = ts.out_tensor;   // the chain's last bucket comes last
        const double rows = double(int64_t(1) << ts.out_axes.size());
        double b = ts.table_leaf ? 0.0 : 8.0 * rows;   // a leaf table is read from the caches, not per bitstring
        for (int ti : ts.in_tensors) {
            // a composed leaf table is read at each bitstring's own output bits: one slice per bitstring
            const int ms = step_of_tensor[size_t(ti)];
            const bool sliced = !ts.table_leaf && ms >= 0 && t.steps[size_t(ms)].composed;
            if (t.tensor_made[ti] >= 0 || sliced) b += 8.0 * double(int64_t(1) << t.tensor_axes[ti].size());
        }
        bytes += b;
        const int mult = int(ts.in_tensors.size()) + 1;
        if (!ts.composed) flops += rows * double(int64_t(1) << ts.vars.size()) * (6.0 * std::max(mult - 1, 0) + 2.0);
        step_of_tensor[size_t(ts.out_tensor)] = int(t.steps.size());
        t.steps.push_back(std::move(ts));
    }
    t.bytes_per_b = bytes;
    t.flops_per_b = flops;
    int n_levels = 0;
    for (auto& st : t.steps) n_levels = std::max(n_levels, st.level + 1);
    t.levels.assign(n_levels, {});
    for (int s = 0; s < int(t.steps.size()); ++s)
        if (!t.steps[s].table_leaf) t.levels[t.steps[s].level].push_back(s);
    // factor encoding: summed variable i is index bit i, table variable j is bit kg + j
    t.max_rank = 0;
    t.max_in = 0;
    for (size_t si = 0; si < t.steps.size(); ++si) {
        TreeStep& st = t.steps[si];
        st.kg = int(st.vars.size());
        if (st.gb() + st.kg + st.sb() > kTreeMaxGIndex) {
            *err = "bucket factor table exceeds the kernel limit";
            return QGM_E_UNSUPPORTED;
        }
        t.max_rank = std::max(t.max_rank, int(st.out_axes.size()));
        t.max_in = std::max(t.max_in, int(st.in_tensors.size()));
        for (auto& grp : step_groups[si]) {
            TGroup tg;
            tg.k_int = int(grp.first.size());
            for (int u : grp.first) tg.vars.push_back(m.free_var[u]);
            for (int f : grp.second) {
                const RawFactor& rf = m.facs[f];
                TFactor tf{};
                tf.type = rf.type;
                tf.mat = rf.mat;
                int* srcs[4][2] = {{&tf.src0, &tf.bit0}, {&tf.src1, &tf.bit1}, {&tf.src2, &tf.bit2}, {&tf.src3, &tf.bit3}};
                for (int k = 0; k < rf.nv; ++k) {
                    const int var = rf.v[k];
                    if (m.kind[var] == VK_FREE) {
                        const int u = m.fi[var];
                        auto own = std::find(grp.first.begin(), grp.first.end(), u);
                        auto it = std::find(st.vars.begin(), st.vars.end(), var);
                        if (own != grp.first.end()) {
                            *srcs[k][0] = TS_INT;
                            *srcs[k][1] = int(own - grp.first.begin());
                        } else if (it != st.vars.end()) {
                            *srcs[k][0] = TS_G;
                            *srcs[k][1] = int(it - st.vars.begin());
                        } else {
                            *srcs[k][0] = TS_G;
                            *srcs[k][1] = st.kg + int(std::find(st.gvars.begin(), st.gvars.end(), var) - st.gvars.begin());
                        }
                    } else if (m.kind[var] == VK_SIG) {
                        *srcs[k][0] = TS_SIG;
                        *srcs[k][1] = int(std::find(st.sig_q.begin(), st.sig_q.end(), m.sig_bit[var]) - st.sig_q.begin());
                    } else {
                        *srcs[k][0] = TS_ZERO;
                        *srcs[k][1] = 0;
                    }
                }
                tg.factors.push_back(tf);
            }
            st.groups.push_back(std::move(tg));
        }
    }
    return QGM_OK;
}

double tree_step_bytes(const TreePlan& t, const TreeStep& st) {
    if (st.table_leaf) return 0.0;   // built once with the plan
    std::vector<char> tab(t.tensor_axes.size(), 0);
    for (const TreeStep& s : t.steps)   // a plain leaf table is a few KiB shared by every bitstring (cache-resident);
        if (s.table_leaf && !s.composed) tab[s.out_tensor] = 1;   // a composed one is read in per-bitstring slices
    double b = 8.0 * double(int64_t(1) << st.out_axes.size());
    for (int tid : st.in_tensors)
        if (!tab[tid]) b += 8.0 * double(int64_t(1) << t.tensor_axes[tid].size());
    return b;
}

static qgm_status tree_from_order(const Plan& p, const Model& m, const std::vector<std::pair<int, int>>& kept,
                                  const std::vector<int>& best, TreePlan& t, std::string* err);

namespace {

// The variables left free by the deltas of Eq. (psi_x) and by slicing, the
// factors over them, and the factors without any (the per-bitstring phase).
// A sliced variable is fixed like an output variable, by bit n + j of the
// batch column's word (j: its position in `sliced`).
void build_model(const Plan& p, const std::vector<int>& sliced, Model& m, std::vector<std::pair<int, int>>& kept) {
    const int nv = int(p.vars.size());
    m.kind.assign(nv, VK_FREE);
    m.fi.assign(nv, -1);
    m.sig_bit.assign(nv, -1);
    for (int v = 0; v < nv; ++v) {
        const VarInfo& vi = p.vars[v];
        const auto sl = std::find(sliced.begin(), sliced.end(), v);
        if (vi.is_c0) {
            m.kind[v] = VK_ZERO;
            if (vi.is_final && vi.open_idx >= 0) {   // open, without non-diagonal gates: only output bit 0
                m.zero_mask |= 1 << vi.open_idx;
            } else if (vi.is_final) {   // a worldline without non-diagonal gates: b = 0 must equal x_q
                TFactor d{};
                d.type = TF_DELTA0;
                d.src0 = TS_SIG;
                d.bit0 = vi.qubit;
                m.phase.push_back(d);
            }
        } else if (vi.is_final && vi.open_idx < 0) {
            m.kind[v] = VK_SIG;
            m.sig_bit[v] = vi.qubit;
        } else if (sl != sliced.end()) {
            m.kind[v] = VK_SIG;
            m.sig_bit[v] = p.n + int(sl - sliced.begin());
        } else {
            m.fi[v] = int(m.free_var.size());
            m.free_var.push_back(v);
        }
    }
    // the open qubits' last variables (free, never summed), by output bit
    kept.clear();
    for (int v = 0; v < nv; ++v)
        if (p.vars[v].is_final && !p.vars[v].is_c0 && p.vars[v].open_idx >= 0) kept.push_back({p.vars[v].open_idx, m.fi[v]});
    std::sort(kept.begin(), kept.end());
    for (auto& k : kept) m.kept.push_back(k.second);
    for (const GateRec& g : p.recs) {
        RawFactor f{};
        f.mat = g.mat;
        if (g.type == 0) { f.type = TF_MAT; f.v[0] = g.var0; f.v[1] = g.var1; f.nv = 2; }
        else if (g.type == 1) { f.type = TF_DIAG; f.v[0] = g.var0; f.v[1] = -1; f.nv = 1; }
        else if (g.type == 3) {   // the 4-clique of a non-diagonal two-qubit gate
            f.type = TF_MAT4; f.v[0] = g.var0; f.v[1] = g.var1; f.v[2] = g.var2; f.v[3] = g.var3; f.nv = 4;
        } else { f.type = TF_CZ; f.mat = -1; f.v[0] = g.var0; f.v[1] = g.var1; f.nv = 2; }
        for (int k = 0; k < f.nv; ++k) {
            const int u = m.fi[f.v[k]];
            if (u >= 0 && std::find(f.free.begin(), f.free.end(), u) == f.free.end()) f.free.push_back(u);
        }
        if (f.free.empty()) m.phase.push_back(fixed_factor(p, m, f));
        else m.facs.push_back(f);
    }
}

// The interaction graph of the free variables: a factor joins its free
// variables pairwise (a 4-clique for a two-qubit gate).
std::vector<uint8_t> model_graph(const Model& m) {
    const int nF = int(m.free_var.size());
    std::vector<uint8_t> adj(size_t(nF) * nF, 0);
    for (auto& f : m.facs)
        for (size_t i = 0; i < f.free.size(); ++i)
            for (size_t j = i + 1; j < f.free.size(); ++j) {
                adj[size_t(f.free[i]) * nF + f.free[j]] = 1;
                adj[size_t(f.free[j]) * nF + f.free[i]] = 1;
            }
    return adj;
}

// Greedy order with the open qubits' variables moved to its end.
std::vector<int> candidate_order(const Model& m, const std::vector<uint8_t>& adj, int crit, int rs) {
    const int nF = int(m.free_var.size());
    std::vector<int> ord = greedy_order(nF, adj, crit, rs == 0 ? 0 : 0x5EED0000ull + uint64_t(rs) * 131 + crit);
    if (!m.kept.empty()) {   // the open qubits' variables close the order, by output bit
        std::vector<int> o2;
        for (int u : ord)
            if (std::find(m.kept.begin(), m.kept.end(), u) == m.kept.end()) o2.push_back(u);
        o2.insert(o2.end(), m.kept.begin(), m.kept.end());
        ord.swap(o2);
    }
    return ord;
}

}  // namespace

qgm_status build_tree_plan(const Plan& p, const std::vector<int>& sliced, TreePlan& t, std::string* err) {
    t = TreePlan{};
    if (p.n_open != 0 && p.opts.tree_exec == 2) {
        *err = "the persistent launch (tree_exec 2) supports no open qubits";
        return QGM_E_UNSUPPORTED;
    }
    if (!sliced.empty() && p.opts.tree_exec == 2) {
        *err = "the persistent launch (tree_exec 2) supports no slicing";
        return QGM_E_UNSUPPORTED;
    }
    if (p.n + int(sliced.size()) > 64) {
        *err = "sliced variables are fixed by the bits above the qubits of a 64-bit word: n + sliced <= 64";
        return QGM_E_UNSUPPORTED;
    }
    Model m;
    std::vector<std::pair<int, int>> kept;
    build_model(p, sliced, m, kept);
    t.sliced = sliced;
    const int nF = int(m.free_var.size());
    t.phase = m.phase;
    t.n_free = nF;
    const std::vector<uint8_t> adj = model_graph(m);
    // candidate orders: deterministic min-degree and min-fill, then randomised tie breaks, ranked by the
    // symbolic cost (bytes before chain merging, a level weighed as 4 KiB per bitstring)
    const int restarts = p.opts.order_restarts > 0 ? p.opts.order_restarts
                                                   : (nF > 1500 ? 1 : (nF > 600 ? 4 : kTreeOrderRestarts));
    std::vector<std::pair<double, std::vector<int>>> cands;
    std::string last_why;
    for (int crit = 0; crit < 2; ++crit)
        for (int rs = 0; rs <= restarts; ++rs) {
            std::vector<int> ord = candidate_order(m, adj, crit, rs);
            SimOut r = simulate(p, m, ord, nullptr, nullptr);
            ++t.n_candidates;
            if (!r.ok) { last_why = r.why; continue; }
            cands.push_back({r.bytes + 4096.0 * r.levels, ord});
        }
    if (cands.empty()) {
        if (nF > 0) { *err = "no elimination order fits the kernels: " + last_why; return QGM_E_UNSUPPORTED; }
        cands.push_back({0.0, {}});
    }
    std::stable_sort(cands.begin(), cands.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    // the first finalists are built in full (chains merged, leaves absorbed, tail chosen) and the plan
    // whose kernels issue the fewest bytes per bitstring, a launch weighed as kTreeLaunchBytes, is kept:
    // merging and absorption change the traffic of each order by different amounts
    const int n_fin = p.opts.order_finalists > 0 ? p.opts.order_finalists : (nF > 600 ? 2 : kTreeOrderFinalists);
    std::vector<std::vector<int>> tried;
    std::vector<std::pair<double, size_t>> scored;   // (score, candidate) of the finalists that build
    qgm_status first_st = QGM_OK;
    std::string first_err;
    for (size_t i = 0; i < cands.size() && int(tried.size()) < n_fin; ++i) {
        if (std::find(tried.begin(), tried.end(), cands[i].second) != tried.end()) continue;
        tried.push_back(cands[i].second);
        TreePlan tc = t;
        std::string e;
        const qgm_status st = tree_from_order(p, m, kept, cands[i].second, tc, &e);
        if (st != QGM_OK) {
            if (first_st == QGM_OK) { first_st = st; first_err = e; }
            continue;
        }
        scored.push_back({tree_issued_bytes_per_b(tc) + kTreeLaunchBytes * tree_launches(tc), i});
    }
    if (scored.empty()) { *err = first_err; return first_st; }
    std::stable_sort(scored.begin(), scored.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    // the lowest score, or the order_pick-th lowest (a caller timing the finalists)
    if (p.opts.order_pick >= int(scored.size())) {
        *err = "order_pick " + std::to_string(p.opts.order_pick) + " beyond the " + std::to_string(scored.size()) +
               " finalists built";
        return QGM_E_INVALID;
    }
    const size_t pick = scored[size_t(p.opts.order_pick)].second;
    TreePlan tc = t;
    const qgm_status st = tree_from_order(p, m, kept, cands[pick].second, tc, err);
    if (st != QGM_OK) return st;
    t = std::move(tc);
    t.n_built = int(scored.size());
    t.order_score = scored[size_t(p.opts.order_pick)].first;
    build_lds_program(t);
    if (p.opts.tree_exec == 3 && !t.lds.ok) {
        *err = "tree_exec 3 (LDS-resident launch) does not fit this plan: " + t.lds.why;
        return QGM_E_UNSUPPORTED;
    }
    return QGM_OK;
}

int tree_pick_slice_var(const Plan& p, const std::vector<int>& sliced, const TreePlan* t) {
    // index spaces (summed and result variables, as variable ids) of the buckets of the built plan, or of
    // the plain min-fill order's buckets without the kernel limits when no order fits
    std::vector<std::vector<int>> spaces;
    if (t) {
        for (const TreeStep& st : t->steps) {
            std::vector<int> sp = st.vars;
            sp.insert(sp.end(), st.out_axes.begin(), st.out_axes.end());
            spaces.push_back(sp);
        }
    } else {
        Model m;
        std::vector<std::pair<int, int>> kept;
        build_model(p, sliced, m, kept);
        if (m.free_var.empty()) return -1;
        const std::vector<int> ord = candidate_order(m, model_graph(m), 1, 0);
        std::vector<RStep> rs;
        std::vector<RTensor> rt;
        SimOut r = simulate(p, m, ord, &rs, &rt, false);
        if (!r.ok) return -1;
        for (const RStep& st : rs) {
            std::vector<int> sp;
            for (int u : st.vars) sp.push_back(m.free_var[u]);
            for (int u : st.out) sp.push_back(m.free_var[u]);
            spaces.push_back(sp);
        }
    }
    int big = 0;
    for (const auto& sp : spaces) big = std::max(big, int(sp.size()));
    // score: sum over the buckets using the variable of 4^(size - largest size), so the variables of the
    // largest buckets come first; open qubits' variables are never sliced
    std::map<int, double> score;
    for (const auto& sp : spaces)
        for (int v : sp)
            if (!(p.vars[v].is_final && p.vars[v].open_idx >= 0)) score[v] += std::ldexp(1.0, 2 * (int(sp.size()) - big));
    int best = -1;
    double bs = 0.0;
    for (const auto& kv : score)
        if (kv.second > bs) { bs = kv.second; best = kv.first; }
    return best;
}

// The plan of one elimination order: buckets, chains merged, leaves absorbed,
// levels, arena rows, wave tasks, the tail and the factor-table layout.
static qgm_status tree_from_order(const Plan& p, const Model& m, const std::vector<std::pair<int, int>>& kept,
                                  const std::vector<int>& best, TreePlan& t, std::string* err) {
    std::vector<RStep> rs;
    std::vector<RTensor> rt;
    SimOut r = simulate(p, m, best, &rs, &rt);
    if (!r.ok) { *err = r.why; return QGM_E_INTERNAL; }
    if (p.opts.no_chain_merge == 0) merge_chains(p, m, rs, rt);
    t.n_absorbed = absorb_leaves(p, m, rs, rt);
    qgm_status fst = finalize_tree(p, m, best, rs, rt, t, err);
    if (fst != QGM_OK) return fst;
    t.n_open = p.n_open;
    t.zero_mask = m.zero_mask;
    for (auto& k : kept) t.open_axis_bit.push_back(k.first);
    for (int u : best) t.order.push_back(m.free_var[u]);
    const int n_levels = int(t.levels.size());
    // last level reading each result (the final product counts as level n_levels)
    const int T = int(t.tensor_axes.size());
    t.tensor_used.assign(T, n_levels);
    for (auto& st : t.steps)
        for (int tid : st.in_tensors) t.tensor_used[tid] = st.level;
    // arena: results whose level intervals overlap get disjoint rows
    std::vector<int> idx(T);
    for (int i = 0; i < T; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return t.tensor_axes[a].size() > t.tensor_axes[b].size(); });
    t.tensor_row.assign(T, -1);
    std::vector<int> placed;
    // a result holds at least 2^kTreeOcBits rows: a wave task writes that many
    auto alloc_rows = [&](int tid) { return int64_t(1) << std::max(int(t.tensor_axes[tid].size()), kTreeOcBits); };
    std::vector<char> is_table(T, 0);
    for (auto& st : t.steps)
        if (st.table_leaf) is_table[st.out_tensor] = 1;
    for (int a : idx) {
        if (is_table[a]) continue;   // lives in the leaf-table area
        const int64_t size = alloc_rows(a);
        std::vector<std::pair<int64_t, int64_t>> busy;
        for (int b : placed)
            if (!(t.tensor_used[b] < t.tensor_made[a] || t.tensor_used[a] < t.tensor_made[b]))
                busy.push_back({t.tensor_row[b], t.tensor_row[b] + alloc_rows(b)});
        std::sort(busy.begin(), busy.end());
        int64_t off = 0;
        for (auto& iv : busy) {
            if (off + size <= iv.first) break;
            off = std::max(off, iv.second);
        }
        t.tensor_row[a] = off;
        t.arena_rows = std::max(t.arena_rows, off + size);
        placed.push_back(a);
    }
    // wave tasks of the buckets with inputs, grouped by level (a level is one launch)
    t.level_task_off.assign(1, 0);
    t.level_max_in.clear();
    t.level_quad.clear();
    t.level_quad_arena.clear();
    std::vector<char> leaf_made(t.tensor_axes.size(), 0);   // results that are leaf tables
    for (const TreeStep& st : t.steps)
        if (st.table_leaf) leaf_made[size_t(st.out_tensor)] = 1;
    for (size_t L = 0; L < t.levels.size(); ++L) {
        int mi = 0;
        for (int sid : t.levels[L]) mi = std::max(mi, int(t.steps[sid].in_tensors.size()));
        const int nin = launch_inputs(mi);
        for (int sid : t.levels[L]) {
            TreeStep& st = t.steps[sid];
            // the 32-row tile runs in the 2- and 3-input launches of levels that are not the tail's (it holds
            // 64 accumulator registers, more than the wider launches leave); elsewhere its 8-row form
            if (st.tile >= 3 && (nin > 3 || st.out_axes.size() < 10)) st.tile -= 2;
            st.quad = st.quad && st.tile == 3 && !st.table_leaf;
            st.unit_rows = st.tile >= 3 ? 32 : (st.tile ? (1 << kTreeOcBits) : tree_unit_rows(nin, st.kg));
        }
        // the quad tiles' tasks first (their launch takes blocks of four tasks)
        std::stable_partition(t.levels[L].begin(), t.levels[L].end(), [&](int sid) { return t.steps[sid].quad; });
        int64_t nq = 0;
        char arena = 1;
        for (int sid : t.levels[L]) {
            TreeStep& st = t.steps[sid];
            st.task_off = t.n_tasks;
            t.n_tasks += st.n_tasks();
            if (st.quad) {
                nq += st.n_tasks();
                for (int tin : st.in_tensors)
                    if (leaf_made[size_t(tin)]) arena = 0;
            }
        }
        t.level_task_off.push_back(t.n_tasks);
        t.level_max_in.push_back(mi);
        t.level_quad.push_back(nq);
        t.level_quad_arena.push_back(arena);
    }
    // tail: the longest run of last levels with few tasks and few inputs
    t.first_level = 0;
    while (t.first_level < int(t.levels.size()) && t.levels[t.first_level].empty()) ++t.first_level;
    // (its task records and the results it makes are kept in LDS: at most kTreeTailMaxTasks records and
    // kTreeTailLdsRows rows over all its levels)
    t.tail_start = int(t.levels.size());
    int64_t tail_tasks = 0, tail_rows = 0, tail_g = 0;
    while (t.n_open == 0 && t.tail_start > std::max(t.first_level, 1) &&   // the tail writes one amplitude per b
           int(t.finals.size()) <= kTreeTailMaxFinal && int(t.levels.size()) - t.tail_start < kTreeTailMaxLevels) {
        const int L = t.tail_start - 1;
        const int64_t nt = t.level_task_off[L + 1] - t.level_task_off[L];
        if (nt > kTreeTailTasks || launch_inputs(t.level_max_in[L]) > kTreeTailInputs) break;
        int64_t rows = 0, ge = 0;
        bool big_tile = false;   // the tail kernel has no 32-row tile unit
        for (int sid : t.levels[L]) {
            rows += alloc_rows(t.steps[sid].out_tensor);
            ge += t.steps[sid].g_entries();
            big_tile = big_tile || t.steps[sid].tile >= 3;
        }
        if (big_tile) break;
        if (tail_tasks + nt > kTreeTailMaxTasks || tail_rows + rows > kTreeTailLdsRows ||
            tail_g + ge > kTreeTailGEntries)
            break;
        tail_tasks += nt;
        tail_rows += rows;
        tail_g += ge;
        t.tail_start = L;
    }
    t.tail_lds_row.assign(T, -1);
    t.tail_lds_rows = 0;
    for (int L = t.tail_start; L < int(t.levels.size()); ++L)
        for (int sid : t.levels[L]) {
            t.tail_lds_row[t.steps[sid].out_tensor] = t.tail_lds_rows;
            t.tail_lds_rows += int(alloc_rows(t.steps[sid].out_tensor));
        }
    // factor tables: the buckets before the tail, then the tail's buckets in one range (which the tail
    // kernel copies to LDS), the leaf tables, the constant 1, and the FP64 values of the factors without
    // free variables (4 per factor, two float2 entries each)
    std::vector<char> in_tail(t.steps.size(), 0);
    for (int L = t.tail_start; L < int(t.levels.size()); ++L)
        for (int sid : t.levels[L]) in_tail[size_t(sid)] = 1;
    int64_t g = 0;
    for (size_t i = 0; i < t.steps.size(); ++i)
        if (!in_tail[i]) {
            t.steps[i].g_off = g;
            g += t.steps[i].g_entries();
        }
    g += g & 1;                   // 16-byte alignment of the tail's range
    t.tail_g0 = g;
    for (size_t i = 0; i < t.steps.size(); ++i)
        if (in_tail[i]) {
            t.steps[i].g_off = g;
            g += t.steps[i].g_entries();
        }
    t.tail_g_entries = g - t.tail_g0;
    for (auto& st : t.steps)
        if (st.table_leaf) {
            st.leaf_off = g;
            g += int64_t(1) << (st.out_axes.size() + st.sig_q.size());
        }
    t.ones_g = g;                 // constant 1 read for inputs a bucket does not have
    g += 1;
    g += g & 1;                   // 16-byte alignment of the FP64 values
    t.phase_g = g;
    g += 8 * std::max<int64_t>(1, int64_t(t.phase.size()));   // at least one factor's room (read, unused)
    t.g_total = g;
    // adjoint layout: each result at its own rows; per level, the expansion scratch of its buckets
    t.tensor_row_all.assign(T, 0);
    t.arena_rows_all = 0;
    for (int i = 0; i < T; ++i) {
        if (is_table[i]) { t.tensor_row_all[i] = -1; continue; }
        t.tensor_row_all[i] = t.arena_rows_all;
        t.arena_rows_all += alloc_rows(i);
    }
    t.scratch_row.assign(t.steps.size(), 0);
    t.hsum_row.assign(t.steps.size(), 0);
    t.scratch_rows = 0;
    t.hsum_rows = 0;   // every bucket keeps its own rows of H sums: the table adjoints are taken after the sweep
    for (auto& lvl : t.levels) {
        int64_t rows = 0;
        for (int sid : lvl) {
            const TreeStep& st = t.steps[sid];
            t.scratch_row[sid] = rows;
            rows += int64_t(st.in_tensors.size() + 1) << (st.out_axes.size() + st.vars.size());
            t.hsum_row[sid] = t.hsum_rows;
            t.hsum_rows += int64_t(1) << (st.gb() + st.kg);
        }
        t.scratch_rows = std::max(t.scratch_rows, rows);
    }
    for (auto& st : t.steps)
        if (st.groups.size() > 16) { *err = "internal: more than 16 factor groups"; return QGM_E_INTERNAL; }
    if (t.n_tasks > kTreeMaxTasks || t.arena_rows >= (int64_t(1) << 31) || t.g_total >= (int64_t(1) << 31) ||
        t.arena_rows_all >= (int64_t(1) << 31)) {
        *err = "bucket plan too large for the device tables (results of rank > 24)";
        return QGM_E_UNSUPPORTED;
    }
    return QGM_OK;
}

// Row loads and stores one wave unit of a bucket issues (64 lanes x 8 bytes
// each): the distinct input rows (an input is read once for the unit rows
// and summed values it does not vary along), the constant 1 for each input
// slot beyond the bucket's own, the distinct factor-table entries, and the
// unit's result rows.
int64_t tree_unit_accesses(const TreePlan& t, const TreeStep& st) {
    if (st.table_leaf) return 0;
    if (st.tile >= 3)   // 8 + 4 (+ 1) input rows and a table row per summed value
        return (int64_t(8 + 4 + 1 + (st.tile == 4 ? 1 : 0)) << st.kg) + st.unit_rows;
    if (st.tile)   // 4 + 2 (+ 1) input rows and a table row per summed value
        return (int64_t(4 + 2 + 1 + (st.tile == 2 ? 1 : 0)) << st.kg) + st.unit_rows;
    const int ob_bits = __builtin_ctz(uint32_t(st.unit_rows));
    const int r = int(st.out_axes.size());
    auto count_in = [&](const std::vector<int>& ax, int lo, int hi, const std::vector<int>& from) {
        int n = 0;
        for (int j = lo; j < hi && j < int(from.size()); ++j)
            if (std::find(ax.begin(), ax.end(), from[j]) != ax.end()) ++n;
        return n;
    };
    int64_t n = 0;
    for (int tid : st.in_tensors) {
        const std::vector<int>& ax = t.tensor_axes[tid];
        n += int64_t(1) << (count_in(ax, 0, std::min(ob_bits, r), st.out_axes) + count_in(ax, 0, st.kg, st.vars));
    }
    const int cls = launch_inputs(t.level_max_in[st.level]);
    n += cls - int(st.in_tensors.size());
    n += int64_t(1) << (count_in(st.gvars, 0, std::min(ob_bits, r), st.out_axes) + st.kg);
    return n + st.unit_rows;
}

double tree_issued_bytes_per_b(const TreePlan& t) {
    double n = 0;
    for (const TreeStep& st : t.steps) n += 8.0 * double(st.n_tasks()) * double(tree_unit_accesses(t, st));
    return n;
}

int tree_launches(const TreePlan& t) {
    return std::max(t.tail_start - t.first_level, 0) + (t.tail_start < int(t.levels.size()) ? 1 : 0);
}

int tree_kernel_launches(const TreePlan& t) {
    int n = t.tail_start < int(t.levels.size()) ? 1 : 0;
    for (int L = t.first_level; L < t.tail_start; ++L) {   // a level with quad tiles and other tasks: two launches
        const int64_t nq = L < int(t.level_quad.size()) ? t.level_quad[size_t(L)] : 0;
        n += (nq > 0 ? 1 : 0) + (t.level_task_off[size_t(L) + 1] - t.level_task_off[size_t(L)] > nq ? 1 : 0);
    }
    return n;
}

}  // namespace qgm
