// C ABI of libqgm: plan construction (host), device table upload, and the
// amplitude executor that enqueues the step kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "qgm.h"

struct qgm_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct qgm_plan_s {
    qgm::Plan p;
    uint32_t max_g_entries = 0;
    // offsets (bytes) of the constant tables inside each device copy
    size_t off_fixed = 0, off_steps = 0, off_ops = 0, off_sig = 0, off_final = 0, total = 0;
    // adjoint tables: per-step wave offsets of the G-entry waves, per-slot (step, op) lists
    size_t off_wave_base = 0, off_step_waves = 0, off_slot_off = 0, off_slot_ops = 0;
    std::vector<int64_t> wave_base;
    std::vector<int32_t> step_waves, slot_off, slot_ops;
    int64_t total_waves = 0;
    int max_ops = 1;
    // tree plans (ordering 1): offsets of the bucket records, factor tables, phase and final rows
    size_t off_ttasks = 0, off_tgtab = 0, off_tgroup = 0, off_tfac = 0, off_ttail = 0, off_tphase = 0, off_tfinal = 0;
    size_t off_tttasks = 0, off_ttfin = 0;   // the tail's task copies (results made in the tail in LDS), its finals
    int n_gtabs = 0;
    size_t off_tpro = 0, off_tg = 0;   // prologue block list; factor tables of a plan without gate values
    int n_pro_blocks = 0;     // prologue blocks of the factor tables (the adjoint's table blocks too)
    int n_pro_phase = 0;      // then the blocks of the phase values (prologue only)
    size_t off_tphq = 0;      // bits read by each phase factor, as the tail stages them
    // tree plans, adjoint: keep-all tasks and final rows, per-bucket records, per-level item lists, slot lists
    size_t off_ttasks_all = 0, off_tfinal_all = 0, off_tbwd = 0, off_tbwdin = 0, off_tbwdg = 0, off_titems = 0;
    size_t off_tslot_off = 0, off_tslot_occ = 0;
    size_t off_tfdep = 0;   // (first task, count) of the bucket making each rank-0 result
    size_t off_tleaf = 0;   // leaf-table records (plans without gate values)
    struct LevelItems { int off = 0, n = 0; int64_t rows = 0; };
    std::vector<LevelItems> lv_exp;
    LevelItems g_all;   // every bucket's table adjoint rows, one launch after the adjoint sweep
    std::vector<std::vector<LevelItems>> lv_red;   // per level: the stages of its staged sums
    std::vector<qgm::TreeBwdIn> red_recs;
    int64_t part_rows[2] = {0, 0};                 // rows of the two partial-sum areas
    std::vector<qgm::TreeBwdItem> items;
    std::vector<int32_t> slot_off_t, slot_occ_t;
    int64_t n_fbar = 0;
    std::vector<int64_t> part_off;   // per factor: first partial sum of its adjoint (n_fbar + 1 entries)
    size_t off_tpart = 0;
    size_t off_status = 0;           // int32 failure record of persistent launches (0: none since the last check)
    // the LDS-resident program (tree plans whose results fit a work-group's LDS)
    size_t off_lstage = 0, off_lentry = 0, off_lrec = 0, off_llvl = 0, off_lfin = 0, off_lzent = 0, off_lz = 0;
    size_t off_lgent = 0;
    // optional per-phase timing
    bool timing = false;
    std::vector<hipEvent_t> events;   // 5 per timed call
    size_t events_used = 0;
};

namespace {

thread_local std::string g_err;

qgm_status fail(qgm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

qgm_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return QGM_E_HIP;
}

// The fixed single-qubit gates of Sec. II, row = the state after the gate.
// H: the table of App. D; T = diag(1, e^{i pi/4}); X^1/2 = RX(pi/2) and
// Y^1/2 = RY(pi/2), whose relative phases are those of App. F, Eq. (phX).
void fixed_matrices(double2 m[qgm::kFixedMats * 4]) {
    const double r = 1.0 / std::sqrt(2.0);
    const double2 H[4] = {{r, 0}, {r, 0}, {r, 0}, {-r, 0}};
    const double2 T[4] = {{1, 0}, {0, 0}, {0, 0}, {std::cos(M_PI / 4), std::sin(M_PI / 4)}};
    const double2 X[4] = {{r, 0}, {0, -r}, {0, -r}, {r, 0}};
    const double2 Y[4] = {{r, 0}, {-r, 0}, {r, 0}, {r, 0}};
    const double2 Tdg[4] = {{1, 0}, {0, 0}, {0, 0}, {std::cos(M_PI / 4), -std::sin(M_PI / 4)}};
    const double2 Xdg[4] = {{r, 0}, {0, r}, {0, r}, {r, 0}};
    const double2 Ydg[4] = {{r, 0}, {r, 0}, {-r, 0}, {r, 0}};
    const double2 PX[4] = {{0, 0}, {1, 0}, {1, 0}, {0, 0}};
    const double2 PY[4] = {{0, 0}, {0, -1}, {0, 1}, {0, 0}};
    const double2 PZ[4] = {{1, 0}, {0, 0}, {0, 0}, {-1, 0}};
    const double2* all[qgm::kFixedMats] = {H, T, X, Y, Tdg, Xdg, Ydg, PX, PY, PZ};
    for (int k = 0; k < qgm::kFixedMats; ++k)
        for (int i = 0; i < 4; ++i) m[k * 4 + i] = all[k][i];
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Bit of a bucket's index space a = (o << k) | w that holds a variable: summed
// variable i -> i, result axis j -> k + j (-1 if the bucket does not carry it).
int bucket_abit(const qgm::TreeStep& st, int var) {
    const int k = st.kg;
    for (int i = 0; i < k; ++i)
        if (st.vars[i] == var) return i;
    for (size_t j = 0; j < st.out_axes.size(); ++j)
        if (st.out_axes[j] == var) return k + int(j);
    return -1;
}

void layout_tree_tables(qgm_plan_t* P) {
    const qgm::TreePlan& t = P->p.tree;
    size_t n_fac = 0, n_groups = 0;
    P->n_gtabs = int(t.steps.size());
    P->n_pro_blocks = 0;
    for (auto& st : t.steps) {
        n_fac += size_t(st.n_factors());
        n_groups += st.groups.size();
        P->n_pro_blocks += int((st.g_entries() + 255) / 256);
    }
    P->n_pro_phase = int((4 * t.phase.size() + 255) / 256);
    const size_t n_tail = t.levels.size() - size_t(t.tail_start);
    P->off_fixed = 0;
    P->off_ttasks = al(sizeof(double2) * qgm::kFixedMats * 4);
    P->off_tgtab = P->off_ttasks + al(sizeof(qgm::TreeTask) * size_t(t.n_tasks + 1));
    P->off_tgroup = P->off_tgtab + al(sizeof(qgm::TreeGTab) * (size_t(P->n_gtabs) + 1));
    P->off_tfac = P->off_tgroup + al(sizeof(qgm::TreeGroup) * (n_groups + 1));
    P->off_ttail = P->off_tfac + al(sizeof(qgm::TFactor) * (n_fac + 1));
    P->off_tphase = P->off_ttail + al(sizeof(qgm::TreeTailLevel) * (n_tail + 1));
    P->off_tfinal = P->off_tphase + al(sizeof(qgm::TFactor) * (t.phase.size() + 1));
    const int64_t n_tail_tasks = t.n_tasks - (n_tail > 0 ? t.level_task_off[size_t(t.tail_start)] : t.n_tasks);
    P->off_tttasks = P->off_tfinal + al(sizeof(int64_t) * (t.finals.size() + 1));
    P->off_ttfin = P->off_tttasks + al(sizeof(qgm::TreeTask) * size_t(n_tail_tasks + 1));
    P->off_tpro = P->off_ttfin + al(sizeof(int32_t) * (t.finals.size() + 1));
    P->off_tphq = P->off_tpro + al(sizeof(qgm::TreeProBlock) * size_t(P->n_pro_blocks + P->n_pro_phase + 1));
    P->off_tg = P->off_tphq + al(sizeof(int32_t) * 2 * (t.phase.size() + 1));
    // adjoint records and item lists (level by level: expansion, staged sums, table adjoints)
    P->items.clear();
    P->red_recs.clear();
    P->part_rows[0] = P->part_rows[1] = 0;
    P->lv_exp.assign(t.levels.size(), {});
    P->lv_red.assign(t.levels.size(), {});
    P->g_all = {};
    auto add = [&](qgm_plan_s::LevelItems& li, int idx, int64_t rows) {
        if (li.n == 0) li.off = int(P->items.size());
        P->items.push_back({idx, int32_t(li.rows)});
        li.rows += rows;
        li.n++;
    };
    for (size_t L = 0; L < t.levels.size(); ++L) {
        for (int sid : t.levels[L]) {
            const qgm::TreeStep& st = t.steps[sid];
            add(P->lv_exp[L], sid, int64_t(1) << (st.out_axes.size() + st.vars.size()));
        }
        // every sum of the level: each input's adjoint (Q_t over the a-bits that are
        // not its axes) and, with gate slots, H over the a-bits outside the table index
        struct Sum {
            int64_t q_row;
            std::vector<int> axes, free;   // source-row bits of the output index; bits still to sum
            int32_t sel, row;              // final destination
        };
        std::vector<Sum> sums;
        for (int sid : t.levels[L]) {
            const qgm::TreeStep& st = t.steps[sid];
            const int a_bits = int(st.out_axes.size()) + st.kg;
            for (size_t k = 0; k < st.in_tensors.size(); ++k) {
                const int tid = st.in_tensors[k];
                Sum u{t.scratch_row[sid] + int64_t(1 + k) * (int64_t(1) << a_bits), {}, {}, 0,
                      int32_t(t.tensor_row_all[tid])};
                std::vector<bool> used(a_bits, false);
                for (int v : t.tensor_axes[tid]) {
                    const int ab = bucket_abit(st, v);
                    u.axes.push_back(ab);
                    used[ab] = true;
                }
                for (int i = 0; i < a_bits; ++i)
                    if (!used[i]) u.free.push_back(i);
                sums.push_back(u);
            }
            if (P->p.n_slots > 0) {
                Sum u{t.scratch_row[sid], {}, {}, 1, int32_t(t.hsum_row[sid])};
                std::vector<bool> used(a_bits, false);
                for (int i = 0; i < st.kg; ++i) u.axes.push_back(i);
                for (int v : st.gvars) u.axes.push_back(bucket_abit(st, v));
                for (int ab : u.axes) used[ab] = true;
                for (int i = 0; i < a_bits; ++i)
                    if (!used[i]) u.free.push_back(i);
                sums.push_back(u);
            }
        }
        // stage s sums up to kTbSumBits bits of every unfinished sum; a sum with bits
        // left writes partial rows (its remaining bits above its axes) to area s % 2
        for (int stage = 0; !sums.empty(); ++stage) {
            P->lv_red[L].push_back({});
            int64_t prow = 0;
            std::vector<Sum> next;
            for (Sum& u : sums) {
                const int m = std::min<int>(qgm::kTbSumBits, int(u.free.size()));
                const int rest = int(u.free.size()) - m;
                qgm::TreeBwdIn e{};
                e.r_t = int32_t(u.axes.size()) + rest;
                e.n_sum = m;
                e.q_row = u.q_row;
                for (size_t p = 0; p < u.axes.size(); ++p) e.pos[p] = u.axes[p];
                for (int i = 0; i < rest; ++i) e.pos[u.axes.size() + i] = u.free[m + i];
                for (int f = 0; f < (1 << m); ++f) {
                    int32_t o = 0;
                    for (int i = 0; i < m; ++i)
                        if ((f >> i) & 1) o += int32_t(1) << u.free[i];
                    e.foff[f] = o;
                }
                if (rest == 0) {
                    e.dst_sel = u.sel;
                    e.dst_row = u.row;
                } else {
                    e.dst_sel = 2;
                    e.dst_row = int32_t(prow);
                    Sum w{prow, {}, {}, u.sel, u.row};
                    for (size_t p = 0; p < u.axes.size(); ++p) w.axes.push_back(int(p));
                    for (int i = 0; i < rest; ++i) w.free.push_back(int(u.axes.size()) + i);
                    prow += int64_t(1) << e.r_t;
                    next.push_back(w);
                }
                add(P->lv_red[L].back(), int(P->red_recs.size()), int64_t(1) << e.r_t);
                P->red_recs.push_back(e);
            }
            P->part_rows[stage % 2] = std::max(P->part_rows[stage % 2], prow);
            sums.swap(next);
        }
    }
    for (size_t L = 0; L < t.levels.size(); ++L)
        for (int sid : t.levels[L]) {
            const qgm::TreeStep& st = t.steps[sid];
            add(P->g_all, sid, int64_t(1) << (st.gb() + st.kg));
        }
    // gate-slot occurrences among the table factors and the phase factors
    {
        std::vector<std::vector<int32_t>> occ(std::max(P->p.n_slots, 0));
        int gi = 0;
        auto note = [&](const qgm::TFactor& f, int index) {
            if ((f.type == qgm::TF_MAT || f.type == qgm::TF_DIAG) && f.mat >= qgm::kFixedMats)
                occ[f.mat - qgm::kFixedMats].push_back(int32_t(index) * 2 + (f.type == qgm::TF_DIAG ? 1 : 0));
        };
        auto is_slot = [](const qgm::TFactor& f) {
            return (f.type == qgm::TF_MAT || f.type == qgm::TF_DIAG) && f.mat >= qgm::kFixedMats;
        };
        // partial sums of the factor adjoints: one per table block for a table factor, one per summing block
        // for a phase factor (factors without a gate slot have none)
        P->part_off.assign(1, 0);
        for (auto& st : t.steps)
            for (auto& g : st.groups)
                for (auto& f : g.factors) {
                    note(f, gi++);
                    P->part_off.push_back(P->part_off.back() + (is_slot(f) ? (st.g_entries() + 255) / 256 : 0));
                }
        P->n_fbar = gi + int64_t(t.phase.size());
        for (size_t i = 0; i < t.phase.size(); ++i) {
            note(t.phase[i], gi + int(i));
            P->part_off.push_back(P->part_off.back() + (is_slot(t.phase[i]) ? int64_t(qgm::kTbPhaseBlocks) : 0));
        }
        P->slot_off_t.assign(1, 0);
        P->slot_occ_t.clear();
        for (auto& v : occ) {
            for (int32_t x : v) P->slot_occ_t.push_back(x);
            P->slot_off_t.push_back(int32_t(P->slot_occ_t.size()));
        }
    }
    const size_t g_bytes = P->p.n_slots == 0 ? al(sizeof(float2) * size_t(t.g_total)) : 0;
    P->off_ttasks_all = P->off_tg + g_bytes;
    P->off_tfinal_all = P->off_ttasks_all + al(sizeof(qgm::TreeTask) * size_t(t.n_tasks + 1));
    P->off_tbwd = P->off_tfinal_all + al(sizeof(int64_t) * (t.finals.size() + 1));
    P->off_tbwdin = P->off_tbwd + al(sizeof(qgm::TreeBwd) * (t.steps.size() + 1));
    P->off_tbwdg = P->off_tbwdin + al(sizeof(qgm::TreeBwdIn) * (P->red_recs.size() + 1));
    P->off_titems = P->off_tbwdg + al(sizeof(qgm::TreeBwdG) * (t.steps.size() + 1));
    P->off_tslot_off = P->off_titems + al(sizeof(qgm::TreeBwdItem) * (P->items.size() + 1));
    P->off_tslot_occ = P->off_tslot_off + al(sizeof(int32_t) * (P->slot_off_t.size() + 1));
    P->off_tfdep = P->off_tslot_occ + al(sizeof(int32_t) * (P->slot_occ_t.size() + 1));
    P->off_tleaf = P->off_tfdep + al(sizeof(int32_t) * 2 * (t.finals.size() + 1));
    P->off_tpart = P->off_tleaf + al(sizeof(qgm::TreeLeaf) * size_t(t.n_table_leaves + 1));
    const qgm::LdsProgram& lp = t.lds;
    P->off_lstage = P->off_tpart + al(sizeof(int64_t) * P->part_off.size());
    P->off_lentry = P->off_lstage + al(sizeof(qgm::LdsStage) * (lp.stages.size() + 1));
    P->off_lrec = P->off_lentry + al(sizeof(qgm::LdsEntry) * (lp.entries.size() + 1));
    P->off_llvl = P->off_lrec + al(sizeof(uint16_t) * (lp.recs.size() + 8));
    P->off_lfin = P->off_llvl + al(sizeof(int32_t) * (lp.level_job_off.size() + 1));
    P->off_lzent = P->off_lfin + al(sizeof(int32_t) * (lp.finals.size() + 1));
    P->off_lgent = P->off_lzent + al(sizeof(uint32_t) * (lp.zent.size() + 1));
    P->off_lz = P->off_lgent + al(sizeof(uint32_t) * (lp.gent.size() + 1));
    // the staged copy of the LDS launch's tables: built once here when the circuit reads no gate values
    P->total = P->off_lz + (P->p.n_slots == 0 ? al(sizeof(float2) * size_t(lp.z_entries + 1)) : 0);
}

// Adjoint tables: the forward tasks with every result at its own rows
// (keep-all layout), the per-bucket expansion records, the input-adjoint and
// table-adjoint records, the level item lists and the gate-slot lists.
void fill_tree_adjoint_tables(const qgm_plan_t* P, char* h) {
    const qgm::TreePlan& t = P->p.tree;
    const auto* tasks = reinterpret_cast<const qgm::TreeTask*>(h + P->off_ttasks);
    auto* tasks_all = reinterpret_cast<qgm::TreeTask*>(h + P->off_ttasks_all);
    // keep-all rows: every row of the forward layout is relocated by its tensor
    std::vector<int64_t> shift(t.tensor_axes.size());
    for (size_t i = 0; i < shift.size(); ++i) shift[i] = t.tensor_row_all[i] - t.tensor_row[i];
    for (size_t sid = 0; sid < t.steps.size(); ++sid) {
        const qgm::TreeStep& st = t.steps[sid];
        if (st.table_leaf) continue;
        for (int64_t c = 0; c < st.n_tasks(); ++c) {
            qgm::TreeTask tk = tasks[st.task_off + c];
            tk.out_row = int32_t(tk.out_row + shift[st.out_tensor]);
            for (size_t k = 0; k < st.in_tensors.size(); ++k)
                if (tk.in_tab[k] < 0) tk.in_row[k] = int32_t(tk.in_row[k] + shift[st.in_tensors[k]]);
            tasks_all[st.task_off + c] = tk;
        }
    }
    auto* fa = reinterpret_cast<int64_t*>(h + P->off_tfinal_all);
    for (size_t i = 0; i < t.finals.size(); ++i) fa[i] = t.tensor_row_all[t.finals[i]];
    auto* bw = reinterpret_cast<qgm::TreeBwd*>(h + P->off_tbwd);
    auto* bg = reinterpret_cast<qgm::TreeBwdG*>(h + P->off_tbwdg);
    for (size_t sid = 0; sid < t.steps.size(); ++sid) {
        const qgm::TreeStep& st = t.steps[sid];
        const int r = int(st.out_axes.size()), k = st.kg;
        qgm::TreeBwd d{};
        d.n_in = int32_t(st.in_tensors.size());
        d.k = k;
        d.r = r;
        d.sb = st.sb();
        d.a_bits = r + k;
        d.out_row = int32_t(t.tensor_row_all[st.out_tensor]);
        d.scratch_row = t.scratch_row[sid];
        d.g_off = st.g_off;
        for (int b = 0; b < st.sb(); ++b) d.sig_q[b] = st.sig_q[b];
        for (int i = 0; i < k; ++i) d.g_str[i] = 1 << i;
        for (int j = 0; j < r; ++j)
            for (int p = 0; p < st.gb(); ++p)
                if (st.out_axes[j] == st.gvars[p]) d.g_str[k + j] = 1 << (k + p);
        for (int ti = 0; ti < d.n_in; ++ti) {
            const int tid = st.in_tensors[ti];
            const std::vector<int>& ax = t.tensor_axes[tid];
            d.in_row[ti] = int32_t(t.tensor_row_all[tid]);
            for (int p = 0; p < int(ax.size()); ++p) d.in_str[ti][bucket_abit(st, ax[p])] = 1 << p;
        }
        bw[sid] = d;
        qgm::TreeBwdG g{};
        g.c_bits = st.gb() + k;
        g.sb = st.sb();
        g.h_row = t.hsum_row[sid];
        g.g_off = st.g_off;
        for (int b = 0; b < st.sb(); ++b) g.sig_q[b] = st.sig_q[b];
        bg[sid] = g;
    }
    std::memcpy(h + P->off_tbwdin, P->red_recs.data(), sizeof(qgm::TreeBwdIn) * P->red_recs.size());
    std::memcpy(h + P->off_titems, P->items.data(), sizeof(qgm::TreeBwdItem) * P->items.size());
    std::memcpy(h + P->off_tslot_off, P->slot_off_t.data(), sizeof(int32_t) * P->slot_off_t.size());
    std::memcpy(h + P->off_tslot_occ, P->slot_occ_t.data(), sizeof(int32_t) * P->slot_occ_t.size());
    std::memcpy(h + P->off_tpart, P->part_off.data(), sizeof(int64_t) * P->part_off.size());
}

// Device records of the buckets: the row stride of every result bit and
// every summed variable in every input (the index arithmetic of the bucket
// product), one task record per wave unit of result rows, the factor tables'
// groups and factors, the tail levels and the prologue's block list.
bool fill_tree_tables(const qgm_plan_t* P, char* h) {
    const qgm::TreePlan& t = P->p.tree;
    auto* tasks = reinterpret_cast<qgm::TreeTask*>(h + P->off_ttasks);
    auto* gt = reinterpret_cast<qgm::TreeGTab*>(h + P->off_tgtab);
    auto* grp = reinterpret_cast<qgm::TreeGroup*>(h + P->off_tgroup);
    auto* fac = reinterpret_cast<qgm::TFactor*>(h + P->off_tfac);
    auto* pro = reinterpret_cast<qgm::TreeProBlock*>(h + P->off_tpro);
    int n_fac = 0, n_grp = 0, n_pro = 0;
    std::vector<char> task_written(size_t(t.n_tasks), 0);   // every task record is written exactly once
    bool tasks_ok = true;
    std::vector<int> maker(t.tensor_axes.size(), -1);   // bucket that makes each result
    for (size_t i = 0; i < t.steps.size(); ++i) maker[t.steps[i].out_tensor] = int(i);
    for (size_t i = 0; i < t.steps.size(); ++i) {
        const qgm::TreeStep& st = t.steps[i];
        const int r = int(st.out_axes.size());
        qgm::TreeGTab g{};
        g.gb = st.gb();
        g.sb = st.sb();
        g.k = st.kg;
        g.n_groups = int32_t(st.groups.size());
        g.group_off = n_grp;
        g.n_fac = st.n_factors();
        g.g_off = st.g_off;
        for (auto& gr : st.groups) {
            grp[n_grp++] = {n_fac, int32_t(gr.factors.size()), gr.k_int, 0};
            for (auto& f : gr.factors) fac[n_fac++] = f;
        }
        for (int64_t sub = 0; sub < (st.g_entries() + 255) / 256; ++sub) pro[n_pro++] = {int32_t(i), int32_t(sub)};
        gt[i] = g;
        const int n_in = int(st.in_tensors.size());
        qgm::TreeTask base{};
        base.k = st.kg;
        base.n_sig = st.sb();
        base.sb = st.sb();
        base.gshift = st.kg + st.sb();
        base.n_in = n_in;
        base.nin_class = qgm::launch_inputs(t.level_max_in[st.level]);
        base.tile = st.tile;
        for (int b = 0; b < st.sb(); ++b) base.sig_q[b] = st.sig_q[b];
        for (int k = 0; k < qgm::kTreeMaxIn; ++k) base.in_tab[k] = -1;
        for (int k = 0; k < n_in; ++k) {
            const qgm::TreeStep& mk = t.steps[maker[st.in_tensors[k]]];
            if (mk.table_leaf) {   // read per lane from its table; nothing to wait for
                base.in_tab[k] = int32_t(mk.leaf_off);
                base.in_tsb[k] = mk.sb();
                uint64_t pack = 0;
                for (int b = 0; b < mk.sb(); ++b) pack |= uint64_t(mk.sig_q[b]) << (6 * b);
                base.in_tsig[k] = pack;
                continue;
            }
            base.dep_off[k] = int32_t(mk.task_off);
            base.dep_n[k] = int32_t(mk.n_tasks());
        }
        std::vector<std::vector<int64_t>> str(n_in, std::vector<int64_t>(r, 0));
        std::vector<int64_t> gstr(r, 0);
        for (int k = 0; k < n_in; ++k) {
            const std::vector<int>& ax = t.tensor_axes[st.in_tensors[k]];
            for (int a = 0; a < int(ax.size()); ++a) {
                for (size_t v = 0; v < st.vars.size(); ++v)
                    if (ax[a] == st.vars[v]) base.in_vs[k][v] = 1 << a;
                for (int j = 0; j < r; ++j)
                    if (st.out_axes[j] == ax[a]) str[k][j] = int64_t(1) << a;
            }
            int64_t low = 0;
            for (int j = 0; j < qgm::kTreeOcBits; ++j) {   // wrapped beyond the result's rank
                const int64_t sj = j < r ? str[k][j] : 0;
                base.in_inc[k][j] = int32_t(sj - low);
                low += sj;
                if (sj != 0) base.in_omask[k] |= 1 << j;
            }
        }
        if (st.tile >= 3) {   // the 32-row tile: row strides of A's unit bits 0, 1, 3 and of B's 2, 4
            const int abit[3] = {0, 1, 3}, bbit[2] = {2, 4};
            for (int j = 0; j < 3; ++j) base.in_inc[0][j] = int32_t(str[0][abit[j]]);
            for (int j = 0; j < 2; ++j) base.in_inc[1][j] = int32_t(str[1][bbit[j]]);
            base.in_inc[1][2] = 0;
            if (n_in > 2)
                for (int j = 0; j < qgm::kTreeOcBits; ++j) base.in_inc[2][j] = 0;
        }
        for (int j = 0; j < r; ++j)
            for (int gi = 0; gi < st.gb(); ++gi)
                if (st.out_axes[j] == st.gvars[gi]) gstr[j] = int64_t(1) << gi;
        int64_t low = 0;
        for (int j = 0; j < qgm::kTreeOcBits; ++j) {
            const int64_t sj = j < r ? gstr[j] : 0;
            base.g_inc[j] = int32_t(sj - low);
            low += sj;
            if (sj != 0) base.g_omask |= 1 << j;
        }
        // task c covers result rows [c * unit_rows, (c + 1) * unit_rows), wrapping for small results (a leaf
        // table has no tasks: the plan builds it)
        const int64_t n_ch = st.table_leaf ? 0 : st.n_tasks();
        for (int64_t c = 0; c < n_ch; ++c) {
            const int64_t o0 = c * st.unit_rows;
            qgm::TreeTask tk = base;
            tk.out_row = int32_t(t.tensor_row[st.out_tensor] + o0);
            int64_t g0 = 0;
            for (int j = 0; j < r; ++j)
                if ((o0 >> j) & 1) g0 += gstr[j];
            tk.g_ent = int32_t(st.g_off + (g0 << base.gshift));
            for (int k = 0; k < qgm::kTreeMaxIn; ++k) {
                if (k >= n_in) { tk.in_row[k] = -1; continue; }
                // a leaf table's rows count from 0 within it
                int64_t row = base.in_tab[k] >= 0 ? 0 : t.tensor_row[st.in_tensors[k]];
                for (int j = 0; j < r; ++j)
                    if ((o0 >> j) & 1) row += str[k][j];
                tk.in_row[k] = int32_t(row);
            }
            const int64_t ti = st.task_off + c;
            if (ti < 0 || ti >= t.n_tasks || task_written[size_t(ti)]) { tasks_ok = false; continue; }
            task_written[size_t(ti)] = 1;
            tasks[ti] = tk;
        }
    }
    for (char w : task_written) tasks_ok = tasks_ok && w;
    if (!tasks_ok || n_pro != P->n_pro_blocks) return false;
    for (int sub = 0; sub < P->n_pro_phase; ++sub) pro[n_pro++] = {-1, sub};   // the phase values
    auto* phq = reinterpret_cast<int32_t*>(h + P->off_tphq);
    for (size_t i = 0; i < t.phase.size(); ++i) {
        const qgm::TFactor& f = t.phase[i];
        phq[2 * i] = f.type == qgm::TF_MAT4 ? -2 : (f.src0 == qgm::TS_SIG ? f.bit0 : -1);
        phq[2 * i + 1] = f.src1 == qgm::TS_SIG ? f.bit1 : -1;
    }
    fill_tree_adjoint_tables(P, h);
    // the tail: its levels, copies of its tasks with the results made in the tail at their LDS rows, and
    // the rank-0 results it multiplies (arena row, or -1 - LDS row)
    auto* tl = reinterpret_cast<qgm::TreeTailLevel*>(h + P->off_ttail);
    auto* tt = reinterpret_cast<qgm::TreeTask*>(h + P->off_tttasks);
    const int64_t tail0 = t.tail_start < int(t.levels.size()) ? t.level_task_off[size_t(t.tail_start)] : t.n_tasks;
    // what the tail kernel stages in LDS must fit its arrays
    if (t.n_tasks - tail0 > qgm::kTreeTailMaxTasks || int(t.levels.size()) - t.tail_start > qgm::kTreeTailMaxLevels ||
        t.tail_lds_rows > qgm::kTreeTailLdsRows || t.tail_g_entries > qgm::kTreeTailGEntries ||
        (t.tail_g0 & 1) != 0 || (t.phase_g & 1) != 0 ||
        (t.tail_start < int(t.levels.size()) && int(t.finals.size()) > qgm::kTreeTailMaxFinal))
        return false;
    for (size_t L = size_t(t.tail_start); L < t.levels.size(); ++L) {
        qgm::TreeTailLevel x{};
        x.task_off = int32_t(t.level_task_off[L] - tail0);
        x.n_tasks = int32_t(t.level_task_off[L + 1] - t.level_task_off[L]);
        x.nin = qgm::launch_inputs(t.level_max_in[L]);
        tl[L - size_t(t.tail_start)] = x;
        for (int sid : t.levels[L]) {
            const qgm::TreeStep& st = t.steps[size_t(sid)];
            const int32_t lo = t.tail_lds_row[size_t(st.out_tensor)];
            if (lo < 0) return false;   // every result made in the tail has LDS rows
            if (st.g_off < t.tail_g0 || st.g_off + st.g_entries() > t.tail_g0 + t.tail_g_entries) return false;
            for (int64_t c = 0; c < st.n_tasks(); ++c) {
                qgm::TreeTask tk = tasks[st.task_off + c];
                tk.out_row = int32_t(lo + (tk.out_row - t.tensor_row[size_t(st.out_tensor)]));
                tk.g_ent = int32_t(tk.g_ent - t.tail_g0);
                for (size_t k = 0; k < st.in_tensors.size(); ++k) {
                    const int tid = st.in_tensors[k];
                    if (tk.in_tab[k] >= 0 || t.tail_lds_row[size_t(tid)] < 0) continue;
                    tk.in_row[k] = int32_t(t.tail_lds_row[size_t(tid)] + (tk.in_row[k] - t.tensor_row[size_t(tid)]));
                    tk.in_tab[k] = -2;
                }
                tt[st.task_off + c - tail0] = tk;
            }
        }
    }
    auto* tf = reinterpret_cast<int32_t*>(h + P->off_ttfin);
    for (size_t i = 0; i < t.finals.size(); ++i) {
        const int32_t lo = t.tail_lds_row[size_t(t.finals[i])];
        tf[i] = lo >= 0 ? -1 - lo : int32_t(t.tensor_row[size_t(t.finals[i])]);
    }
    auto* ph = reinterpret_cast<qgm::TFactor*>(h + P->off_tphase);
    for (size_t i = 0; i < t.phase.size(); ++i) ph[i] = t.phase[i];
    auto* fr = reinterpret_cast<int64_t*>(h + P->off_tfinal);
    for (size_t i = 0; i < t.finals.size(); ++i) fr[i] = t.tensor_row[t.finals[i]];
    auto* lf = reinterpret_cast<qgm::TreeLeaf*>(h + P->off_tleaf);
    int n_lf = 0;
    {
        std::vector<int> made_by(t.tensor_axes.size(), -1);
        for (size_t i = 0; i < t.steps.size(); ++i) made_by[size_t(t.steps[i].out_tensor)] = int(i);
        auto index_of = [](const std::vector<int>& v, int x) {
            const auto it = std::find(v.begin(), v.end(), x);
            return it == v.end() ? -1 : int(it - v.begin());
        };
        for (const qgm::TreeStep& st : t.steps) {
            if (!st.table_leaf) continue;
            qgm::TreeLeaf L{};
            L.g_off = st.g_off;
            L.leaf_off = st.leaf_off;
            L.r = int32_t(st.out_axes.size());
            L.k = st.kg;
            L.sb = st.sb();
            L.depth = st.leaf_depth;
            if (st.composed) {
                L.n_in = int32_t(st.in_tensors.size());
                L.gb = st.gb();
                for (int j = 0; j < st.gb(); ++j) L.gpos[j] = index_of(st.out_axes, st.gvars[size_t(j)]);
                for (int k = 0; k < L.n_in; ++k) {
                    const int ti = st.in_tensors[size_t(k)];
                    const qgm::TreeStep& mk = t.steps[size_t(made_by[size_t(ti)])];
                    const std::vector<int>& ax = t.tensor_axes[size_t(ti)];
                    L.in_off[k] = mk.leaf_off;
                    L.in_sb[k] = mk.sb();
                    L.in_na[k] = int32_t(ax.size());
                    for (size_t a = 0; a < ax.size(); ++a) {
                        const int po = index_of(st.out_axes, ax[a]), pv = index_of(st.vars, ax[a]);
                        L.in_src[k][a] = int8_t(po >= 0 ? po : 16 + pv);
                    }
                    for (int b = 0; b < mk.sb(); ++b) L.in_spos[k][b] = int8_t(index_of(st.sig_q, mk.sig_q[size_t(b)]));
                }
            }
            lf[n_lf++] = L;
        }
    }
    const qgm::LdsProgram& lp = t.lds;
    if (lp.ok) {
        std::memcpy(h + P->off_lstage, lp.stages.data(), sizeof(qgm::LdsStage) * lp.stages.size());
        std::memcpy(h + P->off_lentry, lp.entries.data(), sizeof(qgm::LdsEntry) * lp.entries.size());
        std::memcpy(h + P->off_lrec, lp.recs.data(), sizeof(uint16_t) * lp.recs.size());
        std::memcpy(h + P->off_llvl, lp.level_job_off.data(), sizeof(int32_t) * lp.level_job_off.size());
        std::memcpy(h + P->off_lfin, lp.finals.data(), sizeof(int32_t) * lp.finals.size());
        std::memcpy(h + P->off_lzent, lp.zent.data(), sizeof(uint32_t) * lp.zent.size());
        std::memcpy(h + P->off_lgent, lp.gent.data(), sizeof(uint32_t) * lp.gent.size());
    }
    auto* fd = reinterpret_cast<int32_t*>(h + P->off_tfdep);
    for (size_t i = 0; i < t.finals.size(); ++i) {
        const qgm::TreeStep& mk = t.steps[maker[t.finals[i]]];
        fd[2 * i] = int32_t(mk.task_off);
        fd[2 * i + 1] = int32_t(mk.n_tasks());
    }
    return true;
}

void layout_step_tables(qgm_plan_t* P);

// Offsets of the constant tables in each device copy of the plan; the last 256
// bytes hold the plan's failure record (a persistent launch that gave up).
void layout_tables(qgm_plan_t* P) {
    if (P->p.is_tree) layout_tree_tables(P);
    else layout_step_tables(P);
    P->off_status = P->total;
    P->total += 256;
}

void layout_step_tables(qgm_plan_t* P) {
    const qgm::Plan& p = P->p;
    size_t n_sig = 0;
    for (auto& st : p.steps) n_sig += st.sig_src.size();
    P->off_fixed = 0;
    P->off_steps = al(sizeof(double2) * qgm::kFixedMats * 4);
    P->off_ops = P->off_steps + al(sizeof(qgm::StepTab) * p.steps.size());
    P->off_sig = P->off_ops + al(sizeof(qgm::GOp) * size_t(p.n_ops_total));
    P->off_final = P->off_sig + al(sizeof(int32_t) * (n_sig + 1));
    // adjoint tables
    P->wave_base.clear();
    P->step_waves.clear();
    P->total_waves = 0;
    P->max_ops = 1;
    std::vector<std::vector<int32_t>> per_slot(std::max(p.n_slots, 0));
    for (size_t s = 0; s < p.steps.size(); ++s) {
        const qgm::Step& st = p.steps[s];
        const int64_t waves = (st.g_entries() + 63) / 64;
        P->wave_base.push_back(P->total_waves);
        P->step_waves.push_back(int32_t(waves));
        P->total_waves += waves;
        P->max_ops = std::max(P->max_ops, int(st.ops.size()));
        for (size_t i = 0; i < st.ops.size(); ++i) {
            const qgm::GOp& op = st.ops[i];
            if ((op.type == qgm::GOP_MAT || op.type == qgm::GOP_DIAG) && op.mat >= qgm::kFixedMats)
                per_slot[op.mat - qgm::kFixedMats].push_back(int32_t(s << 16) | int32_t(i));
        }
    }
    P->slot_off.assign(1, 0);
    P->slot_ops.clear();
    for (auto& v : per_slot) {
        for (int32_t x : v) P->slot_ops.push_back(x);
        P->slot_off.push_back(int32_t(P->slot_ops.size()));
    }
    P->off_wave_base = P->off_final + al(sizeof(int32_t) * (p.final_pos.size() + 1));
    P->off_step_waves = P->off_wave_base + al(sizeof(int64_t) * (P->wave_base.size() + 1));
    P->off_slot_off = P->off_step_waves + al(sizeof(int32_t) * (P->step_waves.size() + 1));
    P->off_slot_ops = P->off_slot_off + al(sizeof(int32_t) * (P->slot_off.size() + 1));
    P->total = P->off_slot_ops + al(sizeof(int32_t) * (P->slot_ops.size() + 1));
    P->max_g_entries = 0;
    for (auto& st : p.steps) P->max_g_entries = std::max<uint32_t>(P->max_g_entries, uint32_t(st.g_entries()));
}

void fill_step_tables(const qgm_plan_t* P, char* h) {
    const qgm::Plan& p = P->p;
    auto* tabs = reinterpret_cast<qgm::StepTab*>(h + P->off_steps);
    auto* ops = reinterpret_cast<qgm::GOp*>(h + P->off_ops);
    auto* sig = reinterpret_cast<int32_t*>(h + P->off_sig);
    auto* fin = reinterpret_cast<int32_t*>(h + P->off_final);
    int32_t ops_off = 0, sig_off = 0;
    for (size_t s = 0; s < p.steps.size(); ++s) {
        const qgm::Step& st = p.steps[s];
        qgm::StepTab t{};
        t.vb = st.vb; t.kb = st.kb; t.nb = st.nb; t.sb = st.sb;
        t.ops_off = ops_off; t.n_ops = int32_t(st.ops.size());
        t.sig_off = sig_off; t.g_off = st.g_off;
        tabs[s] = t;
        for (auto& op : st.ops) ops[ops_off++] = op;
        for (int x : st.sig_src) sig[sig_off++] = x;
    }
    for (size_t i = 0; i < p.final_pos.size(); ++i) fin[i] = p.final_pos[i];
    std::memcpy(h + P->off_wave_base, P->wave_base.data(), sizeof(int64_t) * P->wave_base.size());
    std::memcpy(h + P->off_step_waves, P->step_waves.data(), sizeof(int32_t) * P->step_waves.size());
    std::memcpy(h + P->off_slot_off, P->slot_off.data(), sizeof(int32_t) * P->slot_off.size());
    std::memcpy(h + P->off_slot_ops, P->slot_ops.data(), sizeof(int32_t) * P->slot_ops.size());
}

// The largest staged block (entries x sigma values) of an LDS program.
int64_t lds_stage_max(const qgm::LdsProgram& lp) {
    int64_t m = 0;
    for (const qgm::LdsStage& sg : lp.stages) m = std::max<int64_t>(m, int64_t(sg.n) << sg.n_sig);
    return m;
}

// Returns the device copy of the plan's constant tables for the current
// device, uploading it on first use.
qgm_status device_tables(qgm_plan_t* P, char** base) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (auto& d : P->p.dev)
        if (d.device == dev) { *base = static_cast<char*>(d.base); return QGM_OK; }
    // zero-filled host image (calloc: the pages of the areas built on the device are never touched here)
    std::unique_ptr<char, void (*)(void*)> img(static_cast<char*>(std::calloc(P->total, 1)), std::free);
    if (!img) return fail(QGM_E_OOM, "host memory for the plan's tables");
    char* h = img.get();
    fixed_matrices(reinterpret_cast<double2*>(h + P->off_fixed));
    if (P->p.is_tree) {
        if (!fill_tree_tables(P, h)) return fail(QGM_E_INTERNAL, "bucket task records overlap, leave gaps or exceed the tail kernel's LDS arrays");
    } else {
        fill_step_tables(P, h);
    }
    void* d = nullptr;
    e = hipMalloc(&d, P->total);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan tables)");
    // a bucket plan without gate values builds its factor tables and the LDS launch's staged copy on the
    // device below: those areas are zeroed there, the records around them copied
    const bool built = P->p.is_tree && P->p.n_slots == 0;
    const size_t zero[2][2] = {{P->off_tg, P->off_ttasks_all}, {P->off_lz, P->off_status}};
    size_t from = 0;
    for (int r = 0; r <= (built ? 2 : 0) && e == hipSuccess; ++r) {
        const size_t to = built && r < 2 ? zero[r][0] : P->total;
        if (to > from) e = hipMemcpy(static_cast<char*>(d) + from, h + from, to - from, hipMemcpyHostToDevice);
        if (built && r < 2 && e == hipSuccess && zero[r][1] > zero[r][0])
            e = hipMemset(static_cast<char*>(d) + zero[r][0], 0, zero[r][1] - zero[r][0]);
        if (built && r < 2) from = zero[r][1];
    }
    if (e != hipSuccess) { (void)hipFree(d); return hip_fail(e, "uploading the plan tables"); }
    if (built) {
        // the factor tables of a circuit without gate values depend only on the plan: build them once
        char* b = static_cast<char*>(d);
        qgm::launch_tree_prologue(reinterpret_cast<const qgm::TreeProBlock*>(b + P->off_tpro),
                                  P->n_pro_blocks + P->n_pro_phase,
                                  reinterpret_cast<const qgm::TreeGTab*>(b + P->off_tgtab),
                                  reinterpret_cast<const qgm::TreeGroup*>(b + P->off_tgroup),
                                  reinterpret_cast<const qgm::TFactor*>(b + P->off_tfac),
                                  reinterpret_cast<const double2*>(b + P->off_fixed), nullptr,
                                  reinterpret_cast<float2*>(b + P->off_tg), P->p.tree.ones_g,
                                  reinterpret_cast<const qgm::TFactor*>(b + P->off_tphase),
                                  int(P->p.tree.phase.size()), P->p.tree.phase_g, nullptr);
        int64_t max_entries = 0;
        int max_depth = 0;
        for (const qgm::TreeStep& st : P->p.tree.steps)
            if (st.table_leaf) {
                max_entries = std::max<int64_t>(max_entries, int64_t(1) << (st.out_axes.size() + st.sb()));
                max_depth = std::max(max_depth, st.leaf_depth);
            }
        qgm::launch_tree_leaf_tables(reinterpret_cast<const qgm::TreeLeaf*>(b + P->off_tleaf),
                                     P->p.tree.n_table_leaves, max_entries, max_depth,
                                     reinterpret_cast<float2*>(b + P->off_tg), nullptr);
        const qgm::LdsProgram& lp = P->p.tree.lds;
        if (lp.ok)
            qgm::launch_lds_stage(reinterpret_cast<const qgm::LdsStage*>(b + P->off_lstage), int(lp.stages.size()),
                                  reinterpret_cast<const qgm::LdsEntry*>(b + P->off_lentry),
                                  reinterpret_cast<const float2*>(b + P->off_tg), reinterpret_cast<float2*>(b + P->off_lz),
                                  lds_stage_max(lp), nullptr);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) { (void)hipFree(d); return hip_fail(e, "building the plan's factor tables"); }
    }
    P->p.dev.push_back({dev, d});
    *base = static_cast<char*>(d);
    return QGM_OK;
}

qgm::StepParams step_params(const qgm::Step& stp) {
    qgm::StepParams sp{};
    sp.kb = stp.kb; sp.vb = stp.vb; sp.nb = stp.nb; sp.sb = stp.sb;
    sp.row_bits = stp.r_in - stp.kb;
    sp.input_is_one = stp.input_is_one ? 1 : 0;
    for (int j = 0; j < stp.kb; ++j) sp.kpos[j] = stp.kpos[j];
    for (int j = 0; j < stp.vb; ++j) sp.vpos[j] = stp.vpos[j];
    sp.g_off = stp.g_off;
    sp.pair_bit = stp.pair_bit;
    sp.pair_in = stp.pair_in;
    return sp;
}

// Enqueues forward step i reading fin and writing fout.
void forward_step(const qgm::Step& stp, const float2* fin, float2* fout, const uint16_t* vs, const float2* gtab,
                  uint32_t B_eff, hipStream_t s) {
    const qgm::StepParams sp = step_params(stp);
    if (stp.kclass == 1 || stp.kclass == 2) {
        qgm::DenseParams dp{};
        dp.sp = sp;
        dp.bf16x3 = stp.kclass == 2 ? 1 : 0;
        for (int j = 0; j < 4; ++j) dp.inner_pos[j] = stp.inner_pos[j];
        dp.n_outer = int32_t(stp.outer_pos.size());
        for (int j = 0; j < dp.n_outer; ++j) dp.outer_pos[j] = stp.outer_pos[j];
        qgm::launch_dense(dp, fin, fout, vs, gtab, B_eff, s);
    } else {
        qgm::launch_step(sp, fin, fout, vs, gtab, B_eff, s);
    }
}

// Gbar work split for one step at batch B_eff: 8-wide k and n slices, and
// row chunks so that the partial-product kernel has about 2^16 threads.
qgm::GbarParams gbar_params(const qgm::Step& stp, uint32_t B_eff) {
    qgm::GbarParams gp{};
    gp.sp = step_params(stp);
    const int K = 1 << stp.kb, N = 1 << stp.nb;
    gp.kw = std::min(K, 8);
    gp.nw = std::min(N, 8);
    gp.n_kc = K / gp.kw;
    gp.n_nc = N / gp.nw;
    std::vector<int> vp(stp.vpos.begin(), stp.vpos.end());
    const int row_bits = stp.r_in - stp.kb;
    gp.n_free = 0;
    for (int pos = 0; pos < row_bits; ++pos)
        if (std::find(vp.begin(), vp.end(), pos) == vp.end()) gp.free_pos[gp.n_free++] = pos;
    const int64_t base_units = int64_t(gp.n_kc) * gp.n_nc << stp.vb;
    int64_t n_rc = 1;
    while (n_rc * 2 <= (int64_t(1) << gp.n_free) && base_units * n_rc * 2 * B_eff <= (int64_t(1) << 16) &&
           base_units * n_rc * 2 <= 65535)
        n_rc *= 2;
    gp.n_rc = int32_t(n_rc);
    gp.rc_rows = int32_t((int64_t(1) << gp.n_free) / n_rc);
    return gp;
}

// Workspace of qgm_backward for a tree plan: the keep-all arena, the adjoint
// arena, the factor tables (circuits with gate values), the expansion
// scratch, the row sums of H per table row, the table adjoints (FP64) and the
// factor adjoints (FP64).
struct TreeBwdLayout {
    uint64_t arena = 0, adj = 0, g = 0, scratch = 0, hsum = 0, part = 0, gbar = 0, fbar = 0, phibar = 0, fpart = 0,
             total = 0;
};

TreeBwdLayout tree_backward_layout(const qgm_plan_t* P, int64_t B) {
    const qgm::TreePlan& t = P->p.tree;
    const uint64_t be = uint64_t(qgm::tree_pitch(B));
    TreeBwdLayout L;
    L.arena = 0;
    L.adj = al(uint64_t(t.arena_rows_all) * be * 8);
    L.g = 2 * L.adj;
    L.scratch = L.g + (P->p.n_slots > 0 ? al(uint64_t(t.g_total) * 8) : 0);
    L.hsum = L.scratch + al(uint64_t(t.scratch_rows) * be * 8);
    L.part = L.hsum + al(uint64_t(t.hsum_rows) * be * 8);
    L.gbar = L.part + al(uint64_t(P->part_rows[0] + P->part_rows[1]) * be * 8);
    L.fbar = L.gbar + al(uint64_t(t.g_total) * 16);
    L.phibar = L.fbar + al(uint64_t(P->n_fbar) * 4 * 16 + 16);
    L.fpart = L.phibar + al(be * 16);
    L.total = L.fpart + al(uint64_t(P->part_off.empty() ? 0 : P->part_off.back()) * 4 * 16 + 16);
    return L;
}

struct BwdLayout {
    uint64_t frame = 0;
    int c = 1, n_ck = 0;
    uint64_t frames = 0, vids = 0, g = 0, gbar = 0, part = 0, wpart = 0, total = 0;
};

BwdLayout backward_layout(const qgm_plan_t* P, int64_t B) {
    const qgm::Plan& p = P->p;
    BwdLayout L;
    const int S = int(p.steps.size());
    const uint64_t be = uint64_t(qgm::batch_eff(p, B));
    L.frame = al((uint64_t(1) << p.r_max) * be * 8);
    L.c = p.opts.checkpoint_every > 0 ? p.opts.checkpoint_every
                                      : (p.ckpt_every > 0 ? p.ckpt_every : std::max(1, int(std::ceil(std::sqrt(double(S))))));
    L.n_ck = (S - 1) / L.c;
    const uint64_t n_frames = 4 + uint64_t(L.n_ck) + uint64_t(L.c - 1);
    L.frames = 0;
    L.vids = n_frames * L.frame;
    L.g = L.vids + al(uint64_t(S) * be * 2);
    L.gbar = L.g + al(uint64_t(p.g_total) * 8);
    L.part = L.gbar + al(uint64_t(p.g_total) * 16);
    uint64_t part_bytes = 0;
    for (auto& st : p.steps) {
        const qgm::GbarParams gp = gbar_params(st, uint32_t(be));
        const uint64_t units = uint64_t(gp.n_nc) * gp.n_kc * gp.n_rc << st.vb;
        part_bytes = std::max(part_bytes, units * 64 * be * 8);
    }
    L.wpart = L.part + al(part_bytes);
    L.total = L.wpart + al(uint64_t(P->total_waves) * uint64_t(P->max_ops) * 4 * 16);
    return L;
}

}  // namespace

extern "C" {

void qgm_default_opts(qgm_plan_opts* opts) {
    if (opts) std::memset(opts, 0, sizeof *opts);
}

qgm_status qgm_plan(const qgm_circuit* circuit, const int32_t* open_qubits, int32_t n_open,
                    const qgm_plan_opts* opts_in, qgm_plan_t** out) {
    g_err.clear();
    if (!out) return fail(QGM_E_INVALID, "out is NULL");
    *out = nullptr;
    qgm_plan_opts opts;
    qgm_default_opts(&opts);
    if (opts_in) opts = *opts_in;
    auto* P = new (std::nothrow) qgm_plan_t;
    if (!P) return fail(QGM_E_OOM, "out of host memory");
    std::string err;
    qgm_status st;
    try {
        st = qgm::build_plan(circuit, open_qubits, n_open, opts, P->p, &err);
    } catch (const std::bad_alloc&) {
        st = QGM_E_OOM;
        err = "out of host memory while planning";
    } catch (...) {
        st = QGM_E_INTERNAL;
        err = "unexpected exception while planning";
    }
    if (st != QGM_OK) {
        delete P;
        return fail(st, err);
    }
    layout_tables(P);
    *out = P;
    return QGM_OK;
}

qgm_status qgm_plan_info(const qgm_plan_t* plan, int32_t detail, char* json, size_t cap, size_t* needed) {
    g_err.clear();
    if (!plan) return fail(QGM_E_INVALID, "plan is NULL");
    std::string s;
    try {
        s = qgm::plan_json(plan->p, detail);
    } catch (...) {
        return fail(QGM_E_OOM, "out of host memory");
    }
    if (needed) *needed = s.size() + 1;
    if (!json || cap < s.size() + 1) return fail(QGM_E_INVALID, "buffer too small");
    std::memcpy(json, s.c_str(), s.size() + 1);
    return QGM_OK;
}

qgm_status qgm_workspace_bytes(const qgm_plan_t* plan, int64_t B, uint64_t* bytes) {
    g_err.clear();
    if (!plan || !bytes) return fail(QGM_E_INVALID, "plan or bytes is NULL");
    if (B < 0) return fail(QGM_E_INVALID, "B < 0");
    *bytes = qgm::workspace_layout(plan->p, B).total;
    return QGM_OK;
}

}  // extern "C"

// The amplitude call; with out == nullptr and allow_no_out the output stage is
// skipped (the autotuner only needs the frontier buffers filled).
static qgm_status amplitudes_impl(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B, void* out,
                                  void* workspace, uint64_t ws_bytes, void* stream, bool allow_no_out) {
    g_err.clear();
    if (!plan) return fail(QGM_E_INVALID, "plan is NULL");
    if (B < 0) return fail(QGM_E_INVALID, "B < 0");
    if (B == 0) return QGM_OK;
    const qgm::Plan& p = plan->p;
    if (!bits || (!out && !allow_no_out))
        return fail(QGM_E_INVALID, "bits and out must be device pointers");
    if (p.n_slots > 0 && !gate_vals) return fail(QGM_E_INVALID, "the circuit reads gate_vals but it is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(QGM_E_INVALID, "workspace must be 256-byte aligned");
    const int64_t B_pad = qgm::padded_batch(B);
    const int64_t B_eff = qgm::batch_eff(p, B);
    if (B_eff > (int64_t(1) << 26)) return fail(QGM_E_UNSUPPORTED, "batch times slice count exceeds 2^26");
    if (p.is_tree && (B_eff & (B_eff - 1)) != 0)   // the bucket kernels scale arena rows by a shift
        return fail(QGM_E_INTERNAL, "bucket arena pitch is not a power of two");
    if ((int64_t(1) << p.r_max) * (B_eff / 64) >= (int64_t(1) << 31))
        return fail(QGM_E_UNSUPPORTED, "frontier rows times batch blocks exceed 2^31");
    const qgm::WsLayout w = qgm::workspace_layout(p, B);
    if (w.total > 0 && !workspace)
        return fail(QGM_E_INVALID, "workspace is NULL but the call needs " + std::to_string(w.total) + " bytes");
    if (ws_bytes < w.total)
        return fail(QGM_E_OOM, "workspace too small: need " + std::to_string(w.total) + " bytes");
    char* tables = nullptr;
    qgm_status st = device_tables(plan, &tables);
    if (st != QGM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    float2* F[2] = {reinterpret_cast<float2*>(ws + w.f0), reinterpret_cast<float2*>(ws + w.f1)};
    auto* vids = reinterpret_cast<uint16_t*>(ws + w.var_ids);
    auto* gtab = reinterpret_cast<float2*>(ws + w.g);
    const auto* tabs = reinterpret_cast<const qgm::StepTab*>(tables + plan->off_steps);
    const int n_steps = int(p.steps.size());
    hipEvent_t ev[5] = {};
    if (plan->timing) {
        while (plan->events.size() < plan->events_used + 5) {
            hipEvent_t e = nullptr;
            hipError_t he = hipEventCreate(&e);
            if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
            plan->events.push_back(e);
        }
        for (int i = 0; i < 5; ++i) ev[i] = plan->events[plan->events_used + i];
        plan->events_used += 5;
    }
    auto mark = [&](int i) { if (plan->timing) (void)hipEventRecord(ev[i], s); };
    mark(0);
    if (p.is_tree) {
        // bucket elimination: factor tables (only for a circuit with gate values), one launch per tree level,
        // the tail
        // levels and the FP64 product in one launch
        const qgm::TreePlan& t = p.tree;
        float2* arena = reinterpret_cast<float2*>(ws + w.f0);
        float2* gt = p.n_slots > 0 ? reinterpret_cast<float2*>(ws + w.g) : reinterpret_cast<float2*>(tables + plan->off_tg);
        const auto* fixed = reinterpret_cast<const double2*>(tables + plan->off_fixed);
        const auto* slots = static_cast<const float2*>(gate_vals);
        const auto* tasks = reinterpret_cast<const qgm::TreeTask*>(tables + plan->off_ttasks);
        const auto* facs = reinterpret_cast<const qgm::TFactor*>(tables + plan->off_tfac);
        const auto* phase = reinterpret_cast<const qgm::TFactor*>(tables + plan->off_tphase);
        const auto* finals = reinterpret_cast<const int64_t*>(tables + plan->off_tfinal);
        mark(1);
        if (p.n_slots > 0)   // factor tables from this call's gate values
            qgm::launch_tree_prologue(reinterpret_cast<const qgm::TreeProBlock*>(tables + plan->off_tpro),
                                      plan->n_pro_blocks + plan->n_pro_phase,
                                      reinterpret_cast<const qgm::TreeGTab*>(tables + plan->off_tgtab),
                                      reinterpret_cast<const qgm::TreeGroup*>(tables + plan->off_tgroup), facs, fixed,
                                      slots, gt, t.ones_g, phase, int(t.phase.size()), t.phase_g, s);
        mark(2);
        // one pass of the launches over nb batch columns whose words are cb, writing the amplitudes to o
        // (marks the phase events when `marks`)
        auto run = [&](const uint64_t* cb, int64_t nb, void* o, bool c128, bool marks) -> qgm_status {
            const int64_t be = qgm::tree_pitch(nb);
            auto mk = [&](int i) { if (marks) mark(i); };
            if (qgm::tree_lds(p, B)) {
                // one work-group per batch column, every level in LDS, then the FP64 product
                const qgm::LdsProgram& lp = t.lds;
                qgm::LdsArgs a{};
                a.stages = reinterpret_cast<const qgm::LdsStage*>(tables + plan->off_lstage);
                // a circuit without gate values reads the plan's staged copy (a slice is one contiguous
                // read); one with gate values gathers from this call's tables (no staging launch per call)
                a.staged = p.n_slots == 0 ? 1 : 0;
                a.zent = reinterpret_cast<const uint32_t*>(tables + (a.staged ? plan->off_lzent : plan->off_lgent));
                a.ztab = a.staged ? reinterpret_cast<const float2*>(tables + plan->off_lz) : gt;
                a.recs = reinterpret_cast<const uint16_t*>(tables + plan->off_lrec);
                a.phq = reinterpret_cast<const int32_t*>(tables + plan->off_tphq);
                a.pv = reinterpret_cast<const double2*>(gt + t.phase_g);
                a.threads = lp.threads;
                a.n_jobs = int32_t(lp.jobs.size());
                a.recs0 = lp.recs0;
                a.level_job_off = reinterpret_cast<const int32_t*>(tables + plan->off_llvl);
                a.finals = reinterpret_cast<const int32_t*>(tables + plan->off_lfin);
                a.phase = phase;
                a.fixed = fixed;
                a.slots = slots;
                a.gtab = gt;
                a.bits = cb;
                a.out = o;
                a.B = nb;
                a.n_stages = int32_t(lp.stages.size());
                a.n_entries = int32_t(lp.entries.size());
                a.tables0 = lp.tables0;
                a.lds_size = lp.lds_size;
                a.n_levels = int32_t(lp.level_job_off.size()) - 1;
                a.n_final = int32_t(lp.finals.size());
                a.n_phase = int32_t(t.phase.size());
                a.c128 = c128 ? 1 : 0;
                qgm::launch_tree_lds(a, s);
                mk(3);
                return QGM_OK;
            }
            if (qgm::tree_persistent(p, B)) {
                // all levels and the amplitude product in one launch, every result at its own rows
                auto* flags = reinterpret_cast<int32_t*>(ws + w.flags);
                const int64_t stride = qgm::tree_flag_stride(p);
                qgm::launch_persist_init(flags, qgm::tree_flag_words(p, nb), o, nb, c128, s);
                qgm::TreePersist a{};
                const int64_t task0 = t.levels.empty() ? 0 : t.level_task_off[t.first_level];
                a.tasks = reinterpret_cast<const qgm::TreeTask*>(tables + plan->off_ttasks_all) + task0;
                a.task0 = int32_t(task0);
                a.n_tasks = int32_t(t.n_tasks - task0);
                a.final_dep = reinterpret_cast<const int32_t*>(tables + plan->off_tfdep);
                a.n_final_dep = int32_t(t.finals.size());
                a.n_final = int32_t(t.finals.size());
                a.final_rows = reinterpret_cast<const int64_t*>(tables + plan->off_tfinal_all);
                a.phase = phase;
                a.n_phase = int32_t(t.phase.size());
                a.c128 = c128 ? 1 : 0;
                a.fixed = fixed;
                a.slots = slots;
                a.arena = arena;
                a.gtab = gt;
                a.ones_g = t.ones_g;
                a.bits = cb;
                a.B = nb;
                a.B_eff = uint32_t(be);
                a.flag_stride = int32_t(stride);
                int max_class = 1;
                for (int L = t.first_level; L < int(t.levels.size()); ++L)
                    max_class = std::max(max_class, qgm::launch_inputs(t.level_max_in[L]));
                a.max_class = max_class;
                a.flags = flags;
                a.out = o;
                a.status = reinterpret_cast<int32_t*>(tables + plan->off_status);
                a.spin_limit = p.opts.persist_spin > 0 ? p.opts.persist_spin : (1 << 20);
                hipError_t he = qgm::launch_tree_persist(a, s);
                if (he != hipSuccess) return hip_fail(he, "persistent launch");
                mk(3);
                return QGM_OK;
            }
            for (int L = t.first_level; L < t.tail_start; ++L) {
                const int64_t t0 = t.level_task_off[L], t1 = t.level_task_off[L + 1];
                qgm::launch_tree_level(t.level_max_in[L], tasks + t0, int32_t(t1 - t0), arena, arena, gt, t.ones_g,
                                       cb, nb, uint32_t(be), uint32_t((nb + 63) / 64), s,
                                       int32_t(t.level_quad[size_t(L)]), t.level_quad_arena[size_t(L)] != 0);
            }
            const int n_tail = int(t.levels.size()) - t.tail_start;
            if (n_tail > 0) {
                if (o) {
                    qgm::TreeTailArgs ta{};
                    ta.levels = reinterpret_cast<const qgm::TreeTailLevel*>(tables + plan->off_ttail);
                    ta.tasks = reinterpret_cast<const qgm::TreeTask*>(tables + plan->off_tttasks);
                    ta.final_lds = reinterpret_cast<const int32_t*>(tables + plan->off_ttfin);
                    ta.phase = phase;
                    ta.phase_q = reinterpret_cast<const int32_t*>(tables + plan->off_tphq);
                    ta.fixed = fixed;
                    ta.slots = slots;
                    ta.arena = arena;
                    ta.gtab = gt;
                    ta.bits = cb;
                    ta.out = o;
                    ta.ones_g = t.ones_g;
                    ta.tail_g0 = t.tail_g0;
                    ta.phase_g = t.phase_g;
                    ta.B = nb;
                    ta.n_levels = n_tail;
                    ta.n_tasks = int32_t(t.n_tasks - t.level_task_off[size_t(t.tail_start)]);
                    ta.n_final = int32_t(t.finals.size());
                    ta.n_phase = int32_t(t.phase.size());
                    ta.tail_g_entries = int32_t(t.tail_g_entries);
                    ta.c128 = c128 ? 1 : 0;
                    ta.B_eff = uint32_t(be);
                    qgm::launch_tree_tail(ta, s);
                }
                mk(3);
            } else {
                mk(3);
                if (o && t.n_open > 0)   // a set of 2^n_open amplitudes per bitstring
                    qgm::launch_tree_final_open(finals, int(t.finals.size()), phase, int(t.phase.size()), fixed,
                                                slots, arena, t.open_tensor >= 0 ? t.tensor_row[t.open_tensor] : -1,
                                                t.n_open, uint32_t(t.zero_mask), cb, nb, uint32_t(be), o, c128, s);
                else if (o)
                    qgm::launch_tree_final(finals, int(t.finals.size()), phase, int(t.phase.size()), fixed, slots,
                                           arena, cb, nb, uint32_t(be), o, c128, s);
            }
            return QGM_OK;
        };
        if (t.sliced.empty()) {
            if (!out && (qgm::tree_lds(p, B) || qgm::tree_persistent(p, B))) return QGM_OK;   // nothing to fill
            qgm_status rs = run(bits, B, out, p.opts.out_c128 != 0, true);
            if (rs != QGM_OK) return rs;
        } else {
            // slices in chunks of 2^chunk_bits as batch columns; FP64 sums in slice order
            const int S = int(t.sliced.size()), cb = t.chunk_bits;
            auto* cols = reinterpret_cast<uint64_t*>(ws + w.ext);
            auto* part = reinterpret_cast<double2*>(ws + w.part);
            auto* acc = reinterpret_cast<double2*>(ws + w.acc);
            const int64_t n_chunks = int64_t(1) << (S - cb);
            for (int64_t c = 0; c < n_chunks; ++c) {
                qgm::launch_slice_cols(bits, B, p.n, cb, uint64_t(c) << cb, cols, s);
                qgm_status rs = run(cols, B << cb, part, true, false);
                if (rs != QGM_OK) return rs;
                if (out || c + 1 < n_chunks)
                    qgm::launch_slice_sum(part, B, cb, t.n_open, acc, c == 0, c + 1 == n_chunks, out,
                                          p.opts.out_c128 != 0, s);
            }
            mark(3);
        }
        mark(4);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return QGM_OK;
    }
    qgm::launch_boundary(bits, B, uint32_t(B_pad), uint32_t(B_eff), n_steps, tabs,
                         reinterpret_cast<const int32_t*>(tables + plan->off_sig), vids, s);
    mark(1);
    qgm::launch_build_g(tabs, n_steps, plan->max_g_entries, reinterpret_cast<const qgm::GOp*>(tables + plan->off_ops),
                        reinterpret_cast<const double2*>(tables + plan->off_fixed),
                        static_cast<const float2*>(gate_vals), gtab, s);
    mark(2);
    for (int i = 0; i < n_steps; ++i)
        forward_step(p.steps[i], F[i & 1], F[(i + 1) & 1], vids + size_t(i) * size_t(B_eff), gtab, uint32_t(B_eff), s);
    mark(3);
    if (out)
        qgm::launch_finalize(F[n_steps & 1], uint32_t(B_eff), uint32_t(B_pad), B, int(1 << p.sliced.size()), p.n_open,
                             reinterpret_cast<const int32_t*>(tables + plan->off_final), out, p.opts.out_c128 != 0, s);
    mark(4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QGM_OK;
}

// qgm_backward for a tree plan: forward with every result kept, seed, then
// the buckets' adjoints level by level in reverse, then the gate gradients.
static qgm_status tree_backward(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B,
                                const void* grad_amps, void* amps_out, void* gate_grads, void* workspace,
                                uint64_t ws_bytes, void* stream) {
    const qgm::Plan& p = plan->p;
    const qgm::TreePlan& t = p.tree;
    if (t.n_open > 0) return fail(QGM_E_UNSUPPORTED, "qgm_backward with ordering 1 supports no open qubits");
    if (!t.sliced.empty()) return fail(QGM_E_UNSUPPORTED, "qgm_backward with ordering 1 supports no slicing");
    if (p.n_2q > 0) return fail(QGM_E_UNSUPPORTED, "qgm_backward supports no non-diagonal two-qubit gates");
    if (t.n_table_leaves > 0)   // only plans without gate values have them: nothing to differentiate
        return fail(QGM_E_UNSUPPORTED, "qgm_backward needs a circuit with gate values (value-slot gates)");
    if (B == 0) return QGM_OK;
    if (!bits || !grad_amps || !workspace || (p.n_slots > 0 && (!gate_vals || !gate_grads)))
        return fail(QGM_E_INVALID, "bits, grad_amps, workspace (and gate_vals, gate_grads when the circuit has slots) "
                                   "must be device pointers");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(QGM_E_INVALID, "workspace must be 256-byte aligned");
    const int64_t B_eff = qgm::tree_pitch(B);   // the arena's row pitch (a power of two)
    if (B_eff > (int64_t(1) << 26)) return fail(QGM_E_UNSUPPORTED, "batch exceeds 2^26");
    const TreeBwdLayout L = tree_backward_layout(plan, B);
    if (ws_bytes < L.total) return fail(QGM_E_OOM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    char* tables = nullptr;
    qgm_status st = device_tables(plan, &tables);
    if (st != QGM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    auto* arena = reinterpret_cast<float2*>(ws + L.arena);
    auto* adj = reinterpret_cast<float2*>(ws + L.adj);
    auto* scratch = reinterpret_cast<float2*>(ws + L.scratch);
    auto* hsum = reinterpret_cast<float2*>(ws + L.hsum);
    float2* part[2] = {reinterpret_cast<float2*>(ws + L.part),
                       reinterpret_cast<float2*>(ws + L.part) + plan->part_rows[0] * B_eff};
    auto* gbar = reinterpret_cast<double2*>(ws + L.gbar);
    auto* fbar = reinterpret_cast<double2*>(ws + L.fbar);
    float2* gt = p.n_slots > 0 ? reinterpret_cast<float2*>(ws + L.g) : reinterpret_cast<float2*>(tables + plan->off_tg);
    const auto* fixed = reinterpret_cast<const double2*>(tables + plan->off_fixed);
    const auto* slots = static_cast<const float2*>(gate_vals);
    const auto* facs = reinterpret_cast<const qgm::TFactor*>(tables + plan->off_tfac);
    const auto* pro = reinterpret_cast<const qgm::TreeProBlock*>(tables + plan->off_tpro);
    const auto* gtabs = reinterpret_cast<const qgm::TreeGTab*>(tables + plan->off_tgtab);
    const auto* groups = reinterpret_cast<const qgm::TreeGroup*>(tables + plan->off_tgroup);
    const auto* tasks_all = reinterpret_cast<const qgm::TreeTask*>(tables + plan->off_ttasks_all);
    const auto* items = reinterpret_cast<const qgm::TreeBwdItem*>(tables + plan->off_titems);
    const uint32_t be = uint32_t(B_eff);
    if (p.n_slots > 0)   // the factor tables only (the adjoint evaluates the phase factors itself)
        qgm::launch_tree_prologue(pro, plan->n_pro_blocks, gtabs, groups, facs, fixed, slots, gt, t.ones_g, nullptr, 0,
                                  0, s);
    for (int Lv = t.first_level; Lv < int(t.levels.size()); ++Lv) {
        const int64_t t0 = t.level_task_off[Lv], t1 = t.level_task_off[Lv + 1];
        qgm::launch_tree_level(t.level_max_in[Lv], tasks_all + t0, int32_t(t1 - t0), arena, arena, gt, t.ones_g, bits,
                               B, be, be / 64u, s);   // every group of the pitch: the adjoint reads them all
    }
    auto* phibar = reinterpret_cast<double2*>(ws + L.phibar);
    auto* fpart = reinterpret_cast<double2*>(ws + L.fpart);
    const auto* part_off = reinterpret_cast<const int64_t*>(tables + plan->off_tpart);
    qgm::launch_tb_seed(reinterpret_cast<const int64_t*>(tables + plan->off_tfinal_all), int(t.finals.size()),
                        reinterpret_cast<const qgm::TFactor*>(tables + plan->off_tphase), int(t.phase.size()), fixed,
                        slots, arena, adj, bits, B, be, static_cast<const float2*>(grad_amps), amps_out,
                        p.opts.out_c128 != 0, phibar, s);
    if (p.n_slots > 0)
        qgm::launch_tb_phase_adj(reinterpret_cast<const qgm::TFactor*>(tables + plan->off_tphase), int(t.phase.size()),
                                 fixed, slots, bits, B, phibar, part_off, plan->n_fbar - int64_t(t.phase.size()),
                                 fpart, s);
    const auto* bwd = reinterpret_cast<const qgm::TreeBwd*>(tables + plan->off_tbwd);
    const auto* bin = reinterpret_cast<const qgm::TreeBwdIn*>(tables + plan->off_tbwdin);
    const auto* bgd = reinterpret_cast<const qgm::TreeBwdG*>(tables + plan->off_tbwdg);
    for (int Lv = int(t.levels.size()) - 1; Lv >= t.first_level; --Lv) {
        const auto& ex = plan->lv_exp[Lv];
        qgm::launch_tb_expand(items + ex.off, ex.n, ex.rows, bwd, arena, adj, gt, scratch, bits, B, be,
                              p.n_slots > 0, s);
        for (size_t k = 0; k < plan->lv_red[Lv].size(); ++k) {
            const auto& rs = plan->lv_red[Lv][k];
            const float2* src = k == 0 ? scratch : part[(k - 1) % 2];
            qgm::launch_tb_reduce(items + rs.off, rs.n, rs.rows, bin, src, adj, hsum, part[k % 2], be, s);
        }
    }
    if (p.n_slots > 0) {
        const auto& gg = plan->g_all;
        qgm::launch_tb_gbin(items + gg.off, gg.n, gg.rows, bgd, hsum, bits, B, be, gbar, s);
        qgm::launch_tb_gadj(pro, plan->n_pro_blocks, gtabs, groups, facs, fixed, slots, gbar, part_off, fpart, s);
        qgm::launch_tb_fsum(part_off, plan->n_fbar, fpart, fbar, s);
        qgm::launch_tb_slots(reinterpret_cast<const int32_t*>(tables + plan->off_tslot_off),
                             reinterpret_cast<const int32_t*>(tables + plan->off_tslot_occ), p.n_slots, fbar,
                             static_cast<float2*>(gate_grads), s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QGM_OK;
}

extern "C" {

qgm_status qgm_amplitudes(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B, void* out,
                          void* workspace, uint64_t ws_bytes, void* stream) {
    return amplitudes_impl(plan, gate_vals, bits, B, out, workspace, ws_bytes, stream, false);
}

}  // extern "C"

// Workspace of qgm_amplitudes_static: one file-scope device array, of which
// every device the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: the device address of
// each copy comes from hipGetSymbolAddress, taken once per device with that
// device current.
constexpr uint64_t kStaticScratchBytes = uint64_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of `scratch`.
qgm_status static_scratch(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(QGM_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return fail(QGM_E_INTERNAL, "scratch array misaligned");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return QGM_OK;
}

}  // namespace

extern "C" {

qgm_status qgm_amplitudes_static(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B, void* out,
                                 void* stream) {
    g_err.clear();
    if (!plan) return fail(QGM_E_INVALID, "plan is NULL");
    if (B < 0) return fail(QGM_E_INVALID, "B < 0");
    if (B == 0) return QGM_OK;
    if (plan->timing) return fail(QGM_E_INVALID, "per-phase timing records events: turn it off for this entry point");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    bool uploaded = false;
    for (auto& d : plan->p.dev) uploaded = uploaded || d.device == dev;
    if (!uploaded)
        return fail(QGM_E_INVALID, "the plan's tables are not on this device yet: run qgm_amplitudes (or "
                                   "qgm_graph_create) with this plan once on the device first");
    const uint64_t need = qgm::workspace_layout(plan->p, B).total;
    if (need > kStaticScratchBytes)
        return fail(QGM_E_OOM, "the batch needs " + std::to_string(need) + " bytes of workspace, beyond the " +
                               std::to_string(kStaticScratchBytes) + " bytes of the static scratch array");
    void* ws = nullptr;
    qgm_status st = static_scratch(&ws);
    if (st != QGM_OK) return st;
    return amplitudes_impl(plan, gate_vals, bits, B, out, ws, kStaticScratchBytes, stream, false);
}

qgm_status qgm_backward_workspace_bytes(const qgm_plan_t* plan, int64_t B, uint64_t* bytes) {
    g_err.clear();
    if (!plan || !bytes) return fail(QGM_E_INVALID, "plan or bytes is NULL");
    if (B < 0) return fail(QGM_E_INVALID, "B < 0");
    *bytes = plan->p.is_tree ? tree_backward_layout(plan, B).total : backward_layout(plan, B).total;
    return QGM_OK;
}

qgm_status qgm_backward(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B,
                        const void* grad_amps, void* amps_out, void* gate_grads, void* workspace, uint64_t ws_bytes,
                        void* stream) {
    g_err.clear();
    if (!plan) return fail(QGM_E_INVALID, "plan is NULL");
    if (B < 0) return fail(QGM_E_INVALID, "B < 0");
    const qgm::Plan& p = plan->p;
    if (p.is_tree) return tree_backward(plan, gate_vals, bits, B, grad_amps, amps_out, gate_grads, workspace, ws_bytes,
                                        stream);
    if (B == 0) return QGM_OK;
    if (!bits || !grad_amps || !workspace || (p.n_slots > 0 && (!gate_vals || !gate_grads)))
        return fail(QGM_E_INVALID, "bits, grad_amps, workspace (and gate_vals, gate_grads when the circuit has slots) "
                                   "must be device pointers");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(QGM_E_INVALID, "workspace must be 256-byte aligned");
    if (p.n_open > 16) return fail(QGM_E_UNSUPPORTED, "qgm_backward supports at most 16 open qubits");
    const int64_t B_pad = qgm::padded_batch(B);
    const int64_t B_eff = qgm::batch_eff(p, B);
    if (B_eff > (int64_t(1) << 26)) return fail(QGM_E_UNSUPPORTED, "batch times slice count exceeds 2^26");
    if ((int64_t(1) << p.r_max) * (B_eff / 64) > (int64_t(1) << 31))
        return fail(QGM_E_UNSUPPORTED, "frontier rows times batch blocks exceed 2^31");
    const BwdLayout L = backward_layout(plan, B);
    if (ws_bytes < L.total) return fail(QGM_E_OOM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    char* tables = nullptr;
    qgm_status st = device_tables(plan, &tables);
    if (st != QGM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(workspace);
    auto frame = [&](uint64_t i) { return reinterpret_cast<float2*>(ws + L.frames + i * L.frame); };
    float2* fwd[2] = {frame(0), frame(1)};
    float2* adj[2] = {frame(2), frame(3)};
    auto ck = [&](int i) { return frame(4 + uint64_t(i)); };              // holds F_{(i+1)c}
    auto seg = [&](int j) { return frame(4 + uint64_t(L.n_ck) + uint64_t(j)); };
    auto* vids = reinterpret_cast<uint16_t*>(ws + L.vids);
    auto* gtab = reinterpret_cast<float2*>(ws + L.g);
    auto* gbar = reinterpret_cast<double2*>(ws + L.gbar);
    auto* part = reinterpret_cast<float2*>(ws + L.part);
    auto* wpart = reinterpret_cast<double2*>(ws + L.wpart);
    const auto* tabs = reinterpret_cast<const qgm::StepTab*>(tables + plan->off_steps);
    const int S = int(p.steps.size());
    const int c = L.c;
    const uint32_t be = uint32_t(B_eff);
    auto vs = [&](int i) { return vids + size_t(i) * size_t(B_eff); };
    qgm::launch_boundary(bits, B, uint32_t(B_pad), be, S, tabs, reinterpret_cast<const int32_t*>(tables + plan->off_sig),
                         vids, s);
    qgm::launch_build_g(tabs, S, plan->max_g_entries, reinterpret_cast<const qgm::GOp*>(tables + plan->off_ops),
                        reinterpret_cast<const double2*>(tables + plan->off_fixed),
                        static_cast<const float2*>(gate_vals), gtab, s);
    // forward, keeping F_s for s = c, 2c, ... (< S)
    auto loc = [&](int i) -> float2* {   // where F_i lives after the forward (i >= 1)
        if (i < S && i % c == 0) return ck(i / c - 1);
        return fwd[i & 1];
    };
    for (int i = 0; i < S; ++i)
        forward_step(p.steps[i], i == 0 ? fwd[0] : loc(i), loc(i + 1), vs(i), gtab, be, s);
    if (amps_out)
        qgm::launch_finalize(loc(S), be, uint32_t(B_pad), B, int(1 << p.sliced.size()), p.n_open,
                             reinterpret_cast<const int32_t*>(tables + plan->off_final), amps_out,
                             p.opts.out_c128 != 0, s);
    // seed: Fbar_S = conj(grad_amps) on every slice copy
    qgm::launch_seed(static_cast<const float2*>(grad_amps), be, uint32_t(B_pad), B, p.n_open,
                     reinterpret_cast<const int32_t*>(tables + plan->off_final), adj[S & 1], s);
    // backward over checkpoint segments [a, e)
    for (int a = ((S - 1) / c) * c; a >= 0; a -= c) {
        const int e = std::min(a + c, S);
        const float2* fa = a == 0 ? fwd[0] : ck(a / c - 1);
        for (int i = a; i + 1 < e; ++i)   // recompute F_{a+1} .. F_{e-1}
            forward_step(p.steps[i], i == a ? fa : seg(i - a - 1), seg(i - a), vs(i), gtab, be, s);
        for (int i = e - 1; i >= a; --i) {
            const float2* fin = i == a ? fa : seg(i - a - 1);
            const qgm::GbarParams gp = gbar_params(p.steps[i], be);
            qgm::launch_gbar(gp, fin, adj[(i + 1) & 1], part, vs(i), be, gbar, s);
            if (i > 0) qgm::launch_step_t(step_params(p.steps[i]), adj[(i + 1) & 1], adj[i & 1], vs(i), gtab, be, s);
        }
    }
    if (p.n_slots > 0) {
        qgm::launch_gadj(tabs, S, plan->max_g_entries, reinterpret_cast<const qgm::GOp*>(tables + plan->off_ops),
                         reinterpret_cast<const double2*>(tables + plan->off_fixed), static_cast<const float2*>(gate_vals),
                         gbar, reinterpret_cast<const int64_t*>(tables + plan->off_wave_base), wpart, plan->max_ops, s);
        qgm::launch_slot_grads(reinterpret_cast<const int32_t*>(tables + plan->off_slot_off),
                               reinterpret_cast<const int32_t*>(tables + plan->off_slot_ops),
                               reinterpret_cast<const int64_t*>(tables + plan->off_wave_base),
                               reinterpret_cast<const int32_t*>(tables + plan->off_step_waves), wpart, plan->max_ops,
                               p.n_slots, static_cast<float2*>(gate_grads), s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QGM_OK;
}

qgm_status qgm_expectation_circuit(const qgm_circuit* circuit, int32_t n_ops, const int32_t* qubits,
                                   const int32_t* paulis, qgm_gate* gates, int32_t cap, int32_t* n_gates) {
    g_err.clear();
    if (!n_gates) return fail(QGM_E_INVALID, "n_gates is NULL");
    std::vector<qgm_gate> out;
    std::string err;
    const qgm_status st = qgm::expectation_circuit(circuit, n_ops, qubits, paulis, out, &err);
    if (st != QGM_OK) return fail(st, err);
    *n_gates = int32_t(out.size());
    if (int64_t(out.size()) > int64_t(cap) || (!gates && !out.empty()))
        return fail(QGM_E_OOM, "gates holds " + std::to_string(cap) + " gates, " + std::to_string(out.size()) +
                                   " needed (written to n_gates)");
    std::copy(out.begin(), out.end(), gates);
    return QGM_OK;
}

qgm_status qgm_xeb_workspace_bytes(int64_t B, uint64_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(QGM_E_INVALID, "bytes is NULL");
    if (B < 1) return fail(QGM_E_INVALID, "B < 1");
    *bytes = qgm::xeb_workspace_bytes(B);
    return QGM_OK;
}

static qgm_status xeb_check(const void* amps, int64_t B, const void* out, void* workspace, uint64_t ws_bytes) {
    if (B < 1) return fail(QGM_E_INVALID, "B < 1");
    if (!amps || !out || !workspace) return fail(QGM_E_INVALID, "amps, output and workspace must be device pointers");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(QGM_E_INVALID, "workspace must be 256-byte aligned");
    if (ws_bytes < qgm::xeb_workspace_bytes(B))
        return fail(QGM_E_OOM, "workspace too small: need " + std::to_string(qgm::xeb_workspace_bytes(B)) + " bytes");
    return QGM_OK;
}

qgm_status qgm_xeb(const void* amps, int32_t c128, int64_t B, int32_t n_qubits, double* out, void* workspace,
                   uint64_t ws_bytes, void* stream) {
    g_err.clear();
    qgm_status st = xeb_check(amps, B, out, workspace, ws_bytes);
    if (st != QGM_OK) return st;
    if (n_qubits < 1 || n_qubits > 64) return fail(QGM_E_INVALID, "n_qubits must be 1..64");
    qgm::launch_xeb(amps, c128 != 0, B, n_qubits, out, static_cast<double*>(workspace), static_cast<hipStream_t>(stream));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QGM_OK;
}

qgm_status qgm_prob_sums(const void* amps, int32_t c128, int64_t B, int32_t n_open, double* out, void* stream) {
    g_err.clear();
    if (B < 0 || n_open < 0 || n_open > 40) return fail(QGM_E_INVALID, "B < 0 or n_open outside 0..40");
    if (B == 0) return QGM_OK;
    if (!amps || !out) return fail(QGM_E_INVALID, "amps and out must be device pointers");
    if (B > 0x7fffffff) return fail(QGM_E_UNSUPPORTED, "B exceeds 2^31 - 1");
    qgm::launch_prob_sums(amps, c128 ? 1 : 0, B, int64_t(1) << n_open, out, static_cast<hipStream_t>(stream));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QGM_OK;
}

qgm_status qgm_sample_set(const void* amps, int32_t c128, int64_t B, const double* u, int64_t m, int64_t* idx,
                          void* workspace, uint64_t ws_bytes, void* stream) {
    g_err.clear();
    if (m < 0) return fail(QGM_E_INVALID, "m < 0");
    if (m > 0 && (!u || !idx)) return fail(QGM_E_INVALID, "u and idx must be device pointers");
    qgm_status st = xeb_check(amps, B, m > 0 ? static_cast<const void*>(idx) : amps, workspace, ws_bytes);
    if (st != QGM_OK) return st;
    qgm::launch_sample_set(amps, c128 != 0, B, u, m, idx, static_cast<double*>(workspace),
                           static_cast<hipStream_t>(stream));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QGM_OK;
}

qgm_status qgm_graph_create(int32_t n_circ, qgm_plan_t* const* plans, const void* const* gate_vals,
                            const uint64_t* const* bits, const int64_t* B, void* const* out,
                            void* const* workspace, const uint64_t* ws_bytes, qgm_graph_t** graph) {
    g_err.clear();
    if (!graph) return fail(QGM_E_INVALID, "graph is NULL");
    *graph = nullptr;
    if (n_circ < 1 || !plans || !bits || !B || !out || !workspace || !ws_bytes)
        return fail(QGM_E_INVALID, "n_circ >= 1 and every array must be given");
    for (int i = 0; i < n_circ; ++i) {
        if (!plans[i]) return fail(QGM_E_INVALID, "plan " + std::to_string(i) + " is NULL");
        if (plans[i]->p.n_slots > 0 && (!gate_vals || !gate_vals[i]))
            return fail(QGM_E_INVALID, "circuit " + std::to_string(i) + " reads gate_vals but it is NULL");
        const qgm::WsLayout w = qgm::workspace_layout(plans[i]->p, B[i]);
        if (ws_bytes[i] < w.total) return fail(QGM_E_OOM, "workspace of circuit " + std::to_string(i) + " too small");
        for (int j = 0; j < i; ++j)
            if (workspace[j] == workspace[i]) return fail(QGM_E_INVALID, "circuits must not share a workspace");
        char* t = nullptr;
        qgm_status st = device_tables(plans[i], &t);   // no allocation may happen during capture
        if (st != QGM_OK) return st;
    }
    std::vector<hipStream_t> streams(n_circ + 1, nullptr);
    std::vector<hipEvent_t> events(n_circ + 1, nullptr);
    qgm_status result = QGM_OK;
    hipGraph_t g = nullptr;
    auto cleanup = [&]() {
        for (auto e : events) if (e) (void)hipEventDestroy(e);
        for (auto s : streams) if (s) (void)hipStreamDestroy(s);
    };
    for (int i = 0; i <= n_circ; ++i) {
        hipError_t e = hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&events[i], hipEventDisableTiming);
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "stream/event creation"); }
    }
    std::vector<bool> timing(n_circ);
    for (int i = 0; i < n_circ; ++i) { timing[i] = plans[i]->timing; plans[i]->timing = false; }
    hipError_t e = hipStreamBeginCapture(streams[0], hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "hipStreamBeginCapture"); }
    (void)hipEventRecord(events[0], streams[0]);
    // a persistent launch needs the whole GPU at once: with one in the graph, every branch waits for the
    // previous one (nothing runs beside it)
    bool any_persist = false;
    for (int i = 0; i < n_circ; ++i) any_persist = any_persist || qgm::tree_persistent(plans[i]->p, B[i]);
    for (int i = 0; i < n_circ && result == QGM_OK; ++i) {
        (void)hipStreamWaitEvent(streams[i + 1], events[0], 0);
        if (any_persist && i > 0) (void)hipStreamWaitEvent(streams[i + 1], events[i], 0);
        result = qgm_amplitudes(plans[i], gate_vals ? gate_vals[i] : nullptr, bits[i], B[i], out[i], workspace[i],
                                ws_bytes[i], streams[i + 1]);
        (void)hipEventRecord(events[i + 1], streams[i + 1]);
        (void)hipStreamWaitEvent(streams[0], events[i + 1], 0);
    }
    e = hipStreamEndCapture(streams[0], &g);
    for (int i = 0; i < n_circ; ++i) plans[i]->timing = timing[i];
    const std::string amp_err = g_err;
    cleanup();
    if (result != QGM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return fail(result, amp_err);
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    auto* G = new (std::nothrow) qgm_graph_t;
    if (!G) { (void)hipGraphDestroy(g); return fail(QGM_E_OOM, "out of host memory"); }
    G->graph = g;
    e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); delete G; return hip_fail(e, "hipGraphInstantiate"); }
    *graph = G;
    return QGM_OK;
}

qgm_status qgm_graph_launch(qgm_graph_t* graph, void* stream) {
    g_err.clear();
    if (!graph || !graph->exec) return fail(QGM_E_INVALID, "graph is NULL");
    hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return QGM_OK;
}

void qgm_graph_destroy(qgm_graph_t* graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

qgm_status qgm_autotune(qgm_plan_t* plan, const void* gate_vals, const uint64_t* bits, int64_t B, void* workspace,
                        uint64_t ws_bytes, void* stream, int32_t allow_bf16x3, const char* cache_path) {
    g_err.clear();
    if (!plan) return fail(QGM_E_INVALID, "plan is NULL");
    if (B <= 0) return fail(QGM_E_INVALID, "B must be > 0");
    // a full call first: validates the arguments, uploads tables, fills the frontier buffers
    qgm_status st = amplitudes_impl(plan, gate_vals, bits, B, nullptr, workspace, ws_bytes, stream, true);
    if (st != QGM_OK) return st;
    qgm::Plan& p = plan->p;
    if (p.is_tree) return QGM_OK;   // one bucket kernel: nothing to choose
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device properties");
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    std::string path = cache_path ? cache_path : "";
    if (path.empty() && std::getenv("QGM_TUNE_CACHE")) path = std::getenv("QGM_TUNE_CACHE");
    std::map<std::string, double> cache;
    if (!path.empty()) {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string a;
            int kb, vb, nb, sb, r, c;
            long long be;
            double ms;
            if (ls >> a >> kb >> vb >> nb >> sb >> r >> be >> c >> ms) {
                std::ostringstream k;
                k << a << ' ' << kb << ' ' << vb << ' ' << nb << ' ' << sb << ' ' << r << ' ' << be << ' ' << c;
                cache[k.str()] = ms;
            }
        }
    }
    const qgm::WsLayout w = qgm::workspace_layout(p, B);
    const int64_t B_eff = qgm::batch_eff(p, B);
    char* ws = static_cast<char*>(workspace);
    float2* F[2] = {reinterpret_cast<float2*>(ws + w.f0), reinterpret_cast<float2*>(ws + w.f1)};
    auto* vids = reinterpret_cast<uint16_t*>(ws + w.var_ids);
    auto* gtab = reinterpret_cast<float2*>(ws + w.g);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    std::vector<std::string> fresh;
    for (size_t i = 0; i < p.steps.size(); ++i) {
        qgm::Step& stp = p.steps[i];
        int best = qgm::KC_VALU;
        double best_ms = 1e300;
        for (int cand = qgm::KC_VALU; cand <= qgm::KC_MFMA_BF16X3; ++cand) {
            if (!qgm::step_supports(stp, cand)) continue;
            if (cand == qgm::KC_MFMA_BF16X3 && !allow_bf16x3) continue;
            // precision BF16X3: the steps the plan gave the BF16x3 kernel keep it
            if (p.opts.precision == QGM_PREC_BF16X3 && stp.kclass == 2 && cand != qgm::KC_MFMA_BF16X3) continue;
            std::ostringstream k;
            k << arch << ' ' << stp.kb << ' ' << stp.vb << ' ' << stp.nb << ' ' << stp.sb << ' ' << stp.r_in << ' '
              << B_eff << ' ' << cand;
            double ms;
            auto it = cache.find(k.str());
            if (it != cache.end()) {
                ms = it->second;
            } else {
                qgm::configure_step(stp, cand);
                const uint16_t* vs = vids + size_t(i) * size_t(B_eff);
                forward_step(stp, F[i & 1], F[(i + 1) & 1], vs, gtab, uint32_t(B_eff), s);
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < 3; ++r) forward_step(stp, F[i & 1], F[(i + 1) & 1], vs, gtab, uint32_t(B_eff), s);
                (void)hipEventRecord(e1, s);
                e = hipEventSynchronize(e1);
                float t = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
                if (e != hipSuccess) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return hip_fail(e, "timing a step");
                }
                ms = double(t) / 3.0;
                cache[k.str()] = ms;
                std::ostringstream line;
                line.precision(6);
                line << k.str() << ' ' << ms;
                fresh.push_back(line.str());
            }
            if (ms < best_ms) { best_ms = ms; best = cand; }
        }
        qgm::configure_step(stp, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!path.empty() && !fresh.empty()) {
        std::ofstream out(path, std::ios::app);
        for (auto& l : fresh) out << l << '\n';
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "autotune launches");
    return QGM_OK;
}

qgm_status qgm_plan_set_timing(qgm_plan_t* plan, int32_t enable) {
    g_err.clear();
    if (!plan) return fail(QGM_E_INVALID, "plan is NULL");
    plan->timing = enable != 0;
    plan->events_used = 0;
    return QGM_OK;
}

qgm_status qgm_plan_timings(qgm_plan_t* plan, double* ms, int64_t* n_calls) {
    g_err.clear();
    if (!plan || !ms || !n_calls) return fail(QGM_E_INVALID, "NULL argument");
    for (int i = 0; i < 4; ++i) ms[i] = 0.0;
    *n_calls = int64_t(plan->events_used / 5);
    for (size_t c = 0; c + 5 <= plan->events_used; c += 5) {
        hipError_t e = hipEventSynchronize(plan->events[c + 4]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        for (int i = 0; i < 4; ++i) {
            float t = 0.f;
            e = hipEventElapsedTime(&t, plan->events[c + i], plan->events[c + i + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            ms[i] += double(t);
        }
    }
    return QGM_OK;
}

void qgm_plan_destroy(qgm_plan_t* plan) {
    if (!plan) return;
    for (hipEvent_t e : plan->events) (void)hipEventDestroy(e);
    int cur = 0;
    bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto& d : plan->p.dev) {
        if (hipSetDevice(d.device) == hipSuccess) (void)hipFree(d.base);
    }
    if (have_cur) (void)hipSetDevice(cur);
    delete plan;
}

const char* qgm_last_error(void) { return g_err.c_str(); }

qgm_status qgm_plan_check(qgm_plan_t* plan, void* stream) {
    g_err.clear();
    if (!plan) return fail(QGM_E_INVALID, "plan is NULL");
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error");
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (auto& d : plan->p.dev) {
        if (d.device != dev) continue;
        char* rec = static_cast<char*>(d.base) + plan->off_status;
        int32_t v = 0;
        e = hipMemcpy(&v, rec, sizeof v, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading the plan's failure record");
        if (v == 0) return QGM_OK;
        const int32_t zero = 0;
        e = hipMemcpy(rec, &zero, sizeof zero, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "clearing the plan's failure record");
        return fail(QGM_E_INTERNAL, v == 2 ? "a persistent launch found its work-groups on unexpected accelerator "
                                             "complexes and gave up (its amplitudes read NaN)"
                                           : "a persistent launch gave up waiting for another wave (the GPU was "
                                             "shared or its grid was not resident at once); its unfinished "
                                             "amplitudes read NaN");
    }
    return QGM_OK;
}

qgm_status qgm_sync_check(void* stream) {
    g_err.clear();
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error");
    return QGM_OK;
}

}  // extern "C"
