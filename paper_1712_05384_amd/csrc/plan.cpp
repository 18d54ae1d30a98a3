// Host-side planner: worldline variables and factors (Sec. III.A-B), the
// vertical elimination order (Sec. IV.A), grouped bucket elimination (App. A)
// with one step per worldline, and variable slicing.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <sstream>

namespace qgm {

namespace {

bool is_diag_kind(int k) { return k == QGM_T || k == QGM_UD || k == QGM_CZ || k == QGM_TDG || k == QGM_Z; }

int mat_index(int kind, int slot) {
    switch (kind) {
        case QGM_H: return 0;
        case QGM_T: return 1;
        case QGM_XH: return 2;
        case QGM_YH: return 3;
        case QGM_TDG: return 4;
        case QGM_XHDG: return 5;
        case QGM_YHDG: return 6;
        case QGM_X: return 7;
        case QGM_Y: return 8;
        case QGM_Z: return 9;
        default: return kFixedMats + slot;   // QGM_U, QGM_UD
    }
}

// The vertical order of Sec. IV.A: whole worldlines one qubit at a time, with
// qubits taken first along the shorter lattice side.
std::vector<int> vertical_order(int rows, int cols) {
    std::vector<int> o;
    if (rows <= cols) {
        for (int c = 0; c < cols; ++c)
            for (int r = 0; r < rows; ++r) o.push_back(r * cols + c);
    } else {
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) o.push_back(r * cols + c);
    }
    return o;
}

struct Src { uint8_t src = SRC_ZERO; uint8_t bit = 0; };

}  // namespace

int64_t padded_batch(int64_t B) { return (B + 63) / 64 * 64; }

int64_t tree_pitch(int64_t B) {
    int64_t p = 64;
    while (p < B) p <<= 1;
    return p;
}

double Step::bytes_per_b() const {
    double in = input_is_one ? 0.0 : 8.0 * double(int64_t(1) << r_in);
    return in + 8.0 * double(int64_t(1) << r_out) + 2.0;
}

double Step::flops_per_b() const {
    // rows * K * N complex multiply-adds, 8 real flops each
    return 8.0 * double(int64_t(1) << (r_in - kb)) * double(int64_t(1) << kb) * double(int64_t(1) << nb);
}

static qgm_status validate(const qgm_circuit* c, const int32_t* open, int32_t n_open, std::string* err) {
    if (!c) { *err = "circuit is NULL"; return QGM_E_INVALID; }
    if (c->rows < 1 || c->cols < 1 || int64_t(c->rows) * c->cols > 64) {
        *err = "rows and cols must be >= 1 with rows*cols <= 64"; return QGM_E_INVALID;
    }
    if (c->n_gates < 0 || (c->n_gates > 0 && !c->gates)) { *err = "bad gate array"; return QGM_E_INVALID; }
    if (c->n_slots < 0) { *err = "n_slots < 0"; return QGM_E_INVALID; }
    const int n = c->rows * c->cols;
    std::set<std::pair<int, int>> used;   // (cycle, qubit)
    for (int i = 0; i < c->n_gates; ++i) {
        const qgm_gate& g = c->gates[i];
        char buf[160];
        if (g.kind < QGM_H || g.kind > QGM_U2) {
            snprintf(buf, sizeof buf, "gate %d: unknown kind %d", i, g.kind); *err = buf; return QGM_E_INVALID;
        }
        if (g.cycle < 0) { snprintf(buf, sizeof buf, "gate %d: negative cycle", i); *err = buf; return QGM_E_INVALID; }
        if (g.q0 < 0 || g.q0 >= n) {
            snprintf(buf, sizeof buf, "gate %d: qubit %d out of range", i, g.q0); *err = buf; return QGM_E_INVALID;
        }
        const bool two_q = g.kind == QGM_CZ || g.kind == QGM_U2;
        if (two_q) {
            if (g.q1 < 0 || g.q1 >= n || g.q1 == g.q0) {
                snprintf(buf, sizeof buf, "gate %d: a two-qubit gate needs two distinct qubits in range", i); *err = buf;
                return QGM_E_INVALID;
            }
        } else if (g.q1 != -1) {
            snprintf(buf, sizeof buf, "gate %d: single-qubit gate must have q1 = -1", i); *err = buf;
            return QGM_E_INVALID;
        }
        if (g.kind == QGM_U || g.kind == QGM_UD || g.kind == QGM_U2) {
            const int need = g.kind == QGM_U2 ? 4 : 1;   // a two-qubit gate reads four slots
            if (g.slot < 0 || g.slot + need > c->n_slots) {
                snprintf(buf, sizeof buf, "gate %d: slots [%d, %d) out of range [0, %d)", i, g.slot, g.slot + need,
                         c->n_slots);
                *err = buf; return QGM_E_INVALID;
            }
        }
        for (int q : {g.q0, two_q ? g.q1 : -1}) {
            if (q < 0) continue;
            if (!used.insert({g.cycle, q}).second) {
                snprintf(buf, sizeof buf, "gate %d: qubit %d used twice in cycle %d", i, q, g.cycle);
                *err = buf; return QGM_E_INVALID;
            }
        }
    }
    if (n_open < 0 || n_open > n || (n_open > 0 && !open)) { *err = "bad open qubit list"; return QGM_E_INVALID; }
    std::set<int> seen;
    for (int i = 0; i < n_open; ++i) {
        if (open[i] < 0 || open[i] >= n || !seen.insert(open[i]).second) {
            *err = "open qubits must be distinct and in range"; return QGM_E_INVALID;
        }
    }
    return QGM_OK;
}

// Kernel candidates of a step (see configure_step).
bool step_supports(const Step& st, int cand) {
    const int row_bits = st.r_in - st.kb;
    switch (cand) {
        case KC_VALU: return true;
        case KC_VALU_PAIR: {
            if (!(st.kb >= 3 && st.kb <= 5 && row_bits - st.vb >= 1)) return false;
            return true;
        }
        case KC_MFMA_F32:
        case KC_MFMA_BF16X3:
            return !st.input_is_one && st.kb >= 3 && st.kb <= 5 && st.nb >= 3 && st.nb <= 5 &&
                   row_bits - st.vb >= 4 && (1 << st.sb) <= kDenseMaxVariants;
        default: return false;
    }
}

// Sets the kernel of a step:
//  * KC_VALU: the vector-ALU kernel, one row per thread;
//  * KC_VALU_PAIR: the vector-ALU kernel with two rows per thread that differ
//    in a non-V bit (same v, same sigma), so every G read feeds two
//    multiply-adds;
//  * KC_MFMA_F32 / KC_MFMA_BF16X3: the matrix-core kernel (16-row tiles over 4
//    non-V row bits), FP32 or BF16x3 split precision.
void configure_step(Step& st, int cand) {
    st.kclass = 0;
    st.pair_bit = -1;
    st.pair_in = 0;
    st.inner_pos.clear();
    st.outer_pos.clear();
    const int row_bits = st.r_in - st.kb;
    std::set<int> vset(st.vpos.begin(), st.vpos.end());
    if (cand == KC_MFMA_F32 || cand == KC_MFMA_BF16X3) {
        for (int pos = 0; pos < row_bits; ++pos) {
            if (int(st.inner_pos.size()) < 4 && !vset.count(pos)) st.inner_pos.push_back(pos);
            else st.outer_pos.push_back(pos);
        }
        st.kclass = cand == KC_MFMA_BF16X3 ? 2 : 1;
    } else if (cand == KC_VALU_PAIR) {
        for (int pos = 0; pos < row_bits; ++pos) {
            if (vset.count(pos)) continue;
            st.pair_bit = pos;
            const int var = st.out_axes[pos];
            for (int i = 0; i < int(st.in_axes.size()); ++i)
                if (st.in_axes[i] == var) st.pair_in = 1 << i;
            break;
        }
    }
}

// Kernel of a step under a kernel_policy (autotuning may change it later).
static void classify_step(const Plan& p, Step& st) {
    int cand = KC_VALU;
    const int pol = p.opts.precision == QGM_PREC_BF16X3 ? 4 : p.opts.kernel_policy;
    if ((pol == 2 || pol == 4) && step_supports(st, KC_MFMA_F32)) cand = pol == 4 ? KC_MFMA_BF16X3 : KC_MFMA_F32;
    else if (pol == 3 && st.kb + st.nb >= 8 && step_supports(st, KC_VALU_PAIR)) cand = KC_VALU_PAIR;
    configure_step(st, cand);
}

// Builds steps for the current slicing; returns the peak rank.
static qgm_status build_steps(Plan& p, std::string* err) {
    p.steps.clear();
    const int n = p.n;
    std::vector<int> pos(n);
    for (int i = 0; i < n; ++i) pos[p.order[i]] = i;
    // owner step of each gate: the earliest qubit in the order among its qubits
    std::vector<std::vector<int>> owned(n);
    for (int r = 0; r < int(p.recs.size()); ++r) {
        const GateRec& g = p.recs[r];
        int owner = g.q0;
        if (g.type == 2 && pos[g.q1] < pos[g.q0]) owner = g.q1;
        owned[owner].push_back(r);
    }
    auto fixed_src = [&](int v, Src& s) -> bool {
        const VarInfo& vi = p.vars[v];
        if (vi.slice_idx >= 0) { s.src = SRC_SIG; return true; }
        if (vi.is_final && vi.open_idx < 0) { s.src = SRC_SIG; return true; }
        if (vi.is_c0 && vi.open_idx < 0) { s.src = SRC_ZERO; s.bit = 0; return true; }
        return false;
    };
    std::vector<int> S;   // frontier layout: variable at each position
    int r_peak = 0;
    int64_t g_off = 0;
    for (int si = 0; si < n; ++si) {
        const int q = p.order[si];
        Step st;
        st.qubit = q;
        st.input_is_one = (si == 0);
        st.in_axes = S;
        st.r_in = int(S.size());
        std::map<int, int> inpos;
        for (int i = 0; i < int(S.size()); ++i) inpos[S[i]] = i;
        // local variables of this step, in order of first use
        std::vector<int> local;
        std::set<int> local_set;
        auto touch = [&](int v) { if (v >= 0 && local_set.insert(v).second) local.push_back(v); };
        for (int v : p.chain[q]) touch(v);
        for (int r : owned[q]) { touch(p.recs[r].var0); touch(p.recs[r].var1); }
        std::map<int, Src> src;
        std::map<long long, int> sig_bit;   // key: qubit (>=0) or -(1+slice) -> bit
        auto sig_of = [&](int v) -> int {
            const VarInfo& vi = p.vars[v];
            long long key = vi.slice_idx >= 0 ? -(1LL + vi.slice_idx) : (long long)vi.qubit;
            auto it = sig_bit.find(key);
            if (it != sig_bit.end()) return it->second;
            int b = int(st.sig_src.size());
            st.sig_src.push_back(int(key));
            sig_bit[key] = b;
            return b;
        };
        for (int v : local) {
            Src s;
            const VarInfo& vi = p.vars[v];
            const bool own = (vi.qubit == q);
            const bool open_final = vi.is_final && vi.open_idx >= 0;
            if (fixed_src(v, s)) {
                if (s.src == SRC_SIG) s.bit = uint8_t(sig_of(v));
            } else if (inpos.count(v)) {
                if (own && !open_final) st.k_vars.push_back(v);
                else st.v_vars.push_back(v);
                s.src = (own && !open_final) ? SRC_K : SRC_V;
            } else {
                if (own && !open_final) s.src = SRC_INT;
                else { s.src = SRC_N; s.bit = uint8_t(st.n_vars.size()); st.n_vars.push_back(v); }
            }
            src[v] = s;
        }
        // a frontier variable of this qubit that the step does not touch cannot occur:
        // every worldline variable is touched by its gates.
        for (int v : S)
            if (p.vars[v].qubit == q && !src.count(v)) { *err = "internal: untouched frontier variable"; return QGM_E_INTERNAL; }
        // K bits in ascending input position
        std::sort(st.k_vars.begin(), st.k_vars.end(), [&](int a, int b) { return inpos[a] < inpos[b]; });
        for (int i = 0; i < int(st.k_vars.size()); ++i) {
            src[st.k_vars[i]].bit = uint8_t(i);
            st.kpos.push_back(inpos[st.k_vars[i]]);
        }
        // output layout: input axes without K (order kept), then N axes
        std::set<int> kset(st.k_vars.begin(), st.k_vars.end());
        for (int v : S) if (!kset.count(v)) st.out_axes.push_back(v);
        const int row_bits = int(st.out_axes.size());
        for (int v : st.n_vars) st.out_axes.push_back(v);
        std::map<int, int> outpos;
        for (int i = 0; i < int(st.out_axes.size()); ++i) outpos[st.out_axes[i]] = i;
        std::sort(st.v_vars.begin(), st.v_vars.end(), [&](int a, int b) { return outpos[a] < outpos[b]; });
        for (int i = 0; i < int(st.v_vars.size()); ++i) {
            src[st.v_vars[i]].bit = uint8_t(i);
            st.vpos.push_back(outpos[st.v_vars[i]]);
        }
        st.kb = int(st.k_vars.size());
        st.vb = int(st.v_vars.size());
        st.nb = int(st.n_vars.size());
        st.sb = int(st.sig_src.size());
        st.r_out = int(st.out_axes.size());
        (void)row_bits;
        if (st.kb > kMaxKB || st.vb > kMaxBits || st.sb > kMaxBits + 4 || st.nb > kMaxNB ||
            st.r_out > kMaxRank || st.r_in > kMaxRank) {
            char buf[200];
            snprintf(buf, sizeof buf, "step for qubit %d exceeds kernel limits (K=%d V=%d N=%d sigma=%d rank %d->%d)",
                     q, st.kb, st.vb, st.nb, st.sb, st.r_in, st.r_out);
            *err = buf;
            return QGM_E_UNSUPPORTED;
        }
        // factor program along the worldline of q (time order)
        auto emit = [&](uint8_t type, int v, int mat) {
            GOp op{};
            op.type = type;
            op.mat = mat;
            if (v >= 0) { op.src = src[v].src; op.bit = src[v].bit; }
            st.ops.push_back(op);
        };
        {
            int c0 = p.chain[q][0];
            if (src[c0].src != SRC_ZERO && src[c0].src != SRC_INT) emit(GOP_PROJECT, c0, -1);
        }
        for (int r : owned[q]) {
            const GateRec& g = p.recs[r];
            if (g.type == 0) {
                emit(GOP_MAT, -1, g.mat);
                if (src[g.var0].src != SRC_INT) emit(GOP_PROJECT, g.var0, -1);
            } else if (g.type == 1) {
                emit(GOP_DIAG, -1, g.mat);
            } else {
                int partner = (g.q0 == q) ? g.var1 : g.var0;
                if (src[partner].src == SRC_ZERO) continue;   // (-1)^{b*0} = 1
                emit(GOP_CZ, partner, -1);
            }
        }
        emit(GOP_END, p.chain[q].back(), -1);
        if (int(st.ops.size()) > kMaxOps) {
            *err = "factor program of qubit " + std::to_string(q) + " is longer than " + std::to_string(kMaxOps) + " ops";
            return QGM_E_UNSUPPORTED;
        }
        if (src[p.chain[q].back()].src == SRC_INT) { *err = "internal: final variable summed"; return QGM_E_INTERNAL; }
        st.g_off = g_off;
        g_off += st.g_entries();
        classify_step(p, st);
        r_peak = std::max(r_peak, std::max(st.r_in, st.r_out));
        S = st.out_axes;
        p.steps.push_back(std::move(st));
    }
    // the last frontier holds exactly the open variables
    if (int(S.size()) != p.n_open) { *err = "internal: final frontier is not the open set"; return QGM_E_INTERNAL; }
    p.final_pos.assign(p.n_open, -1);
    for (int i = 0; i < int(S.size()); ++i) p.final_pos[p.vars[S[i]].open_idx] = i;
    p.g_total = g_off;
    p.r_max = r_peak;
    p.n_ops_total = 0;
    for (auto& st : p.steps) p.n_ops_total += int64_t(st.ops.size());
    return QGM_OK;
}

// Picks the next variable to slice: among the non-open variables of the
// largest frontier, the one whose sliced plan moves the fewest bytes in total
// (every slice copy repeats the steps where the variable is not alive, so a
// short-lived variable costs more than it saves); ties go to the lower peak.
static int pick_slice_var(Plan& p, std::string* err) {
    int peak = -1, best_step = -1;
    bool out_side = false;
    for (int i = 0; i < int(p.steps.size()); ++i) {
        if (p.steps[i].r_in > peak) { peak = p.steps[i].r_in; best_step = i; out_side = false; }
        if (p.steps[i].r_out > peak) { peak = p.steps[i].r_out; best_step = i; out_side = true; }
    }
    if (best_step < 0) return -1;
    const std::vector<int> axes = out_side ? p.steps[best_step].out_axes : p.steps[best_step].in_axes;
    int best = -1, best_peak = 1 << 30;
    double best_bytes = 0;
    const int slice_idx = int(p.sliced.size());
    for (int v : axes) {
        if (p.vars[v].open_idx >= 0) continue;
        p.vars[v].slice_idx = slice_idx;
        std::string e;
        if (build_steps(p, &e) == QGM_OK) {
            double bytes = 0;
            for (auto& st : p.steps) bytes += st.bytes_per_b();
            if (best < 0 || bytes < best_bytes || (bytes == best_bytes && p.r_max < best_peak)) {
                best = v;
                best_bytes = bytes;
                best_peak = p.r_max;
            }
        }
        p.vars[v].slice_idx = -1;
    }
    if (best < 0) { *err = "no slicing candidate yields a valid plan"; return -1; }
    return best;
}

// <0|U^dag O U|0> for a Pauli string O is the amplitude at x = 0 of the circuit
// U, O, U^dag (the graphical model of Sec. III.B with the operator's factors).
// A gate of U outside the backward light cone of O's qubits cancels against
// its inverse (U_a^dag U_a = 1) and is left out: walking U backwards from O,
// a gate is kept when it touches a qubit of the cone, and a kept CZ adds its
// other qubit.  Output: the kept gates, O at cycle d (d = 1 + the last cycle),
// then the inverses of the kept gates in reverse order at cycle 2d - t.
qgm_status expectation_circuit(const qgm_circuit* c, int32_t n_ops, const int32_t* qubits, const int32_t* paulis,
                               std::vector<qgm_gate>& out, std::string* err) {
    qgm_status st = validate(c, nullptr, 0, err);
    if (st != QGM_OK) return st;
    const int n = c->rows * c->cols;
    if (n_ops < 1 || !qubits || !paulis) { *err = "the operator needs at least one (qubit, Pauli) pair"; return QGM_E_INVALID; }
    std::vector<char> in_cone(n, 0);
    for (int i = 0; i < n_ops; ++i) {
        if (qubits[i] < 0 || qubits[i] >= n) { *err = "operator qubit out of range"; return QGM_E_INVALID; }
        if (paulis[i] != QGM_X && paulis[i] != QGM_Y && paulis[i] != QGM_Z) {
            *err = "operator kinds must be QGM_X, QGM_Y or QGM_Z";
            return QGM_E_INVALID;
        }
        if (in_cone[qubits[i]]) { *err = "operator qubits must be distinct"; return QGM_E_INVALID; }
        in_cone[qubits[i]] = 1;
    }
    std::vector<int> idx(c->n_gates);
    int d = 0;
    for (int i = 0; i < c->n_gates; ++i) {
        idx[i] = i;
        const qgm_gate& g = c->gates[i];
        if (g.kind == QGM_U || g.kind == QGM_UD) {
            *err = "expectation circuits take fixed gate kinds only (no value slots)";
            return QGM_E_UNSUPPORTED;
        }
        d = std::max(d, g.cycle + 1);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return c->gates[a].cycle < c->gates[b].cycle; });
    std::vector<char> keep(c->n_gates, 0);
    for (int k = c->n_gates - 1; k >= 0; --k) {
        const qgm_gate& g = c->gates[idx[k]];
        const bool touches = in_cone[g.q0] || (g.kind == QGM_CZ && in_cone[g.q1]);
        if (!touches) continue;
        keep[idx[k]] = 1;
        in_cone[g.q0] = 1;
        if (g.kind == QGM_CZ) in_cone[g.q1] = 1;
    }
    auto inverse = [](int kind) {
        switch (kind) {
            case QGM_T: return int(QGM_TDG);
            case QGM_TDG: return int(QGM_T);
            case QGM_XH: return int(QGM_XHDG);
            case QGM_XHDG: return int(QGM_XH);
            case QGM_YH: return int(QGM_YHDG);
            case QGM_YHDG: return int(QGM_YH);
            default: return kind;   // H, CZ, X, Y, Z are their own inverses
        }
    };
    out.clear();
    for (int k = 0; k < c->n_gates; ++k)
        if (keep[idx[k]]) out.push_back(c->gates[idx[k]]);
    for (int i = 0; i < n_ops; ++i) out.push_back(qgm_gate{paulis[i], d, qubits[i], -1, -1});
    for (int k = c->n_gates - 1; k >= 0; --k)
        if (keep[idx[k]]) {
            qgm_gate g = c->gates[idx[k]];
            g.kind = inverse(g.kind);
            g.cycle = 2 * d - g.cycle;
            out.push_back(g);
        }
    return QGM_OK;
}

static qgm_status build_tree_sliced(Plan& p, std::string* err);

qgm_status build_plan(const qgm_circuit* c, const int32_t* open, int32_t n_open,
                      const qgm_plan_opts& opts, Plan& p, std::string* err) {
    qgm_status st = validate(c, open, n_open, err);
    if (st != QGM_OK) return st;
    if (opts.ordering != 0 && opts.ordering != 1) { *err = "ordering must be 0 or 1"; return QGM_E_INVALID; }
    if (opts.precision != QGM_PREC_C64 && opts.precision != QGM_PREC_BF16X3) {
        *err = "precision must be QGM_PREC_C64 (0) or QGM_PREC_BF16X3 (1)";
        return QGM_E_INVALID;
    }
    if (opts.kernel_policy < 0 || opts.kernel_policy > 4) { *err = "kernel_policy must be 0..4"; return QGM_E_INVALID; }
    if (opts.precision == QGM_PREC_BF16X3 && opts.ordering == 1) {
        *err = "precision BF16X3 runs on the matrix-core worldline steps of ordering 0; the bucket kernels are FP32";
        return QGM_E_UNSUPPORTED;
    }
    if (opts.precision == QGM_PREC_BF16X3 && opts.kernel_policy != 0 && opts.kernel_policy != 4) {
        *err = "precision BF16X3 selects the BF16x3 kernels: kernel_policy must be 0 or 4";
        return QGM_E_INVALID;
    }
    if (opts.tree_exec < 0 || opts.tree_exec > 3) { *err = "tree_exec must be 0..3"; return QGM_E_INVALID; }
    if (opts.no_tile < 0 || opts.no_tile > 1) { *err = "no_tile must be 0 or 1"; return QGM_E_INVALID; }
    if (opts.no_compose < 0 || opts.no_compose > 1) { *err = "no_compose must be 0 or 1"; return QGM_E_INVALID; }
    if (opts.reserved0 != 0) { *err = "reserved0 must be 0"; return QGM_E_INVALID; }
    if (opts.order_finalists < 0 || opts.order_finalists > kTreeMaxFinalists) {
        *err = "order_finalists must be in [0, 64]";
        return QGM_E_INVALID;
    }
    if (opts.order_restarts < 0 || opts.order_restarts > kTreeMaxRestarts) {
        *err = "order_restarts must be in [0, 1024]";
        return QGM_E_INVALID;
    }
    if (opts.order_pick < 0 || opts.order_pick >= kTreeMaxFinalists) {
        *err = "order_pick must be in [0, 63]";
        return QGM_E_INVALID;
    }
    if (opts.persist_spin < 0) { *err = "persist_spin must be >= 0"; return QGM_E_INVALID; }
    const int max_sliced = opts.ordering == 1 ? kTreeMaxSliced : 12;
    if (opts.min_sliced_vars < 0 || opts.min_sliced_vars > max_sliced || opts.max_rank < 0) {
        *err = "min_sliced_vars must be in [0, " + std::to_string(max_sliced) + "] and max_rank >= 0";
        return QGM_E_INVALID;
    }
    p.opts = opts;
    p.rows = c->rows;
    p.cols = c->cols;
    p.n = c->rows * c->cols;
    p.n_slots = c->n_slots;
    p.n_open = n_open;
    p.open_qubits.assign(open, open + n_open);
    const int n = p.n;
    // time order: (cycle, list index)
    std::vector<int> idx(c->n_gates);
    for (int i = 0; i < c->n_gates; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return c->gates[a].cycle < c->gates[b].cycle; });
    // worldline variables: b_q^0 for every qubit, then one per non-diagonal gate
    p.vars.clear();
    p.chain.assign(n, {});
    for (int q = 0; q < n; ++q) {
        VarInfo v; v.qubit = q; v.k = 0; v.is_c0 = true;
        p.vars.push_back(v);
        p.chain[q].push_back(q);
    }
    p.recs.clear();
    p.n_diag_gates = p.n_nondiag_gates = p.n_cz = p.n_2q = 0;
    for (int i : idx) {
        const qgm_gate& g = c->gates[i];
        GateRec r;
        r.gate_index = i;
        r.q0 = g.q0;
        if (g.kind == QGM_CZ) {
            r.type = 2; r.q1 = g.q1;
            r.var0 = p.chain[g.q0].back(); r.var1 = p.chain[g.q1].back();
            p.n_cz++;
        } else if (g.kind == QGM_U2) {   // both worldlines open a variable; the factor couples all four
            r.type = 3; r.q1 = g.q1; r.mat = kFixedMats + g.slot;
            r.var2 = p.chain[g.q0].back(); r.var3 = p.chain[g.q1].back();
            for (int k = 0; k < 2; ++k) {
                const int q = k == 0 ? g.q0 : g.q1;
                VarInfo v; v.qubit = q; v.k = int(p.chain[q].size());
                const int id = int(p.vars.size());
                p.vars.push_back(v);
                (k == 0 ? r.var0 : r.var1) = id;
                p.chain[q].push_back(id);
            }
            p.n_2q++;
        } else if (is_diag_kind(g.kind)) {
            r.type = 1; r.var0 = p.chain[g.q0].back(); r.mat = mat_index(g.kind, g.slot);
            p.n_diag_gates++;
        } else {
            r.type = 0; r.mat = mat_index(g.kind, g.slot);
            VarInfo v; v.qubit = g.q0; v.k = int(p.chain[g.q0].size());
            int id = int(p.vars.size());
            p.vars.push_back(v);
            r.var1 = p.chain[g.q0].back();
            r.var0 = id;
            p.chain[g.q0].push_back(id);
            p.n_nondiag_gates++;
        }
        p.recs.push_back(r);
    }
    for (int q = 0; q < n; ++q) p.vars[p.chain[q].back()].is_final = true;
    for (int i = 0; i < n_open; ++i) p.vars[p.chain[open[i]].back()].open_idx = i;
    if (p.n_2q > 0 && opts.ordering != 1) {
        *err = "non-diagonal two-qubit gates need bucket elimination (ordering 1)";
        return QGM_E_UNSUPPORTED;
    }
    p.sliced.clear();
    p.is_tree = opts.ordering == 1;
    if (p.is_tree) return build_tree_sliced(p, err);
    p.order = vertical_order(p.rows, p.cols);
    st = build_steps(p, err);
    if (st != QGM_OK) return st;
    while ((opts.max_rank > 0 && p.r_max > opts.max_rank) || int(p.sliced.size()) < opts.min_sliced_vars) {
        if (p.sliced.size() >= 12) { *err = "max_rank needs more than 12 sliced variables"; return QGM_E_OOM; }
        int v = pick_slice_var(p, err);
        if (v < 0) {
            if (opts.max_rank > 0 && p.r_max > opts.max_rank) { *err = "no variable left to slice"; return QGM_E_OOM; }
            break;
        }
        p.vars[v].slice_idx = int(p.sliced.size());
        p.sliced.push_back(v);
        st = build_steps(p, err);
        if (st != QGM_OK) return st;
    }
    if (opts.precision == QGM_PREC_BF16X3 &&
        std::none_of(p.steps.begin(), p.steps.end(), [](const Step& x) { return x.kclass == 2; })) {
        *err = "precision BF16X3: no step of this plan fits the BF16x3 matrix-core kernel (K and N of 2^3..2^5)";
        return QGM_E_UNSUPPORTED;
    }
    // the slices of ordering 0 run as batch columns, which does not shrink the frontier: the budget is a check
    if (opts.mem_budget > 0 && workspace_layout(p, 64).total > opts.mem_budget) {
        *err = "mem_budget: the vertical plan needs " + std::to_string(workspace_layout(p, 64).total) +
               " bytes per 64 bitstrings (ordering 1 slices to fit a budget)";
        return QGM_E_OOM;
    }
    // checkpoints of qgm_backward: as many as the budget holds (less recomputation), at least the sqrt(steps)
    // schedule
    p.ckpt_every = 0;
    if (opts.checkpoint_budget > 0 && opts.checkpoint_every == 0) {
        const int S = int(p.steps.size());
        const uint64_t frame = (uint64_t(1) << p.r_max) * 64 * 8;
        const int c_sqrt = std::max(1, int(std::ceil(std::sqrt(double(S)))));
        for (int c = 1; c <= c_sqrt; ++c) {
            const uint64_t frames = uint64_t((S - 1) / c) + uint64_t(c - 1);
            if (frames * frame <= opts.checkpoint_budget) { p.ckpt_every = c; break; }
        }
        if (p.ckpt_every == 0) {
            *err = "checkpoint_budget: the sqrt(steps) checkpoint schedule needs " +
                   std::to_string((uint64_t((S - 1) / c_sqrt) + uint64_t(c_sqrt - 1)) * frame) +
                   " bytes per 64 bitstrings";
            return QGM_E_OOM;
        }
    }
    return QGM_OK;
}

// Ordering 1: bucket plans with sliced variables added one at a time (the one
// in the most of the largest results) until the plan fits the kernels and
// meets min_sliced_vars, max_rank and mem_budget; then the largest chunk of
// slices per launch sequence whose workspace fits the budget.
static qgm_status build_tree_sliced(Plan& p, std::string* err) {
    const qgm_plan_opts& opts = p.opts;
    std::vector<int> sliced;
    std::string why;
    while (true) {
        std::string e;
        const qgm_status st = build_tree_plan(p, sliced, p.tree, &e);
        if (st != QGM_OK && st != QGM_E_UNSUPPORTED) { *err = e; return st; }
        bool more = false;
        if (st == QGM_E_UNSUPPORTED) {
            // a persistent-launch or open-qubit refusal is not cured by slicing
            if (e.find("persistent") != std::string::npos || e.find("tree_exec 3") != std::string::npos) {
                *err = e;
                return st;
            }
            more = true;
            why = e;
        } else {
            p.r_max = p.tree.max_rank;
            p.g_total = p.tree.g_total;
            p.tree.chunk_bits = int(sliced.size());
            if (int(sliced.size()) < opts.min_sliced_vars) {
                more = true;
            } else if (opts.max_rank > 0 && p.tree.max_rank > opts.max_rank) {
                more = true;
                why = "max_rank " + std::to_string(opts.max_rank) + " (the plan's largest result has rank " +
                      std::to_string(p.tree.max_rank) + ")";
            } else if (opts.mem_budget > 0) {
                // the largest chunk of slices that fits; slice further when even one slice at a time does not
                int cb = int(sliced.size());
                while (cb > 0 && workspace_layout_chunk(p, 64, cb).total > opts.mem_budget) --cb;
                if (workspace_layout_chunk(p, 64, cb).total > opts.mem_budget) {
                    more = true;
                    why = "mem_budget " + std::to_string(opts.mem_budget) + " bytes (one slice at a time needs " +
                          std::to_string(workspace_layout_chunk(p, 64, cb).total) + " per 64 bitstrings)";
                } else {
                    p.tree.chunk_bits = cb;
                }
            }
        }
        if (!more) break;
        if (int(sliced.size()) >= kTreeMaxSliced || p.n + int(sliced.size()) >= 64) {
            *err = "slicing " + std::to_string(sliced.size()) + " variables does not meet " + why;
            return opts.mem_budget > 0 || opts.max_rank > 0 ? QGM_E_OOM : QGM_E_UNSUPPORTED;
        }
        const int v = tree_pick_slice_var(p, sliced, st == QGM_OK ? &p.tree : nullptr);
        if (v < 0) {
            *err = "no variable left to slice: " + why;
            return opts.mem_budget > 0 || opts.max_rank > 0 ? QGM_E_OOM : QGM_E_UNSUPPORTED;
        }
        sliced.push_back(v);
    }
    for (size_t j = 0; j < sliced.size(); ++j) p.vars[sliced[j]].slice_idx = int(j);
    p.steps.clear();
    p.order.clear();
    p.final_pos.clear();
    if (opts.checkpoint_budget > 0) {
        // the bucket path's adjoint keeps every result: no schedule to trade
        const uint64_t keep = uint64_t(p.tree.arena_rows_all) * 64 * 8;
        if (keep > opts.checkpoint_budget) {
            *err = "checkpoint_budget: the bucket adjoint keeps every result, " + std::to_string(keep) +
                   " bytes per 64 bitstrings";
            return QGM_E_OOM;
        }
    }
    return QGM_OK;
}

bool tree_persistent(const Plan& p, int64_t) { return p.is_tree && p.opts.tree_exec == 2; }

bool tree_lds(const Plan& p, int64_t) {
    return p.is_tree && p.tree.lds.ok && (p.opts.tree_exec == 3 || p.opts.tree_exec == 0);
}

int64_t tree_flag_stride(const Plan& p) { return (p.tree.n_tasks + 31) / 32 * 32; }

int64_t tree_flag_words(const Plan& p, int64_t B) {
    return kPersistFlags0 + tree_pitch(B) / 64 * tree_flag_stride(p);   // one flag row per group of the pitch
}

WsLayout workspace_layout(const Plan& p, int64_t B) { return workspace_layout_chunk(p, B, p.tree.chunk_bits); }

WsLayout workspace_layout_chunk(const Plan& p, int64_t B, int chunk_bits) {
    auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
    WsLayout w;
    if (p.is_tree) {
        // results (lifetime-packed rows; every result at its own rows for the persistent launch), factor
        // tables only when the circuit reads gate values (otherwise the plan's device tables hold them,
        // built once), the persistent launch's flags; with slicing, the words of one chunk's batch columns,
        // their amplitudes (complex128) and, over several chunks, the FP64 running sums
        const bool persist = tree_persistent(p, B);
        const uint64_t cols = uint64_t(B) << chunk_bits;
        const uint64_t be = uint64_t(tree_pitch(int64_t(cols)));
        w.f0 = w.f1 = 0;
        const uint64_t arena = tree_lds(p, B) ? 0 : al(uint64_t(persist ? p.tree.arena_rows_all : p.tree.arena_rows) * be * 8);
        w.g = arena;
        w.flags = w.g + (p.n_slots > 0 ? al(uint64_t(p.tree.g_total) * 8) : 0);
        w.var_ids = w.flags;
        uint64_t end = w.flags + (persist ? al(uint64_t(tree_flag_words(p, B)) * 4) : 0);
        if (!p.tree.sliced.empty()) {
            const uint64_t n_out = uint64_t(1) << p.n_open;
            w.ext = end;
            w.part = w.ext + al(cols * 8);
            w.acc = w.part + al(cols * n_out * 16);
            end = w.acc + (chunk_bits < int(p.tree.sliced.size()) ? al(uint64_t(B) * n_out * 16) : 0);
        }
        w.total = end;
        return w;
    }
    const uint64_t be = uint64_t(batch_eff(p, B));
    const uint64_t fbytes = al((uint64_t(1) << p.r_max) * be * 8);
    w.f0 = 0;
    w.f1 = fbytes;
    w.var_ids = 2 * fbytes;
    w.g = w.var_ids + al(uint64_t(p.steps.size()) * be * 2);
    w.total = w.g + al(uint64_t(p.g_total) * 8);
    return w;
}

static const char* kernel_name(const Step& st) {
    if (st.kclass == 1) return "mfma_f32";
    if (st.kclass == 2) return "mfma_bf16x3";
    return st.pair_bit >= 0 ? "valu_pair" : "valu";
}

static void json_ints(std::ostringstream& o, const std::vector<int>& v) {
    o << "[";
    for (size_t i = 0; i < v.size(); ++i) o << (i ? "," : "") << v[i];
    o << "]";
}

static void json_factor(std::ostringstream& o, const TFactor& f) {
    o << "[" << f.type << "," << f.mat << "," << f.src0 << "," << f.bit0 << "," << f.src1 << "," << f.bit1;
    if (f.type == TF_MAT4) o << "," << f.src2 << "," << f.bit2 << "," << f.src3 << "," << f.bit3;
    o << "]";
}

static std::string tree_json(const Plan& p, int detail) {
    const TreePlan& t = p.tree;
    const double sl_mult = double(int64_t(1) << t.sliced.size());   // per amplitude: every slice's column
    std::ostringstream o;
    o.precision(17);
    o << "{\"ordering\":1,\"n\":" << p.n << ",\"rows\":" << p.rows << ",\"cols\":" << p.cols
      << ",\"n_vars\":" << p.vars.size() << ",\"n_free\":" << t.n_free << ",\"n_open\":" << t.n_open
      << ",\"n_slots\":" << p.n_slots
      << ",\"n_steps\":0,\"n_buckets\":" << t.steps.size() << ",\"n_levels\":" << t.levels.size()
      << ",\"max_rank\":" << t.max_rank << ",\"max_inputs\":" << t.max_in << ",\"n_sliced\":" << t.sliced.size()
      << ",\"slice_chunk_bits\":" << t.chunk_bits
      << ",\"chain_merge\":" << (p.opts.no_chain_merge ? 0 : 1) << ",\"n_tasks\":" << t.n_tasks
      << ",\"absorbed_buckets\":" << t.n_absorbed << ",\"tail_levels\":" << (int(t.levels.size()) - t.tail_start)
      << ",\"first_level\":" << t.first_level << ",\"tail_start\":" << t.tail_start << ",\"tail_lds_rows\":" << t.tail_lds_rows
      << ",\"level_launches\":" << tree_launches(t) << ",\"kernel_launches\":" << tree_kernel_launches(t)
      << ",\"level_quad\":[";
    for (size_t L = 0; L < t.level_quad.size(); ++L) o << (L ? "," : "") << t.level_quad[L];
    o << "]"
      << ",\"n_cz\":" << p.n_cz << ",\"n_diag_1q\":" << p.n_diag_gates << ",\"n_nondiag_1q\":" << p.n_nondiag_gates << ",\"n_2q\":" << p.n_2q
      << ",\"g_entries\":" << t.g_total << ",\"arena_rows\":" << t.arena_rows
      << ",\"orders_tried\":" << t.n_candidates << ",\"orders_built\":" << t.n_built << ",\"order_score\":" << t.order_score << ",\"bytes_per_amp\":" << t.bytes_per_b * sl_mult
      << ",\"flops_per_amp\":" << t.flops_per_b * sl_mult << ",\"n_phase\":" << t.phase.size()
      << ",\"open_tensor\":" << t.open_tensor << ",\"zero_mask\":" << t.zero_mask
      << ",\"table_leaves\":" << t.n_table_leaves
      << ",\"lds_ok\":" << (t.lds.ok ? 1 : 0) << ",\"lds_entries\":" << t.lds.lds_size
      << ",\"lds_jobs\":" << t.lds.jobs.size() << ",\"lds_tables0\":" << t.lds.tables0
      << ",\"lds_threads\":" << t.lds.threads << ",\"lds_recs0\":" << t.lds.recs0
      << ",\"lds_bytes_per_amp\":" << double(lds_bytes_per_amp(t.lds)) * sl_mult
      << ",\"lds_why\":\"" << t.lds.why << "\"";
    std::vector<int> sl_q, sl_k;
    for (int v : t.sliced) { sl_q.push_back(p.vars[v].qubit); sl_k.push_back(p.vars[v].k); }
    o << ",\"sliced_qubit\":"; json_ints(o, sl_q);
    o << ",\"sliced_k\":"; json_ints(o, sl_k);
    o << ",\"order\":"; json_ints(o, t.order);
    o << ",\"finals\":"; json_ints(o, t.finals);
    o << ",\"steps\":[],\"buckets\":[";
    for (size_t i = 0; i < t.steps.size(); ++i) {
        const TreeStep& st = t.steps[i];
        o << (i ? "," : "") << "{\"vars\":";
        json_ints(o, st.vars);
        o << ",\"kg\":" << st.kg << ",\"level\":" << st.level << ",\"r_out\":" << st.out_axes.size()
          << ",\"n_in\":" << st.in_tensors.size() << ",\"gb\":" << st.gb() << ",\"sb\":" << st.sb()
          << ",\"n_factors\":" << st.n_factors() << ",\"g_off\":" << st.g_off
          << ",\"bytes_per_b\":" << tree_step_bytes(t, st) << ",\"unit_rows\":" << st.unit_rows << ",\"tile\":" << st.tile << ",\"quad\":" << (st.quad ? 1 : 0) << ",\"composed\":" << (st.composed ? 1 : 0)
          << ",\"table_leaf\":" << (st.table_leaf ? 1 : 0) << ",\"leaf_off\":" << st.leaf_off
          << ",\"issued_bytes_per_b\":" << 8 * st.n_tasks() * tree_unit_accesses(t, st);
        if (detail >= 1) {
            o << ",\"out_tensor\":" << st.out_tensor;
            o << ",\"out_axes\":"; json_ints(o, st.out_axes);
            o << ",\"in_tensors\":"; json_ints(o, st.in_tensors);
            o << ",\"gvars\":"; json_ints(o, st.gvars);
            o << ",\"sig_q\":"; json_ints(o, st.sig_q);
            o << ",\"groups\":[";
            for (size_t gi = 0; gi < st.groups.size(); ++gi) {
                o << (gi ? "," : "") << "{\"k\":" << st.groups[gi].k_int << ",\"vars\":";
                json_ints(o, st.groups[gi].vars);
                o << ",\"factors\":[";
                for (size_t j = 0; j < st.groups[gi].factors.size(); ++j) {
                    if (j) o << ",";
                    json_factor(o, st.groups[gi].factors[j]);
                }
                o << "]}";
            }
            o << "]";
        }
        o << "}";
    }
    o << "]";
    if (detail >= 1) {
        o << ",\"tensors\":[";
        for (size_t i = 0; i < t.tensor_axes.size(); ++i) {
            o << (i ? "," : "") << "{\"axes\":";
            json_ints(o, t.tensor_axes[i]);
            o << ",\"made\":" << t.tensor_made[i] << ",\"used\":" << t.tensor_used[i] << ",\"row\":" << t.tensor_row[i]
              << ",\"alloc_rows\":" << (int64_t(1) << std::max(int(t.tensor_axes[i].size()), kTreeOcBits)) << "}";
        }
        o << "],\"phase\":[";
        for (size_t j = 0; j < t.phase.size(); ++j) { if (j) o << ","; json_factor(o, t.phase[j]); }
        o << "]";
    }
    if (detail >= 2 && t.lds.ok) {   // the LDS-resident program, for the CPU interpreter of the tests
        const LdsProgram& L = t.lds;
        o << ",\"lds\":{\"size\":" << L.lds_size << ",\"tables0\":" << L.tables0 << ",\"stages\":[";
        for (size_t i = 0; i < L.stages.size(); ++i) {
            o << (i ? "," : "") << "{\"bucket\":" << L.stage_bucket[i] << ",\"sig_q\":[";
            for (int b = 0; b < L.stages[i].n_sig; ++b) o << (b ? "," : "") << L.stages[i].sig_q[b];
            o << "],\"n\":" << L.stages[i].n << ",\"zoff\":" << L.stages[i].zoff << ",\"e0\":" << L.stages[i].e0 << "}";
        }
        o << "],\"z_entries\":" << L.z_entries << ",\"entries\":[";
        for (size_t i = 0; i < L.entries.size(); ++i)
            o << (i ? "," : "") << "[" << L.entries[i].src << "," << L.entries[i].stage << "," << (L.zent[i] & 0xFFFFFFu) << "]";
        o << "],\"jobs\":[";
        for (size_t j = 0; j < L.jobs.size(); ++j) {
            const LdsJob& jb = L.jobs[j];
            o << (j ? "," : "") << "{\"bucket\":" << L.job_bucket[j] << ",\"nin\":" << jb.nin << ",\"k\":" << jb.k
              << ",\"lanes\":" << jb.lanes << ",\"rl\":" << jb.rl << ",\"out_row\":" << (jb.out_row - kLdsHeader) / 8
              << ",\"in_w\":[";
            for (int k = 0; k < jb.nin; ++k) {
                o << (k ? "," : "") << "[";
                for (int w = 0; w < (1 << jb.k); ++w) o << (w ? "," : "") << jb.in_w[k][w] / 8;
                o << "]";
            }
            o << "],\"tw\":[";
            for (int w = 0; w < (1 << jb.k); ++w) o << (w ? "," : "") << jb.tw[w] / 8;
            o << "],\"base\":[";
            for (int sl = 0; sl <= jb.nin; ++sl)
                o << (sl ? "," : "") << (jb.base[sl < jb.nin ? sl : kLdsMaxIn] - kLdsHeader) / 8;
            o << "],\"str\":[";
            for (int sl = 0; sl <= jb.nin; ++sl) {
                o << (sl ? "," : "") << "[";
                for (int i = 0; i < 6; ++i) o << (i ? "," : "") << jb.str[sl < jb.nin ? sl : kLdsMaxIn][i] / 8;
                o << "]";
            }
            o << "],\"strx\":[";
            for (int x = 0; x < 2; ++x) {
                o << (x ? ",[" : "[");
                for (int sl = 0; sl <= jb.nin; ++sl) o << (sl ? "," : "") << jb.strx[x][sl < jb.nin ? sl : kLdsMaxIn] / 8;
                o << "]";
            }
            o << "]}";
        }
        o << "],\"level_job_off\":[";
        for (size_t i = 0; i < L.level_job_off.size(); ++i) o << (i ? "," : "") << L.level_job_off[i];
        o << "],\"finals\":[";
        for (size_t i = 0; i < L.finals.size(); ++i) o << (i ? "," : "") << (L.finals[i] - kLdsHeader) / 8;
        o << "]}";
    }
    o << "}";
    return o.str();
}

std::string plan_json(const Plan& p, int detail) {
    if (p.is_tree) return tree_json(p, detail);
    std::ostringstream o;
    o.precision(17);
    double bytes = 0, flops = 0;
    for (auto& st : p.steps) { bytes += st.bytes_per_b(); flops += st.flops_per_b(); }
    o << "{\"ordering\":0,\"n\":" << p.n << ",\"rows\":" << p.rows << ",\"cols\":" << p.cols << ",\"n_vars\":" << p.vars.size()
      << ",\"n_open\":" << p.n_open << ",\"n_slots\":" << p.n_slots << ",\"n_steps\":" << p.steps.size()
      << ",\"max_rank\":" << p.r_max << ",\"n_sliced\":" << p.sliced.size()
      << ",\"checkpoint_every\":" << (p.opts.checkpoint_every > 0 ? p.opts.checkpoint_every : p.ckpt_every)
      << ",\"n_cz\":" << p.n_cz << ",\"n_diag_1q\":" << p.n_diag_gates << ",\"n_nondiag_1q\":" << p.n_nondiag_gates << ",\"n_2q\":" << p.n_2q
      << ",\"g_entries\":" << p.g_total
      << ",\"bytes_per_amp\":" << bytes * double(int64_t(1) << p.sliced.size())
      << ",\"flops_per_amp\":" << flops * double(int64_t(1) << p.sliced.size());
    o << ",\"open_qubits\":"; json_ints(o, p.open_qubits);
    o << ",\"order\":"; json_ints(o, p.order);
    o << ",\"final_pos\":"; json_ints(o, p.final_pos);
    std::vector<int> sl_q, sl_k;
    for (int v : p.sliced) { sl_q.push_back(p.vars[v].qubit); sl_k.push_back(p.vars[v].k); }
    o << ",\"sliced_qubit\":"; json_ints(o, sl_q);
    o << ",\"sliced_k\":"; json_ints(o, sl_k);
    o << ",\"steps\":[";
    for (size_t i = 0; i < p.steps.size(); ++i) {
        const Step& st = p.steps[i];
        o << (i ? "," : "") << "{\"qubit\":" << st.qubit << ",\"r_in\":" << st.r_in << ",\"r_out\":" << st.r_out
          << ",\"kb\":" << st.kb << ",\"vb\":" << st.vb << ",\"nb\":" << st.nb << ",\"sb\":" << st.sb
          << ",\"input_is_one\":" << (st.input_is_one ? 1 : 0) << ",\"g_off\":" << st.g_off
          << ",\"kernel\":\"" << kernel_name(st) << "\""
          << ",\"bytes_per_b\":" << st.bytes_per_b() << ",\"flops_per_b\":" << st.flops_per_b();
        if (detail >= 1) {
            o << ",\"kpos\":"; json_ints(o, st.kpos);
            o << ",\"vpos\":"; json_ints(o, st.vpos);
            o << ",\"sig_src\":"; json_ints(o, st.sig_src);
            o << ",\"in_axes\":"; json_ints(o, st.in_axes);
            o << ",\"out_axes\":"; json_ints(o, st.out_axes);
            o << ",\"ops\":[";
            for (size_t j = 0; j < st.ops.size(); ++j) {
                const GOp& g = st.ops[j];
                o << (j ? "," : "") << "[" << int(g.type) << "," << int(g.src) << "," << int(g.bit) << "," << g.mat << "]";
            }
            o << "]";
        }
        o << "}";
    }
    o << "]";
    if (detail >= 1) {
        o << ",\"vars\":[";
        for (size_t i = 0; i < p.vars.size(); ++i) {
            const VarInfo& v = p.vars[i];
            o << (i ? "," : "") << "[" << v.qubit << "," << v.k << "," << (v.is_c0 ? 1 : 0) << ","
              << (v.is_final ? 1 : 0) << "," << v.open_idx << "," << v.slice_idx << "]";
        }
        o << "]";
    }
    o << "}";
    return o.str();
}

}  // namespace qgm
