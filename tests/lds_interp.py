"""CPU interpreter of the LDS-resident program of a bucket plan (qgm_amplitudes
with tree_exec 3), complex128.

It executes the program the planner exports (plan JSON detail 2, "lds"): the
table slices copied at a bitstring's output bits, then level by level the jobs
-- 64 result rows of one bucket (128 or 256 for a job of two or four rows
per lane, the further rows at the strides of result bits 6 and 7), lane l reading its inputs and the factor-table slice at the
job's base offsets plus the strides of its six lane bits plus the
per-summed-value offsets --
and finally phase x the rank-0 results.  Every LDS entry read must have been
written (entries start as NaN) and stay inside the program's LDS size, and
no level may write an entry that the same level reads, which is what the
kernel's one barrier per level relies on.  The table contents come from the
bucket definitions of the same JSON (the semantics the device's table
builder implements).  It is neither the oracle nor a fallback of the product
path.
"""
import numpy as np

from tree_interp import TS_SIG, _eval, bucket_table


def _table_area(info, gate_vals):
    """The table area as the device builds it, as a dict offset -> value:
    bucket s's factor table at g_off, entry (c << sb) | sigma with
    c = (g << kg) | w, and a leaf bucket's result table at leaf_off, entry
    (o << sb) | sigma with o over the result's axes in the planner's order.  A
    composed leaf (inputs all leaf tables) sums over w its factor table times
    its inputs' tables, read at the entries its result index, w and output
    bits select (its output bits are its own, then its inputs' others)."""
    area = {}
    tensors = info["tensors"]
    maker = {st["out_tensor"]: st for st in info["buckets"]}
    leaf = {}   # leaf tables as arrays [2^r, 2^sb], by result
    for st in info["buckets"]:
        G = bucket_table(st, gate_vals)             # [2^(gb + kg), 2^sb]
        sb, kg = st["sb"], st["kg"]
        if not st["table_leaf"]:
            for c in range(G.shape[0]):
                for sg in range(G.shape[1]):
                    area[st["g_off"] + (c << sb) + sg] = G[c, sg]
            continue
        out_axes = st["out_axes"]
        r = st["r_out"]
        O = np.arange(1 << r)[:, None]
        SG = np.arange(1 << sb)[None, :]
        g = np.zeros_like(O)
        for j, ax in enumerate(st["gvars"]):
            g |= ((O >> out_axes.index(ax)) & 1) << j
        R = np.zeros((1 << r, 1 << sb), dtype=np.complex128)
        for w in range(1 << kg):
            term = G[(g << kg) | w, SG]
            if st.get("composed", 0):
                for tin in st["in_tensors"]:
                    mk = maker[tin]
                    idx = np.zeros_like(O)
                    for a, ax in enumerate(tensors[tin]["axes"]):
                        bit = ((O >> out_axes.index(ax)) & 1) if ax in out_axes else \
                            np.full_like(O, (w >> st["vars"].index(ax)) & 1)
                        idx |= bit << a
                    s_t = np.zeros_like(SG)
                    for b, q in enumerate(mk["sig_q"]):
                        s_t |= ((SG >> st["sig_q"].index(q)) & 1) << b
                    term = term * leaf[tin][idx, s_t]
            R = R + term
        leaf[st["out_tensor"]] = R
        for o in range(1 << r):
            for sg in range(1 << sb):
                area[st["leaf_off"] + (o << sb) + sg] = R[o, sg]
    return area


def run_lds_program(info, gate_vals, bits):
    """Amplitudes complex128 [B] of a detail-2 plan with an LDS program."""
    L = info["lds"]
    area = _table_area(info, gate_vals)
    size = L["size"]
    out = np.zeros(len(bits), dtype=np.complex128)
    stage_q = [st["sig_q"] for st in L["stages"]]
    S, n = info.get("n_sliced", 0), info["n"]
    for bi, x in enumerate(np.asarray(bits, dtype=np.uint64)):
        # a sliced plan: one program run per slice s (sliced variable j fixed by bit n + j), summed
        out[bi] = sum(_run_column(info, L, area, stage_q, size, int(x) | (s << n), gate_vals) for s in range(1 << S))
    return out


def _run_column(info, L, area, stage_q, size, x, gate_vals):
    """One batch column (bitstring word x, slice bits above the qubits) through the LDS program."""
    lds = np.full(size, np.nan, dtype=np.complex128)
    sig = [sum(((x >> q) & 1) << i for i, q in enumerate(sq)) for sq in stage_q]
    stages = L["stages"]
    for e, (src, s, zsrc) in enumerate(L["entries"]):
        dst = L["tables0"] + e
        assert 0 <= dst < size
        # the device reads the staged copy: staged[zoff + sigma * n + i] = area[src of entry e0 + i + sigma]
        st = stages[s]
        i = e - st["e0"]
        assert 0 <= i < st["n"] and zsrc == st["zoff"] + i
        assert st["zoff"] + sig[s] * st["n"] + i < L["z_entries"]
        lds[dst] = area[L["entries"][st["e0"] + i][0] + sig[s]]
        assert L["entries"][st["e0"] + i][0] == src
    offs = L["level_job_off"]
    for lv in range(len(offs) - 1):
        writes, reads = {}, set()
        for j in range(offs[lv], offs[lv + 1]):
            jb = L["jobs"][j]
            nin, k, lanes = jb["nin"], jb["k"], jb["lanes"]
            for lane in range(64 << jb["rl"]):
                # the lane's offsets: the job's base plus the strides of the lane's six bits (inputs, then
                # the table); row m of a job of 2 or 4 rows per lane adds the strides of result bits 6, 7
                m, ln = lane >> 6, lane & 63
                off = [jb["base"][sl] + sum(((ln >> i) & 1) * jb["str"][sl][i] for i in range(6))
                       + sum(((m >> x) & 1) * jb["strx"][x][sl] for x in range(2))
                       for sl in range(nin + 1)]
                acc = 0j
                for w in range(1 << k):
                    a = off[nin] + jb["tw"][w]
                    assert 0 <= a < size
                    v = lds[a]
                    reads.add(a)
                    for t in range(nin):
                        a = off[t] + jb["in_w"][t][w]
                        assert 0 <= a < size, (j, lane, t, w, a)
                        reads.add(a)
                        v = v * lds[a]
                    acc += v
                if ln < lanes:
                    dst = jb["out_row"] + lane
                    assert 0 <= dst < L["tables0"], (j, lane, dst)
                    assert not np.isnan(acc), (lv, j, lane)
                    assert dst not in writes
                    writes[dst] = acc
        assert not (set(writes) & reads), "a level writes an entry it reads"
        for d, v in writes.items():
            lds[d] = v
    amp = 1.0 + 0j
    for f in info["phase"]:
        amp = amp * complex(_eval(f, lambda src, bit: ((x >> bit) & 1) if src == TS_SIG else 0, gate_vals))
    for fr in L["finals"]:
        assert not np.isnan(lds[fr])
        amp *= lds[fr]
    return amp
