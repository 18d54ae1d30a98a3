"""CPU interpreter of a bucket-elimination plan (ordering 1), complex128.

It executes the planner's output -- bucket factor groups (a bucket without
inputs folded into its reader's table), summed variables (several for a
merged chain), axis layouts, variant bits, tree levels and arena rows -- with
the semantics the HIP bucket kernels implement, so the planner can be checked against the oracle without a
GPU.  Results live in a simulated arena: every row remembers which result
wrote it, a read checks that the row still holds that result, and a level's
writes may not land on rows of a result that the level (or a later one) still
reads.  It is neither the oracle nor a fallback of the product path.
"""
import numpy as np

from oracle.gates import gate_matrix

TS_ZERO, TS_G, TS_SIG, TS_INT = 0, 1, 2, 3
TF_MAT, TF_DIAG, TF_CZ, TF_DELTA0, TF_MAT4 = 0, 1, 2, 3, 4


# matrix index -> gate kind of the library's fixed matrices (H, T, X^1/2, Y^1/2, their inverses, X, Y, Z);
# index 10 + s is value slot s
_FIXED_KIND = (0, 1, 2, 3, 7, 8, 9, 10, 11, 12)


def _mat(idx, gate_vals):
    if idx < len(_FIXED_KIND):
        return gate_matrix(_FIXED_KIND[idx], -1, None)
    return np.asarray(gate_vals[idx - len(_FIXED_KIND)], dtype=np.complex128).reshape(2, 2)


def _factor4(f, a0, a1, c0, c1, gate_vals):
    """Two-qubit gate factor: M[2 a0 + a1][2 c0 + c1], row r in value slot (mat - 10) + r."""
    s0 = f[1] - len(_FIXED_KIND)
    M = np.stack([np.asarray(gate_vals[s0 + r], dtype=np.complex128).reshape(4) for r in range(4)])
    return M[2 * a0 + a1, 2 * c0 + c1]


def _eval(f, val, gate_vals):
    """A factor record's value; val(src, bit) gives each variable's values."""
    if f[0] == TF_MAT4:
        return _factor4(f, val(f[2], f[3]), val(f[4], f[5]), val(f[6], f[7]), val(f[8], f[9]), gate_vals)
    return _factor(f, val(f[2], f[3]), val(f[4], f[5]), gate_vals)


def _factor(f, a, b, gate_vals):
    typ, mat = f[0], f[1]
    if typ == TF_MAT:
        return _mat(mat, gate_vals)[a, b]
    if typ == TF_DIAG:
        return _mat(mat, gate_vals)[a, a]
    if typ == TF_CZ:
        return np.where((a & b) == 1, -1.0, 1.0)
    return np.where(a == 1, 0.0, 1.0)


def bucket_table(st, gate_vals):
    """G of a bucket as [2^(gb+kg) (index c = (g << kg) | w), 2^sb]: the product
    over its factor groups of (product of the group's factors), summed over the
    group's own variables (TS_INT) for an absorbed bucket."""
    gb, sb, kg = st["gb"], st["sb"], st["kg"]
    c = np.arange(1 << (gb + kg))[:, None]
    sig = np.arange(1 << sb)[None, :]
    acc = np.ones((1 << (gb + kg), 1 << sb), dtype=np.complex128)

    def val(src, bit, iv):
        if src == TS_G:
            return ((c >> bit) & 1) + 0 * sig
        if src == TS_SIG:
            return ((sig >> bit) & 1) + 0 * c
        if src == TS_INT:
            return ((iv >> bit) & 1) + 0 * (c + sig)
        return np.zeros_like(c + sig)

    for grp in st["groups"]:
        total = np.zeros_like(acc)
        for iv in range(1 << grp["k"]):
            term = np.ones_like(acc)
            for f in grp["factors"]:
                term = term * _eval(f, lambda src, bit: val(src, bit, iv), gate_vals)
            total += term
        acc = acc * total
    return acc


def run_tree_plan(info, gate_vals, bits):
    """Executes a detail-1 tree plan for uint64 bitstrings; returns complex128 [B]
    (or [B, 2^n_open]).  A sliced plan runs once per slice s, with s in the bits
    above the n qubits of every word (sliced variable j is fixed by bit n + j),
    and the slices are summed."""
    bits = np.asarray(bits, dtype=np.uint64)
    S = info.get("n_sliced", 0)
    if S == 0:
        return _run_tree_columns(info, gate_vals, bits)
    return sum(_run_tree_columns(info, gate_vals, bits | np.uint64(s << info["n"])) for s in range(1 << S))


def _run_tree_columns(info, gate_vals, bits):
    B = len(bits)
    tensors = info["tensors"]
    arena = np.zeros((max(info["arena_rows"], 1), B), dtype=np.complex128)
    owner = np.full(max(info["arena_rows"], 1), -1)
    xb = lambda q: ((bits >> np.uint64(q)) & np.uint64(1)).astype(np.int64)

    tables = {}   # results of leaf-table buckets (built with the plan, not in the arena)

    def read(tid):
        if tid in tables:
            return tables[tid]
        t = tensors[tid]
        rows = slice(t["row"], t["row"] + (1 << len(t["axes"])))
        assert (owner[rows] == tid).all(), f"result {tid} was overwritten before it was read"
        return arena[rows]

    levels = {}
    for st in info["buckets"]:
        levels.setdefault(st["level"], []).append(st)
    for L in sorted(levels):
        pending = []
        for st in levels[L]:
            summed = st["vars"]
            kg = st["kg"]
            out_axes = st["out_axes"]
            r = len(out_axes)
            o = np.arange(1 << r)
            bit_of = {ax: (o >> j) & 1 for j, ax in enumerate(out_axes)}
            sig = np.zeros(B, dtype=np.int64)
            for i, q in enumerate(st["sig_q"]):
                sig |= xb(q) << i
            acc = np.zeros((1 << r, B), dtype=np.complex128)
            G = bucket_table(st, gate_vals)
            g = np.zeros(1 << r, dtype=np.int64)
            for j, gv in enumerate(st["gvars"]):
                g |= bit_of[gv] << j
            for w in range(1 << len(summed)):
                val = {var: (w >> i) & 1 for i, var in enumerate(summed)}
                term = np.array(G[(g << kg) | w][:, sig])
                for tid in st["in_tensors"]:
                    T = read(tid)
                    idx = np.zeros(1 << r, dtype=np.int64)
                    for a, ax in enumerate(tensors[tid]["axes"]):
                        idx |= (val[ax] if ax in val else bit_of[ax]) << a
                    term *= T[idx]
                acc += term
            if st.get("table_leaf", 0):
                tables[st["out_tensor"]] = acc
                continue
            pending.append((st["out_tensor"], acc))
        for tid, acc in pending:
            t = tensors[tid]
            # the device writes every reserved row (rows beyond 2^rank repeat the first ones)
            rows = np.arange(t["row"], t["row"] + t["alloc_rows"])
            assert t["row"] + t["alloc_rows"] <= info["arena_rows"]
            for rr in rows:
                prev = owner[rr]
                assert prev < 0 or prev == tid or tensors[prev]["used"] < L, \
                    f"level {L} overwrites result {prev} still in use"
            arena[rows] = np.tile(acc, (len(rows) // len(acc), 1))
            owner[rows] = tid
    amp = np.ones(B, dtype=np.complex128)
    for f in info["phase"]:
        amp = amp * _eval(f, lambda src, bit: xb(bit) if src == TS_SIG else np.zeros(B, dtype=np.int64), gate_vals)
    for tid in info["finals"]:
        amp = amp * read(tid)[0]
    n_open = info.get("n_open", 0)
    if n_open == 0:
        return amp
    # a set of amplitudes per bitstring: output bit i <-> open qubit i; the result over the open
    # qubits' variables has one axis per output bit outside zero_mask, in order
    zm = info["zero_mask"]
    out = np.zeros((B, 1 << n_open), dtype=np.complex128)
    R = read(info["open_tensor"]) if info["open_tensor"] >= 0 else None
    for o in range(1 << n_open):
        if o & zm:
            continue
        row, j = 0, 0
        for i in range(n_open):
            if (zm >> i) & 1:
                continue
            row |= ((o >> i) & 1) << j
            j += 1
        out[:, o] = amp * (R[row] if R is not None else 1.0)
    return out
