"""CPU interpreter of a plan's step program (test helper, complex128).

It executes the planner's output -- factor programs, axis layouts, variant
sources -- with the semantics the HIP kernels implement, so planner logic can
be checked against the oracle without a GPU.  It is neither the oracle nor a
fallback of the product path: it only runs inside tests.
"""
import numpy as np

from oracle.gates import gate_matrix

GOP_PROJECT, GOP_MAT, GOP_DIAG, GOP_CZ, GOP_END = range(5)
SRC_ZERO, SRC_K, SRC_V, SRC_N, SRC_SIG, SRC_INT = range(6)


# matrix index -> gate kind of the library's fixed matrices (H, T, X^1/2, Y^1/2, their inverses, X, Y, Z);
# index 10 + s is value slot s
_FIXED_KIND = (0, 1, 2, 3, 7, 8, 9, 10, 11, 12)


def _mat(idx, gate_vals):
    if idx < len(_FIXED_KIND):
        return gate_matrix(_FIXED_KIND[idx], -1, None)
    return np.asarray(gate_vals[idx - len(_FIXED_KIND)], dtype=np.complex128).reshape(2, 2)


def build_g(step, gate_vals):
    vb, kb, nb, sb = step["vb"], step["kb"], step["nb"], step["sb"]
    tot = 1 << (vb + kb + nb + sb)
    e = np.arange(tot)
    sig = e & ((1 << sb) - 1)
    n = (e >> sb) & ((1 << nb) - 1)
    k = (e >> (sb + nb)) & ((1 << kb) - 1)
    v = e >> (sb + nb + kb)
    s0 = np.ones(tot, dtype=np.complex128)
    s1 = np.zeros(tot, dtype=np.complex128)
    res = np.zeros(tot, dtype=np.complex128)

    def val(src, bit):
        return {SRC_K: (k >> bit) & 1, SRC_V: (v >> bit) & 1, SRC_N: (n >> bit) & 1,
                SRC_SIG: (sig >> bit) & 1}.get(src, np.zeros(tot, dtype=np.int64))

    for typ, src, bit, mat in step["ops"]:
        x = val(src, bit)
        if typ == GOP_PROJECT:
            s0 = np.where(x == 1, 0, s0)
            s1 = np.where(x == 0, 0, s1)
        elif typ == GOP_MAT:
            m = _mat(mat, gate_vals)
            s0, s1 = m[0, 0] * s0 + m[0, 1] * s1, m[1, 0] * s0 + m[1, 1] * s1
        elif typ == GOP_DIAG:
            m = _mat(mat, gate_vals)
            s0, s1 = m[0, 0] * s0, m[1, 1] * s1
        elif typ == GOP_CZ:
            s1 = np.where(x == 1, -s1, s1)
        else:
            res = np.where(x == 1, s1, s0)
    return res.reshape(1 << vb, 1 << kb, 1 << nb, 1 << sb)


def run_plan(info, gate_vals, bits):
    """Executes a detail-1 plan description for uint64 bitstrings; returns
    complex128 [B, 2^n_open]."""
    bits = np.asarray(bits, dtype=np.uint64)
    B = len(bits)
    B_pad = (B + 63) // 64 * 64
    n_sl = info["n_sliced"]
    B_eff = B_pad << n_sl
    be = np.arange(B_eff)
    slice_idx = be // B_pad
    bidx = be % B_pad
    x = np.zeros(B_eff, dtype=np.uint64)
    x[bidx < B] = bits[bidx[bidx < B]]
    F = np.ones((1, B_eff), dtype=np.complex128)
    for st in info["steps"]:
        sig = np.zeros(B_eff, dtype=np.int64)
        for i, src in enumerate(st["sig_src"]):
            if src >= 0:
                bit = ((x >> np.uint64(src)) & np.uint64(1)).astype(np.int64)
            else:
                bit = (slice_idx >> (-src - 1)) & 1
            sig |= bit << i
        G = build_g(st, gate_vals)
        kb, nb = st["kb"], st["nb"]
        row_bits = st["r_in"] - kb
        rows = np.arange(1 << row_bits)
        inrow = rows.copy()
        for p in st["kpos"]:
            inrow = ((inrow >> p) << (p + 1)) | (inrow & ((1 << p) - 1))
        v = np.zeros_like(rows)
        for i, p in enumerate(st["vpos"]):
            v |= ((rows >> p) & 1) << i
        koff = np.zeros(1 << kb, dtype=np.int64)
        for kk in range(1 << kb):
            for i, p in enumerate(st["kpos"]):
                koff[kk] |= ((kk >> i) & 1) << p
        if st["input_is_one"]:
            A = np.zeros((len(rows), 1 << kb, B_eff), dtype=np.complex128)
            A[:, 0, :] = 1
        else:
            A = F[inrow[:, None] + koff[None, :], :]          # [rows, K, B]
        Gs = G[v][:, :, :, sig]                                # [rows, K, N, B]
        C = np.einsum("rkb,rknb->rnb", A, Gs)
        F = C.transpose(1, 0, 2).reshape((1 << nb) * len(rows), B_eff)
    n_open = info["n_open"]
    out = np.zeros((B, 1 << n_open), dtype=np.complex128)
    for o in range(1 << n_open):
        pos = 0
        for i, p in enumerate(info["final_pos"]):
            pos |= ((o >> i) & 1) << p
        acc = np.zeros(B_pad, dtype=np.complex128)
        for s in range(1 << n_sl):
            acc += F[pos, s * B_pad:(s + 1) * B_pad]
        out[:, o] = acc[:B]
    return out
