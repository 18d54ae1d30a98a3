"""Host planner tests (no GPU): graphical model of App. D, step-program
semantics checked against the oracle through a CPU interpreter, slicing,
open qubits, error handling and the exported C-ABI symbols."""
import ctypes
import itertools
import os
import re

import numpy as np
import pytest

import oracle
from paper_1712_05384_amd import circuits as C
from paper_1712_05384_amd import _native as N
import paper_1712_05384_amd as Q
from plan_interp import run_plan, build_g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_are_exported():
    """Every function include/qgm.h declares is exported by libqgm.so."""
    hdr = open(os.path.join(ROOT, "include", "qgm.h")).read()
    declared = set(re.findall(r"^\s*(?:qgm_status|void|const char\*)\s+(qgm_\w+)\s*\(", hdr, re.M))
    assert declared == set(N.EXPORTED)
    L = N.lib()
    for name in declared:
        assert getattr(L, name) is not None


def test_app_d_graph_and_tables():
    """App. D: six variables b_j^k (two chains of three joined by the CZ edge),
    the frontier after the first worldline holds one variable (the reduced
    graph is a 2-clique, treewidth 2), and the first step's operand, for
    output bit x_0 = 0, times the factors left on b_1^1 (psi_H(0,b) psi_H(b,0),
    1/2 each) is the table tau2 = (1/2, 0)."""
    d = C.example_app_d()
    info = Q.plan(d).info(1)
    assert info["n_vars"] == 6 and info["n_cz"] == 1 and info["n_steps"] == 2
    assert info["max_rank"] == 1
    st0 = info["steps"][0]
    assert st0["kb"] == 0 and st0["nb"] == 1 and st0["sb"] == 1
    g = build_g(st0, None)                       # [v, k, n, sigma]
    h = oracle.gate_matrix(0, -1, None)
    tau2 = g[0, 0, :, 0] * np.array([h[0, b] * h[b, 0] for b in (0, 1)])
    assert np.allclose(tau2, [0.5, 0.0], atol=1e-15)
    got = run_plan(info, None, np.arange(4, dtype=np.uint64))[:, 0]
    assert np.allclose(got, [0.5, 0.5, 0.5, -0.5], atol=1e-15)


def _check(c, bits, open_qubits=(), **opts):
    info = Q.plan(c, open_qubits, **opts).info(1)
    got = run_plan(info, c.gate_vals, bits)
    n = c.n
    for o in range(1 << len(open_qubits)):
        xb = bits.copy()
        for i, q in enumerate(open_qubits):
            xb = (xb & ~np.uint64(1 << q)) | np.uint64(((o >> i) & 1) << q)
        ref = oracle.sv_amplitudes(n, c.gates, c.gate_vals, xb)
        assert np.abs(got[:, o] - ref).max() < 1e-12, (c.name, open_qubits, o)
    return info


@pytest.mark.parametrize("rows,cols,depth,seed", [(1, 1, 5, 1), (1, 3, 8, 2), (2, 2, 1, 3), (2, 2, 2, 4),
                                                  (3, 3, 12, 5), (2, 4, 16, 6), (4, 2, 16, 7), (3, 4, 10, 8)])
def test_step_program_matches_oracle(rows, cols, depth, seed):
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, 70, seed)
    _check(c, bits)


def test_parameterised_and_clifford_circuits():
    c = C.parameterised_circuit(3, 3, 9, 11)
    _check(c, C.random_bitstrings(c.n, 20, 11))
    k = C.clifford_variant(C.random_grid_circuit(3, 3, 10, 12))
    _check(k, C.random_bitstrings(k.n, 20, 12))


@pytest.mark.parametrize("open_qubits", [(0,), (4,), (8, 0), (3, 5, 1), tuple(range(9))])
def test_open_qubits(open_qubits):
    """Leaving output deltas out of Eq. (psi_x) gives sets of amplitudes."""
    c = C.random_grid_circuit(3, 3, 10, 21)
    _check(c, C.random_bitstrings(c.n, 5, 21), open_qubits)


@pytest.mark.parametrize("nsl", [1, 2, 3])
def test_slicing_is_exact(nsl):
    """Summing over all assignments of the sliced variables gives the unsliced result."""
    c = C.random_grid_circuit(3, 4, 14, 31)
    info = _check(c, C.random_bitstrings(c.n, 8, 31), min_sliced_vars=nsl)
    assert info["n_sliced"] == nsl


def test_max_rank_slicing_reduces_rank():
    c = C.random_grid_circuit(4, 4, 16, 41)
    base = Q.plan(c).info(0)["max_rank"]
    info = _check(c, C.random_bitstrings(c.n, 4, 41), max_rank=base - 2)
    assert info["max_rank"] <= base - 2 and info["n_sliced"] >= 2


def test_qubit_without_gates_and_open_untouched():
    """A qubit with no non-diagonal gate keeps b^0 = b^{d} = 0: amplitude 0 when x_q = 1."""
    g = np.array([(C.H, 0, 0, -1, -1), (C.CZ, 1, 0, 1, -1), (C.T, 2, 1, -1, -1), (C.H, 3, 0, -1, -1)])
    c = C.Circuit(1, 3, g)
    _check(c, np.arange(8, dtype=np.uint64))
    _check(c, np.arange(8, dtype=np.uint64), (1,))
    _check(c, np.arange(8, dtype=np.uint64), (2, 0))


def test_workload_plan_sizes():
    """Planner statistics for the benchmark workloads (printed in the plan JSON)."""
    for name in ("c1_4x4_d16", "c2_5x5_d25", "c3_5x6_d30"):
        c, _ = C.workload(name)
        info = Q.plan(c).info(0)
        assert info["n_steps"] == c.n
        assert info["max_rank"] <= 24
        assert sum(s["flops_per_b"] for s in info["steps"]) == info["flops_per_amp"]


@pytest.mark.parametrize("bad", [
    dict(gates=[(C.CZ, 1, 0, 0, -1)]),
    dict(gates=[(C.H, 0, 9, -1, -1)]),
    dict(gates=[(C.H, 0, 0, -1, -1), (C.T, 0, 0, -1, -1)]),
    dict(gates=[(C.U, 0, 0, -1, 3)]),
    dict(gates=[(13, 0, 0, -1, -1)]),
    dict(gates=[(C.H, -1, 0, -1, -1)]),
    dict(gates=[(C.H, 0, 0, 1, -1)]),
])
def test_invalid_circuits_rejected(bad):
    c = C.Circuit(2, 2, np.array(bad["gates"], dtype=np.int32))
    with pytest.raises(N.QgmError) as e:
        Q.plan(c)
    assert e.value.status == N.QGM_E_INVALID


def test_invalid_open_qubits_rejected():
    c = C.random_grid_circuit(2, 2, 4, 1)
    for op in ((0, 0), (4,), (-1,)):
        with pytest.raises(N.QgmError) as e:
            Q.plan(c, op)
        assert e.value.status == N.QGM_E_INVALID


def test_null_arguments_and_small_workspace():
    L = N.lib()
    h = ctypes.c_void_p()
    assert L.qgm_plan(None, None, 0, None, ctypes.byref(h)) == N.QGM_E_INVALID
    assert b"NULL" in L.qgm_last_error()
    c = C.random_grid_circuit(2, 2, 4, 1)
    p = Q.plan(c)
    assert p.workspace_bytes(64) > 0
    # too small a workspace is refused before any device call
    st = L.qgm_amplitudes(p.handle, None, ctypes.c_void_p(256), 64, ctypes.c_void_p(256),
                          ctypes.c_void_p(256), 16, None)
    assert st == N.QGM_E_OOM
    # a circuit that reads gate_vals refuses NULL
    pc = Q.plan(C.parameterised_circuit(2, 2, 4, 1))
    st = L.qgm_amplitudes(pc.handle, None, ctypes.c_void_p(256), 64, ctypes.c_void_p(256),
                          ctypes.c_void_p(256), 1 << 40, None)
    assert st == N.QGM_E_INVALID


def test_kernel_classification():
    """Policy 0 (and 1) keep every step on the vector-ALU kernel with one row per thread;
    policy 2 puts every step the matrix-core kernel supports on it; policy 3 pairs rows
    on dense steps (|K| + |N| >= 8 bits, K of 2^3..2^5)."""
    c, _ = C.workload("c2_5x5_d25")
    for pol in (0, 1):
        assert all(s["kernel"] == "valu" for s in Q.plan(c, kernel_policy=pol).info(0)["steps"])
    for s in Q.plan(c, kernel_policy=3).info(0)["steps"]:
        assert (s["kernel"] == "valu_pair") == (3 <= s["kb"] <= 5 and s["kb"] + s["nb"] >= 8)
    forced = Q.plan(c, kernel_policy=2).info(0)["steps"]
    for s in forced:
        ok = 3 <= s["kb"] <= 5 and 3 <= s["nb"] <= 5 and s["r_in"] - s["kb"] - s["vb"] >= 4 and s["sb"] <= 4
        assert (s["kernel"] == "mfma_f32") == (ok and not s["input_is_one"])
    assert any(s["kernel"] == "mfma_f32" for s in forced)


# --- bucket-elimination plans (ordering 1) -------------------------------------------------

from tree_interp import run_tree_plan  # noqa: E402


def _check_tree(c, bits, ref=None, **opts):
    info = Q.plan(c, ordering=1, **opts).info(1)
    got = run_tree_plan(info, c.gate_vals, bits)
    if ref is None:
        ref = oracle.sv_amplitudes(c.n, c.gates, c.gate_vals, bits)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, 2 ** (-c.n / 2) * 1e3), c.name
    return info


@pytest.mark.parametrize("rows,cols,depth,seed", [(1, 1, 5, 1), (1, 3, 8, 2), (2, 2, 1, 3), (2, 2, 2, 4),
                                                  (3, 3, 12, 5), (2, 4, 16, 6), (4, 2, 16, 7), (3, 4, 10, 8)])
def test_tree_plan_matches_oracle(rows, cols, depth, seed):
    """Bucket elimination of App. A along the planner's greedy order, run by the
    CPU interpreter with arena-overlap checks, equals the state vector."""
    c = C.random_grid_circuit(rows, cols, depth, seed)
    _check_tree(c, C.random_bitstrings(c.n, 40, seed))


def test_tree_plan_parameterised_clifford_and_bare_qubit():
    c = C.parameterised_circuit(3, 3, 9, 11)
    _check_tree(c, C.random_bitstrings(c.n, 20, 11))
    k = C.clifford_variant(C.random_grid_circuit(3, 3, 10, 12))
    _check_tree(k, C.random_bitstrings(k.n, 20, 12))
    g = np.array([(C.H, 0, 0, -1, -1), (C.CZ, 1, 0, 1, -1), (C.T, 2, 1, -1, -1), (C.H, 3, 0, -1, -1)])
    info = _check_tree(C.Circuit(1, 3, g), np.arange(8, dtype=np.uint64))
    assert any(f[0] == 3 for f in info["phase"])   # the x_q = 0 delta of the bare worldline


@pytest.mark.parametrize("name", ["c1_4x4_d16", "c2_5x5_d25", "c4_5x5_d20_U"])
def test_tree_plan_workloads_against_bucket_oracle(name):
    c, bits = C.workload(name)
    bits = bits[:6]
    ref = oracle.bucket_amplitudes(c.n, c.gates, c.gate_vals, bits)
    info = _check_tree(c, bits, ref)
    assert info["n_levels"] <= info["n_buckets"]


def test_tree_orders_beat_vertical():
    """Greedy treewidth orders need far less traffic than the vertical order
    (Sec. IV.B: heuristic orders beat the vertical one)."""
    for name, factor in (("c2_5x5_d25", 10), ("c3_5x6_d30", 8), ("c5_6x6_d24", 30)):
        c, _ = C.workload(name)
        t = Q.plan(c, ordering=1).info(0)
        v = Q.plan(c).info(0)
        assert t["bytes_per_amp"] * factor < v["bytes_per_amp"], (name, t["bytes_per_amp"], v["bytes_per_amp"])
        assert t["max_rank"] < v["max_rank"]


def test_tree_plan_is_deterministic_and_consistent():
    c, _ = C.workload("c2_5x5_d25")
    a = Q.plan(c, ordering=1).info(1)
    b = Q.plan(c, ordering=1).info(1)
    assert a == b
    summed = [v for s in a["buckets"] for v in s["vars"]]
    summed += [v for s in a["buckets"] for g in s["groups"] for v in g["vars"]]   # absorbed buckets
    assert sorted(a["order"]) == sorted(summed)
    assert a["absorbed_buckets"] == sum(len(s["groups"]) - 1 for s in a["buckets"]) > 0
    assert a["n_free"] == len(a["order"])
    assert abs(sum(s["bytes_per_b"] for s in a["buckets"]) - a["bytes_per_amp"]) < 1e-6 * a["bytes_per_amp"]
    # every result is read by exactly one later bucket or by the final product; a composed leaf table
    # (built with the plan) reads leaf tables only
    readers = [0] * len(a["tensors"])
    for s in a["buckets"]:
        for t in s["in_tensors"]:
            readers[t] += 1
            if s["level"] >= 0:
                assert a["tensors"][t]["made"] < s["level"]
            else:
                assert s["composed"] and a["tensors"][t]["made"] == -1
    for t in a["finals"]:
        readers[t] += 1
    assert readers == [1] * len(a["tensors"])


def test_tree_plan_refusals():
    """What the bucket path refuses: the persistent launch with open qubits or
    slicing, BF16x3 precision, too many sliced variables; out-of-range options
    are QGM_E_INVALID."""
    c = C.random_grid_circuit(3, 3, 8, 1)
    for oq, kw, status in (((0,), dict(tree_exec=2), N.QGM_E_UNSUPPORTED),
                           ((), dict(tree_exec=2, min_sliced_vars=1), N.QGM_E_UNSUPPORTED),
                           ((), dict(precision=N.QGM_PREC_BF16X3), N.QGM_E_UNSUPPORTED),
                           ((), dict(min_sliced_vars=25), N.QGM_E_INVALID),
                           ((), dict(precision=2), N.QGM_E_INVALID)):
        with pytest.raises(N.QgmError) as e:
            Q.plan(c, oq, ordering=1, **kw)
        assert e.value.status == status, kw
    with pytest.raises(N.QgmError) as e:
        Q.plan(c, ordering=2)
    assert e.value.status == N.QGM_E_INVALID
    # the adjoint is supported: its workspace holds every result and its adjoint
    p = Q.plan(c, ordering=1)
    assert p.backward_workspace_bytes(64) > 2 * p.workspace_bytes(64) - 4096


@pytest.mark.parametrize("rows,cols,depth,seed", [(3, 3, 12, 5), (2, 4, 16, 6), (3, 4, 10, 8)])
def test_tree_plan_without_chain_merge(rows, cols, depth, seed):
    """One variable per bucket (no merged chains) gives the same amplitudes."""
    c = C.random_grid_circuit(rows, cols, depth, seed)
    info = _check_tree(c, C.random_bitstrings(c.n, 20, seed), chain_merge=False)
    assert all(len(s["vars"]) == 1 for s in info["buckets"])


def test_chain_merge_shortens_the_tree():
    """Merged chains sum up to three variables per bucket: fewer levels, fewer
    buckets and less traffic, the same elimination order (the first order by
    symbolic cost, which merging does not change)."""
    for name in ("c2_5x5_d25", "c3_5x6_d30"):
        c, _ = C.workload(name)
        a = Q.plan(c, ordering=1, chain_merge=False, order_finalists=1).info(0)
        b = Q.plan(c, ordering=1, order_finalists=1).info(1)
        assert b["order"] == a["order"]
        assert b["n_levels"] < a["n_levels"] and b["n_buckets"] < a["n_buckets"]
        assert b["bytes_per_amp"] < a["bytes_per_amp"]
        assert max(len(s["vars"]) for s in b["buckets"]) <= 3
        for s in b["buckets"]:
            assert s["kg"] == len(s["vars"])


def _issued_score(info):
    return sum(b["issued_bytes_per_b"] for b in info["buckets"]) + 8192 * info["level_launches"]


def test_order_finalists_scored_by_issued_bytes():
    """The planner builds the first candidate orders in full and keeps the one
    whose kernels issue the fewest bytes per bitstring (plus 8 KiB per launch):
    never worse than the first order by symbolic cost (order_finalists = 1),
    strictly better on the 5x5 depth-25 and depth-24 circuits, the same
    amplitudes through the interpreter, and the option checked."""
    for name, better in (("c2_5x5_d25", True), ("c5_5x5_d24", True), ("c5_4x5_d20", False), ("c3_5x6_d30", False)):
        c, _ = C.workload(name)
        one = Q.plan(c, ordering=1, order_finalists=1).info(1)
        dflt = Q.plan(c, ordering=1).info(1)
        assert one["orders_built"] == 1 and 1 < dflt["orders_built"] <= 64 and dflt["orders_tried"] == 2 * 65
        assert _issued_score(dflt) <= _issued_score(one)
        if better:
            assert _issued_score(dflt) < 0.9 * _issued_score(one)
            assert dflt["order"] != one["order"]
    for seed, (rows, cols, depth) in enumerate([(3, 3, 12), (2, 4, 16), (3, 4, 10)]):
        c = C.random_grid_circuit(rows, cols, depth, 40 + seed)
        bits = C.random_bitstrings(c.n, 24, seed)
        a = _check_tree(c, bits, order_finalists=1)
        b = _check_tree(c, bits, order_finalists=64)
        assert _issued_score(b) <= _issued_score(a)
        assert b["orders_built"] <= b["orders_tried"]
    c = C.random_grid_circuit(2, 2, 4, 1)
    for bad in (-1, 65):
        with pytest.raises(Exception):
            Q.plan(c, ordering=1, order_finalists=bad)
    for bad in (-1, 1025):
        with pytest.raises(Exception):
            Q.plan(c, ordering=1, order_restarts=bad)
    for bad in (-1, 64):
        with pytest.raises(Exception):
            Q.plan(c, ordering=1, order_pick=bad)
    with pytest.raises(Exception):   # beyond the finalists that build
        Q.plan(c, ordering=1, order_finalists=2, order_pick=5)
    # order_pick keeps the finalist of that rank: scores rise with the rank, rank 0 is the default plan, and
    # a lower-ranked plan still gives the state vector's amplitudes through the interpreter
    c, _ = C.workload("c2_5x5_d25")
    picks = [Q.plan(c, ordering=1, order_pick=k).info(1) for k in range(4)]
    assert all(a["order_score"] <= b["order_score"] for a, b in zip(picks, picks[1:]))
    assert picks[0]["order"] == Q.plan(c, ordering=1).info(1)["order"] and picks[1]["order"] != picks[0]["order"]
    assert abs(picks[0]["order_score"] - _issued_score(picks[0])) < 1e-6 * picks[0]["order_score"]
    c = C.random_grid_circuit(3, 4, 12, 44)
    bits = C.random_bitstrings(c.n, 16, 44)
    _check_tree(c, bits, order_pick=1)
    c, _ = C.workload("c3_5x6_d30")
    again = [Q.plan(c, ordering=1).info(1) for _ in range(2)]   # seeded restarts, stable ranking: one plan
    assert again[0]["order"] == again[1]["order"] and again[0]["order_score"] == again[1]["order_score"]
    few = Q.plan(c, ordering=1, order_restarts=4).info(0)
    assert few["orders_tried"] == 2 * 5 and few["orders_built"] == 10
    assert _issued_score(Q.plan(c, ordering=1).info(1)) <= _issued_score(Q.plan(c, ordering=1, order_restarts=4).info(1))


def test_tree_exec_modes_and_persistent_workspace():
    """tree_exec 2 keeps every result at its own rows and adds completion
    flags; 1 runs one launch per level; 3 (and 0, auto, when the plan fits)
    keeps every result in LDS, so it needs no arena (only the per-call factor
    tables of a circuit with gate values)."""
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(4, 4, 16, 2)
    per = Q.plan(c, ordering=1, tree_exec=2)
    lev = Q.plan(c, ordering=1, tree_exec=1)
    lds = Q.plan(c, ordering=1, tree_exec=3)
    auto = Q.plan(c, ordering=1)
    assert per.workspace_bytes(1024) > lev.workspace_bytes(1024)
    assert auto.workspace_bytes(1024) == lds.workspace_bytes(1024) == 0
    assert per.workspace_bytes(64) > lev.workspace_bytes(64)
    cp = C.parameterised_circuit(3, 3, 10, 2)
    assert 0 < Q.plan(cp, ordering=1, tree_exec=3).workspace_bytes(1024) < Q.plan(cp, ordering=1, tree_exec=1).workspace_bytes(1024)
    with pytest.raises(Exception):
        Q.plan(c, ordering=1, tree_exec=4)


def _oracle_open(c, bits, open_qubits):
    cols = []
    for o in range(1 << len(open_qubits)):
        xb = bits.copy()
        for i, q in enumerate(open_qubits):
            xb = (xb & ~np.uint64(1 << q)) | np.uint64(((o >> i) & 1) << q)
        cols.append(oracle.sv_amplitudes(c.n, c.gates, c.gate_vals, xb))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("rows,cols,depth,seed,open_qubits", [(2, 2, 6, 1, (0,)), (3, 3, 10, 2, (4, 0)),
                                                             (3, 4, 12, 3, (11, 3, 7)), (2, 3, 8, 4, (0, 1, 2, 3, 4, 5)),
                                                             (4, 3, 14, 5, tuple(range(12)))])
def test_tree_plan_open_qubits(rows, cols, depth, seed, open_qubits):
    """Sets of amplitudes (Sec. III.A): the open qubits' last variables are never
    summed; one bucket over them (a chain beyond 8 inputs) gives every completion."""
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, 12, seed)
    info = Q.plan(c, open_qubits, ordering=1).info(1)
    assert info["n_open"] == len(open_qubits) and info["tail_levels"] == 0
    got = run_tree_plan(info, c.gate_vals, bits)
    ref = _oracle_open(c, bits, open_qubits)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() < 1e-12


def test_tree_plan_open_qubit_without_non_diagonal_gates():
    """An open qubit whose worldline has only diagonal gates ends in 0: its
    output bit set gives amplitude 0 (zero_mask)."""
    g = np.array([(C.H, 0, 0, -1, -1), (C.CZ, 1, 0, 1, -1), (C.T, 2, 1, -1, -1), (C.H, 3, 0, -1, -1),
                  (C.H, 0, 2, -1, -1), (C.CZ, 4, 1, 2, -1), (C.XH, 5, 2, -1, -1)])
    c = C.Circuit(1, 3, g)
    bits = np.arange(8, dtype=np.uint64)
    for oq in ((1,), (1, 0), (2, 1)):
        info = Q.plan(c, oq, ordering=1).info(1)
        assert info["zero_mask"] == (1 << oq.index(1))
        got = run_tree_plan(info, c.gate_vals, bits)
        assert np.abs(got - _oracle_open(c, bits, oq)).max() < 1e-12


def test_tree_plan_open_bucket_chain():
    """More than 8 results end on the open qubits' variables: the product over
    them runs as a chain of buckets (1x18: H, CZ on 9 disjoint pairs, X^1/2;
    one open qubit per pair)."""
    n = 18
    g = [(C.H, 0, q, -1, -1) for q in range(n)] + [(C.CZ, 1, 2 * i, 2 * i + 1, -1) for i in range(9)] + \
        [(C.XH, 2, q, -1, -1) for q in range(n)]
    c = C.Circuit(1, n, np.array(g))
    oq = tuple(range(0, n, 2))
    info = Q.plan(c, oq, ordering=1).info(1)
    assert sum(1 for b in info["buckets"] if b["kg"] == 0) >= 2
    bits = C.random_bitstrings(n, 3, 5)
    got = run_tree_plan(info, c.gate_vals, bits)
    psi = oracle.sv_state(n, c.gates, None)
    ref = np.zeros_like(got)
    for o in range(1 << len(oq)):
        x = bits.copy()
        for i, q in enumerate(oq):
            x = (x & ~np.uint64(1 << q)) | np.uint64(((o >> i) & 1) << q)
        ref[:, o] = psi[x.astype(np.int64)]
    assert np.abs(got - ref).max() < 1e-12


def test_tree_plan_leaf_tables():
    """Buckets without inputs of a circuit without gate values become tables
    over (result index, output bits), built with the plan, with no level of
    their own, and so do buckets whose inputs are all such tables when their
    result and output bits are few (composed leaves: their output bits are
    their own, then their inputs' others); a circuit with gate values keeps
    them as buckets."""
    c, bits = C.workload("c2_5x5_d25")
    info = Q.plan(c, ordering=1).info(1)
    leaves = [b for b in info["buckets"] if b["table_leaf"]]
    assert info["table_leaves"] == len(leaves) > 0
    assert all(b["level"] == -1 for b in leaves)
    tens = info["tensors"]
    maker = {b["out_tensor"]: b for b in info["buckets"]}
    composed = [b for b in leaves if b["composed"]]
    assert composed and all(b["n_in"] == 0 for b in leaves if not b["composed"])
    for b in composed:
        assert all(maker[t]["table_leaf"] for t in b["in_tensors"])
        sig = set(b["sig_q"])
        assert all(set(maker[t]["sig_q"]) <= sig for t in b["in_tensors"])
        assert b["r_out"] + len(sig) <= 18 and len(sig) <= 10
    off = Q.plan(c, ordering=1, compose=False).info(1)
    assert not any(b["composed"] for b in off["buckets"]) and off["n_levels"] > info["n_levels"]
    assert min(b["level"] for b in info["buckets"] if not b["table_leaf"]) == 0
    got = run_tree_plan(info, None, bits[:16])
    assert np.abs(got - oracle.sv_amplitudes(c.n, c.gates, None, bits[:16])).max() < 1e-12
    c4, _ = C.workload("c4_5x5_d20_U")
    assert Q.plan(c4, ordering=1).info(0)["table_leaves"] == 0


def test_tail_fits_the_tail_kernels_lds_arrays():
    """The last levels run in one work-group per bitstring group with their task
    records, factor tables and results in LDS: at most 32 task records, 64
    result rows, 2048 factor-table entries and 16 levels."""
    import paper_1712_05384_amd as Q
    circs = [C.random_grid_circuit(r, c, d, s) for (r, c, d, s) in
             [(3, 4, 16, 2), (4, 4, 16, 4), (4, 5, 20, 1), (5, 5, 25, 201), (2, 6, 18, 3)]]
    for c in circs:
        info = Q.plan(c, ordering=1).info(1)
        tail = [bk for bk in info["buckets"] if bk["level"] >= info["tail_start"]]
        rows = sum(2 ** max(bk["r_out"], 3) for bk in tail)
        tasks = sum(max(1, 2 ** bk["r_out"] // bk["unit_rows"]) for bk in tail)
        gent = sum(2 ** (len(bk["gvars"]) + bk["kg"] + bk["sb"]) for bk in tail)
        assert rows == info["tail_lds_rows"] <= 64
        assert tasks <= 32 and gent <= 2048 and info["tail_levels"] <= 16


def test_tail_plan_with_many_phase_factors_closed_form():
    """60 qubits: a 3x4 block and H then T on the other 48 (each contributes
    <x|TH|0> = (1, e^{i pi/4})[x] / sqrt 2); the plan, run by the interpreter."""
    import paper_1712_05384_amd as Q
    from tree_interp import run_tree_plan
    blk = C.random_grid_circuit(3, 4, 12, 3)
    n = 60
    g = [tuple(int(v) for v in r) for r in blk.gates] + [(C.H, 0, q, -1, -1) for q in range(12, n)] + \
        [(C.T, 1, q, -1, -1) for q in range(12, n)]
    c = C.Circuit(1, n, np.array(g, dtype=np.int32))
    info = Q.plan(c, ordering=1, order_restarts=16, order_finalists=1).info(1)   # this plan has tail levels
    assert info["n_phase"] > 64 and info["tail_levels"] > 0
    bits = C.random_bitstrings(n, 12, 11)
    ref = oracle.sv_state(12, blk.gates, None)[(bits & np.uint64(0xFFF)).astype(np.int64)]
    for q in range(12, n):
        ref = ref * np.where(((bits >> np.uint64(q)) & np.uint64(1)).astype(bool), np.exp(1j * np.pi / 4), 1.0) / np.sqrt(2)
    assert np.abs(run_tree_plan(info, None, bits) - ref).max() < 1e-12 * 2 ** (-n / 2)


def test_tile_buckets_planned_and_interpreted():
    """Buckets with two bits carried by one input only and one by another only
    become tile units (8 result rows, those three bits lowest; with three and
    two such bits and at least 1024 rows, 32-row units whose five bits come
    lowest); the plan computes the same amplitudes with and without them."""
    import paper_1712_05384_amd as Q
    from tree_interp import run_tree_plan
    c, _ = C.workload("c3_5x6_d30")
    info = Q.plan(c, ordering=1).info(1)
    tiles = [bk for bk in info["buckets"] if bk["tile"]]
    assert len(tiles) >= 3
    tensors = info["tensors"]

    def alone(u, t, ins):   # result bit u carried by input t and by no other input
        return u in tensors[ins[t]]["axes"] and all(u not in tensors[o]["axes"] for k, o in enumerate(ins) if k != t)

    for bk in tiles:
        ins, out = bk["in_tensors"], bk["out_axes"]
        big = bk["tile"] >= 3
        assert bk["n_in"] == bk["tile"] + 1 - 2 * big and bk["kg"] >= 2 and bk["unit_rows"] == (32 if big else 8)
        # inputs in the order A (unit bits 0, 1, and 3 for the 32-row tile), B (bit 2, and 4), C (none)
        assert alone(out[0], 0, ins) and alone(out[1], 0, ins) and alone(out[2], 1, ins)
        if big:
            assert alone(out[3], 0, ins) and alone(out[4], 1, ins) and bk["r_out"] >= 10
        assert not set(out[:5 if big else 3]) & set(bk["gvars"])
    assert any(bk["tile"] >= 3 for bk in tiles)
    assert not any(bk["tile"] for bk in Q.plan(c, ordering=1, tile=False).info(1)["buckets"])
    c2 = C.random_grid_circuit(4, 4, 16, 3)
    bits = C.random_bitstrings(c2.n, 8, 3)
    ref = oracle.sv_amplitudes(c2.n, c2.gates, None, bits)
    for tile in (True, False):
        got = run_tree_plan(Q.plan(c2, ordering=1, tile=tile).info(1), None, bits)
        assert np.abs(got - ref).max() < 1e-12


def test_quad_tiles_planned():
    """Two-input 32-row tiles with two more bits carried by input B alone take
    them as result bits 5 and 6 (quad tiles: tasks 4m .. 4m + 3 read the same
    rows of A and the same table entries); a level's quad tasks come first, a
    multiple of 4, and a level with quad and other tasks is two launches."""
    import paper_1712_05384_amd as Q
    c, _ = C.workload("c5_6x7_d27")
    info = Q.plan(c, ordering=1, tree_exec=1).info(1)
    tensors, bks = info["tensors"], info["buckets"]
    quads = [bk for bk in bks if bk["quad"]]
    assert len(quads) >= 4 and max(bk["r_out"] for bk in quads) >= 17
    for bk in quads:
        ins, out = bk["in_tensors"], bk["out_axes"]
        assert bk["tile"] == 3 and bk["n_in"] == 2 and bk["r_out"] >= 10
        for u in out[5:7]:
            assert u in tensors[ins[1]]["axes"] and u not in tensors[ins[0]]["axes"] and u not in bk["gvars"]
    mixed = 0
    for L, nq in enumerate(info["level_quad"]):
        inl = [bk for bk in bks if bk["level"] == L and not bk["table_leaf"]]
        want = sum(1 << (bk["r_out"] - 5) for bk in inl if bk["quad"])
        assert nq == want and nq % 4 == 0
        if nq and any(not bk["quad"] for bk in inl):
            mixed += 1
    assert mixed >= 1 and info["kernel_launches"] == info["level_launches"] + mixed
    # no quad tile where the second input has fewer than four bits alone: the 5x5 depth-25 plan has none
    c2, _ = C.workload("c2_5x5_d25")
    assert not any(bk["quad"] for bk in Q.plan(c2, ordering=1, tree_exec=1).info(1)["buckets"])


def test_tile_in_tail_and_option_validation():
    """4x4 depth 16, the first order's plan: a tile bucket runs in the tail (tile
    units reading and writing the tail's LDS); an invalid no_tile value is rejected."""
    import paper_1712_05384_amd as Q
    c, _ = C.workload("c1_4x4_d16")
    info = Q.plan(c, ordering=1, order_restarts=16, order_finalists=1, compose=False).info(1)
    assert any(bk["tile"] and bk["level"] >= info["tail_start"] for bk in info["buckets"])
    cs, keep = Q.api._circuit_struct(c.rows, c.cols, c.gates, 0)
    opts = N.QgmPlanOpts()
    L = N.lib()
    L.qgm_default_opts(ctypes.byref(opts))
    opts.ordering = 1
    opts.no_tile = 2
    h = ctypes.c_void_p()
    assert L.qgm_plan(ctypes.byref(cs), None, 0, ctypes.byref(opts), ctypes.byref(h)) == N.QGM_E_INVALID


def test_bucket_workspace_uses_power_of_two_pitch():
    """The bucket arena's row pitch is the padded batch rounded up to a power of
    two: a batch of 130 (3 groups of 64) takes the workspace of a batch of 256."""
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(3, 4, 12, 5)
    p = Q.plan(c, ordering=1, tree_exec=1)
    assert p.workspace_bytes(130) == p.workspace_bytes(256) > p.workspace_bytes(128)
    assert p.workspace_bytes(64) == p.workspace_bytes(1)


@pytest.mark.parametrize("rows,cols,depth,seed", [(3, 4, 18, 3), (3, 4, 20, 4), (4, 4, 16, 3), (4, 4, 20, 2),
                                                  (4, 4, 24, 1), (5, 5, 25, 201)])
def test_tile_plans_random_circuits_interpreted(rows, cols, depth, seed):
    """Plans with tile units (inputs reordered, tile bits lowest; the 5x5 depth-25
    plan of the first order by symbolic cost among 16 restarts per criterion has a
    three-input tile; without composed leaf tables, which take the small tile
    buckets of these circuits) and without,
    for the chosen order and the first one, with and without composed leaves,
    run by the interpreter, against the state vector."""
    import paper_1712_05384_amd as Q
    from tree_interp import run_tree_plan
    c = C.random_grid_circuit(rows, cols, depth, seed)
    kinds = set()
    for fin in (0, 1):
        kinds |= {bk["tile"] for bk in Q.plan(c, ordering=1, order_restarts=16 * fin, order_finalists=fin,
                                              compose=False).info(1)["buckets"]}
    assert kinds & {1, 2, 3, 4}
    if (rows, cols, depth, seed) == (5, 5, 25, 201):
        assert 2 in kinds
    bits = C.random_bitstrings(c.n, 4, seed)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    for fin in (0, 1):
        for tile in (True, False):
            for compose in (True, False):
                got = run_tree_plan(Q.plan(c, ordering=1, tile=tile, order_restarts=16 * fin, order_finalists=fin,
                                           compose=compose).info(1), None, bits)
                assert np.abs(got - ref).max() < 1e-12


# --- the LDS-resident program (tree_exec 3) -------------------------------------------------


@pytest.mark.parametrize("rows,cols,depth,seed,B", [(1, 1, 3, 1, 3), (2, 2, 1, 2, 2), (3, 3, 10, 1, 4),
                                                    (4, 4, 16, 3, 4), (4, 5, 20, 2, 3), (1, 5, 12, 3, 3)])
def test_lds_program_interpreted_matches_oracle(rows, cols, depth, seed, B):
    """The program one work-group runs per bitstring (tables copied at the output
    bits, 64-row jobs at 16-bit LDS offsets, one barrier per level), executed on
    the CPU with its bounds and same-level read/write checks, equals the FP64
    state vector."""
    from lds_interp import run_lds_program
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, B, seed)
    info = Q.plan(c, ordering=1).info(2)
    assert info["lds_ok"] == 1
    got = run_lds_program(info, None, bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(got - ref).max() < 1e-12 * 2 ** (-c.n / 2)


def test_lds_program_gate_values_and_benchmark_plan():
    """Gate values (per-call tables, no leaf tables) and the 5x5 depth-25
    benchmark plan (27 buckets, 11 levels) through the LDS interpreter."""
    from lds_interp import run_lds_program
    cp = C.parameterised_circuit(3, 4, 12, 3)
    bits = C.random_bitstrings(cp.n, 3, 3)
    info = Q.plan(cp, ordering=1).info(2)
    got = run_lds_program(info, cp.gate_vals, bits)
    assert np.abs(got - oracle.sv_amplitudes(cp.n, cp.gates, cp.gate_vals, bits)).max() < 1e-12 * 2 ** (-cp.n / 2)
    c, bits = C.workload("c2_5x5_d25")
    info = Q.plan(c, ordering=1).info(2)
    assert info["lds_ok"] == 1 and info["lds_entries"] * 8 <= 62 * 1024
    got = run_lds_program(info, None, bits[:2])
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits[:2])
    assert np.abs(got - ref).max() < 1e-12 * 2 ** (-c.n / 2)
    # the LDS bytes the bench's roofline uses: per kept row 2^k (inputs + table) reads and one write, plus the
    # copied table entries, counted from the exported jobs
    L = info["lds"]
    want = 8 * len(L["entries"]) + sum(j["lanes"] * (1 << j["rl"]) * 8 * ((1 << j["k"]) * (j["nin"] + 1) + 1)
                                       for j in L["jobs"])
    assert info["lds_bytes_per_amp"] == want


def test_lds_program_limits():
    """Open qubits and plans whose results exceed the LDS stay on the level
    launches; asking for the LDS launch there is QGM_E_UNSUPPORTED."""
    c = C.random_grid_circuit(3, 3, 10, 1)
    info = Q.plan(c, (0, 4), ordering=1).info(0)
    assert info["lds_ok"] == 0 and "open" in info["lds_why"]
    big, _ = C.workload("c3_5x6_d30")
    assert Q.plan(big, ordering=1).info(0)["lds_ok"] == 0
    with pytest.raises(N.QgmError) as ei:
        Q.plan(big, ordering=1, tree_exec=3)
    assert ei.value.status == N.QGM_E_UNSUPPORTED


@pytest.mark.parametrize("wl", ["c2_5x5_d25", "c5_5x5_d24", "c5_6x6_d24", "c5_4x5_d20"])
def test_lds_jobs_balanced_over_waves(wl):
    """The kernel gives wave w the jobs w, w + W, ... of a level; the planner
    orders each level's jobs so that the heaviest wave (cost: loads per lane
    plus a fixed part) stays within the list-scheduling bound of the mean load
    plus one job, and every level still covers each bucket's rows once."""
    c, _ = C.workload(wl)
    info = Q.plan(c, ordering=1).info(2)
    L = info["lds"]
    W = info["lds_threads"] // 64
    off = L["level_job_off"]
    cost = lambda j: 16 + (1 << j["rl"]) * (j["nin"] + 1) * (1 << j["k"])
    for lv in range(len(off) - 1):
        jobs = L["jobs"][off[lv]:off[lv + 1]]
        load = [0] * W
        for i, j in enumerate(jobs):
            load[i % W] += cost(j)
        if jobs:
            assert max(load) <= sum(load) / W + max(cost(j) for j in jobs)
        if W < len(jobs) <= 8:   # small levels: the best split the assignment allows, by brute force
            n, full, extra = len(jobs), len(jobs) // W, len(jobs) % W
            cap = [full + (w < extra) for w in range(W)]
            best = None
            for asg in itertools.product(range(W), repeat=n):
                if all(asg.count(w) == cap[w] for w in range(W)):
                    m = max(sum(cost(jobs[i]) for i in range(n) if asg[i] == w) for w in range(W))
                    best = m if best is None else min(best, m)
            assert max(load) == best, (wl, lv, load, best)
        rows = {}
        for j in jobs:   # rows per bucket: 64 << rl per job (fewer lanes for buckets under 64 rows)
            rows[j["bucket"]] = rows.get(j["bucket"], 0) + j["lanes"] * (1 << j["rl"])
        for b, n in rows.items():
            assert n == 1 << info["buckets"][b]["r_out"], (wl, lv, b)


# ---- slicing of bucket plans (Sec. V outlook: space-time tradeoffs) ----------

@pytest.mark.parametrize("rows,cols,depth,seed,msv", [(3, 4, 12, 7, 1), (3, 4, 12, 7, 3), (4, 4, 16, 2, 2),
                                                      (2, 5, 14, 9, 4)])
def test_tree_slicing_interpreted_matches_oracle(rows, cols, depth, seed, msv):
    """A sliced bucket plan fixes each sliced variable by a bit above the
    qubits of a batch column's word; the sum over its 2^s slices, run through
    the CPU interpreter of the exported plan, equals the state-vector
    amplitudes, and so does its LDS program."""
    from lds_interp import run_lds_program
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, 6, seed)
    p = Q.plan(c, ordering=1, min_sliced_vars=msv)
    info = p.info(2)
    assert info["n_sliced"] == msv == len(info["sliced_qubit"]) and info["slice_chunk_bits"] == msv
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(run_tree_plan(info, None, bits) - ref).max() < 1e-12 * 2 ** (-c.n / 2)
    if info["lds_ok"]:
        assert np.abs(run_lds_program(info, None, bits[:2]) - ref[:2]).max() < 1e-12 * 2 ** (-c.n / 2)
    # the slicing variables are gone from every result, and the sliced plan's largest result is no larger
    sl = set(zip(info["sliced_qubit"], info["sliced_k"]))
    assert info["max_rank"] <= Q.plan(c, ordering=1).info(0)["max_rank"]
    assert len(sl) == msv


def test_tree_slicing_gate_values_and_open_qubits():
    cp = C.parameterised_circuit(3, 4, 12, 3)
    bits = C.random_bitstrings(cp.n, 4, 3)
    info = Q.plan(cp, ordering=1, min_sliced_vars=2).info(2)
    ref = oracle.sv_amplitudes(cp.n, cp.gates, cp.gate_vals, bits)
    assert np.abs(run_tree_plan(info, cp.gate_vals, bits) - ref).max() < 1e-12 * 2 ** (-cp.n / 2)
    c = C.random_grid_circuit(3, 3, 10, 4)
    oq = (1, 5)
    info = Q.plan(c, oq, ordering=1, min_sliced_vars=2).info(2)
    assert info["n_sliced"] == 2
    got = run_tree_plan(info, None, C.random_bitstrings(c.n, 3, 4))
    for i, x in enumerate(C.random_bitstrings(c.n, 3, 4)):
        for o in range(4):
            y = int(x)
            for j, q in enumerate(oq):
                y = (y & ~(1 << q)) | (((o >> j) & 1) << q)
            want = oracle.sv_amplitudes(c.n, c.gates, None, np.array([y], dtype=np.uint64))[0]
            assert abs(got[i, o] - want) < 1e-12 * 2 ** (-c.n / 2)


def test_tree_mem_budget_and_max_rank():
    """mem_budget bounds the workspace of 64 bitstrings: the planner slices and
    then runs as many slices per chunk as fit; max_rank bounds every result;
    a budget that no slicing meets is QGM_E_OOM."""
    c, _ = C.workload("c3_5x6_d30")
    free = Q.plan(c, ordering=1)
    assert free.info(0)["n_sliced"] == 0
    budget = free.workspace_bytes(64) // 2
    p = Q.plan(c, ordering=1, mem_budget=budget, tree_exec=1)
    info = p.info(0)
    assert info["n_sliced"] >= 1 and p.workspace_bytes(64) <= budget
    assert info["slice_chunk_bits"] <= info["n_sliced"]
    # the same slices all at once take more memory than the budget allows
    p_all = Q.plan(c, ordering=1, min_sliced_vars=info["n_sliced"], tree_exec=1)
    if info["slice_chunk_bits"] < info["n_sliced"]:
        assert p_all.workspace_bytes(64) > budget
    r = Q.plan(c, ordering=1, max_rank=10).info(0)
    assert r["max_rank"] <= 10 and r["n_sliced"] >= 1
    # the LDS-resident launch of a circuit without gate values needs no workspace at all; the level
    # launches need their arena, which no slicing brings to one byte
    small = C.random_grid_circuit(2, 3, 8, 1)
    assert Q.plan(small, ordering=1, mem_budget=1).workspace_bytes(64) == 0
    with pytest.raises(N.QgmError) as e:
        Q.plan(small, ordering=1, mem_budget=1, tree_exec=1)
    assert e.value.status == N.QGM_E_OOM


def test_tree_headline_circuits_plan_with_slicing():
    """The 5x9 depth-40 and 7x8 depth-30 circuits (Abstract) plan on the bucket
    path: slicing brings every result under the kernels' rank limit, and a
    memory budget slices further."""
    for r, cc, d in ((5, 9, 40), (7, 8, 30)):
        c = C.random_grid_circuit(r, cc, d, 1)
        p = Q.plan(c, ordering=1)
        info = p.info(0)
        assert info["max_rank"] <= 28 and info["n"] + info["n_sliced"] <= 64
        b = Q.plan(c, ordering=1, mem_budget=2 << 30)
        assert b.workspace_bytes(64) <= 2 << 30 and b.info(0)["n_sliced"] > info["n_sliced"]


def test_precision_and_checkpoint_budget_ordering_0():
    """precision BF16X3 gives every supporting step the BF16x3 kernel (the same
    plan as kernel_policy 4); checkpoint_budget picks the checkpoint interval
    with the least recomputation that fits, at most ceil(sqrt(steps))."""
    c, _ = C.workload("c3_5x6_d30")
    a = Q.plan(c, precision=N.QGM_PREC_BF16X3, min_sliced_vars=2).info(0)
    b = Q.plan(c, kernel_policy=4, min_sliced_vars=2).info(0)
    ka = [s["kernel"] for s in a["steps"]]
    assert ka == [s["kernel"] for s in b["steps"]] and "mfma_bf16x3" in ka
    with pytest.raises(N.QgmError) as e:
        Q.plan(c, precision=N.QGM_PREC_BF16X3, kernel_policy=2)
    assert e.value.status == N.QGM_E_INVALID
    tiny = C.random_grid_circuit(2, 2, 4, 1)
    with pytest.raises(N.QgmError) as e:
        Q.plan(tiny, precision=N.QGM_PREC_BF16X3)
    assert e.value.status == N.QGM_E_UNSUPPORTED
    cp = C.parameterised_circuit(3, 3, 12, 2)
    info = Q.plan(cp).info(0)
    S, r = info["n_steps"], info["max_rank"]
    frame = (1 << r) * 64 * 8
    c_sqrt = int(np.ceil(np.sqrt(S)))
    assert Q.plan(cp).info(0)["checkpoint_every"] == 0
    assert Q.plan(cp, checkpoint_budget=(S - 1) * frame).info(0)["checkpoint_every"] == 1
    need_sqrt = ((S - 1) // c_sqrt + c_sqrt - 1) * frame
    ce = Q.plan(cp, checkpoint_budget=need_sqrt).info(0)["checkpoint_every"]
    assert 1 <= ce <= c_sqrt and ((S - 1) // ce + ce - 1) * frame <= need_sqrt
    with pytest.raises(N.QgmError) as e:
        Q.plan(cp, checkpoint_budget=need_sqrt - 1)
    assert e.value.status == N.QGM_E_OOM
    with pytest.raises(N.QgmError) as e:
        Q.plan(cp, ordering=1, checkpoint_budget=1024)
    assert e.value.status == N.QGM_E_OOM
