"""Non-diagonal two-qubit gates (the 4-clique of Sec. III.B): oracle pins (the
numpy state vector against the C one, Kronecker products, CZ and SWAP as
two-qubit gates) and the bucket planner's circuits run by its CPU interpreter."""
import numpy as np
import pytest

import oracle
from oracle.statevector import sv_state_numpy
import paper_1712_05384_amd as Q
from paper_1712_05384_amd import circuits as C
from paper_1712_05384_amd import _native as N
from tree_interp import run_tree_plan


def haar_2x2(rng):
    q, r = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def haar_4x4(rng):
    q, r = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def u2_slots(M):
    """The four value slots of a two-qubit gate: row r of M as a 2x2 block."""
    return [np.asarray(M[r], dtype=np.complex128).reshape(2, 2) for r in range(4)]


def brickwork(rows, cols, layers, seed):
    """H on every qubit, then layers of Haar two-qubit gates on alternating
    neighbour pairs with Haar single-qubit gates between them."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    gates, vals = [], []
    for q in range(n):
        gates.append((C.H, 0, q, -1, -1))
    cyc = 1
    for layer in range(layers):
        pairs = []
        for r in range(rows):
            for c in range(layer % 2, cols - 1, 2):
                pairs.append((r * cols + c, r * cols + c + 1))
        if layer % 3 == 2:
            pairs = [(r * cols + c, (r + 1) * cols + c) for c in range(cols) for r in range(layer % 2, rows - 1, 2)]
        for a, b in pairs:
            gates.append((C.U2, cyc, a, b, len(vals)))
            vals.extend(u2_slots(haar_4x4(rng)))
        cyc += 1
        for q in range(n):
            if rng.random() < 0.5:
                gates.append((C.U, cyc, q, -1, len(vals)))
                vals.append(haar_2x2(rng))
        cyc += 1
    return C.Circuit(rows, cols, np.array(gates, dtype=np.int32), np.array(vals), f"brick{rows}x{cols}_{layers}")


def test_numpy_state_vector_matches_the_c_oracle():
    for seed in range(3):
        c = C.random_grid_circuit(3, 3, 10, seed)
        assert np.abs(sv_state_numpy(c.n, c.gates, None) - oracle.sv_state(c.n, c.gates, None)).max() < 1e-13
    c = C.parameterised_circuit(3, 3, 8, 4)
    assert np.abs(sv_state_numpy(c.n, c.gates, c.gate_vals) - oracle.sv_state(c.n, c.gates, c.gate_vals)).max() < 1e-13


def test_two_qubit_gate_pins():
    rng = np.random.default_rng(1)
    A, B = haar_2x2(rng), haar_2x2(rng)
    base = [(C.H, 0, 0, -1, -1), (C.XH, 0, 1, -1, -1), (C.T, 1, 0, -1, -1)]
    # A (x) B as one two-qubit gate equals A on q0 and B on q1
    c2 = C.Circuit(1, 2, np.array(base + [(C.U2, 2, 0, 1, 0)], dtype=np.int32), np.array(u2_slots(np.kron(A, B))))
    c1 = C.Circuit(1, 2, np.array(base + [(C.U, 2, 0, -1, 0), (C.U, 2, 1, -1, 1)], dtype=np.int32), np.array([A, B]))
    assert np.abs(oracle.sv_state(2, c2.gates, c2.gate_vals) - oracle.sv_state(2, c1.gates, c1.gate_vals)).max() < 1e-13
    # diag(1, 1, 1, -1) as a two-qubit gate equals CZ
    cz = np.diag([1, 1, 1, -1]).astype(np.complex128)
    c3 = C.Circuit(1, 2, np.array(base + [(C.U2, 2, 0, 1, 0)], dtype=np.int32), np.array(u2_slots(cz)))
    c4 = C.Circuit(1, 2, np.array(base + [(C.CZ, 2, 0, 1, -1)], dtype=np.int32))
    assert np.abs(oracle.sv_state(2, c3.gates, c3.gate_vals) - oracle.sv_state(2, c4.gates, None)).max() < 1e-13
    # SWAP moves |1> from qubit 0 to qubit 1: index 2 (bit 1 set) gets amplitude 1
    swap = np.eye(4)[[0, 2, 1, 3]].astype(np.complex128)
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    c5 = C.Circuit(1, 2, np.array([(C.U, 0, 0, -1, 0), (C.U2, 1, 0, 1, 1)], dtype=np.int32),
                   np.array([X] + u2_slots(swap)))
    psi = oracle.sv_state(2, c5.gates, c5.gate_vals)
    assert np.allclose(psi, [0, 0, 1, 0])


@pytest.mark.parametrize("rows,cols,layers,seed", [(1, 2, 1, 1), (2, 2, 3, 2), (2, 3, 4, 3), (3, 3, 5, 4)])
def test_bucket_plan_with_two_qubit_gates(rows, cols, layers, seed):
    c = brickwork(rows, cols, layers, seed)
    bits = C.random_bitstrings(c.n, 16, seed)
    info = Q.plan(c, ordering=1).info(1)
    assert info["n_2q"] == int((c.gates[:, 0] == C.U2).sum())
    got = run_tree_plan(info, c.gate_vals, bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, c.gate_vals, bits)
    assert np.abs(got - ref).max() < 1e-12


def test_two_qubit_gates_need_ordering_1():
    c = brickwork(2, 2, 2, 5)
    with pytest.raises(N.QgmError) as e:
        Q.plan(c, ordering=0)
    assert e.value.status == N.QGM_E_UNSUPPORTED
    bad = C.Circuit(1, 2, np.array([(C.U2, 0, 0, 1, 2)], dtype=np.int32), np.zeros((4, 2, 2)))
    with pytest.raises(N.QgmError) as e:
        Q.plan(bad, ordering=1)
    assert e.value.status == N.QGM_E_INVALID
