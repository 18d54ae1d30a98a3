"""Expectation values <0|U^dag O U|0> of Pauli strings (Sec. III.B): oracle pins
(hand-computed values, Pauli algebra), the light-cone circuit checked on the
oracle's own state vector, and both planners' circuits run by the CPU plan
interpreters."""
import numpy as np
import pytest

import oracle
from oracle.observable import apply_pauli_string
import paper_1712_05384_amd as Q
from paper_1712_05384_amd import circuits as C
from plan_interp import run_plan
from tree_interp import run_tree_plan


def _circ(rows, cols, gates):
    return C.Circuit(rows, cols, np.array(gates, dtype=np.int32).reshape(-1, 5))


def test_oracle_expectation_by_hand():
    """|+> = H|0>: <X> = 1, <Z> = 0, <Y> = 0; RX(pi/2)|0> = (|0> - i|1>)/sqrt2: <Y> = -1, <Z> = 0;
    |00> after nothing but H on qubit 1: <Z_0> = 1, <Z_0 X_1> = 1."""
    c = _circ(1, 1, [(C.H, 0, 0, -1, -1)])
    assert np.isclose(oracle.expectation(1, c.gates, None, {0: "X"}), 1)
    assert np.isclose(oracle.expectation(1, c.gates, None, {0: "Z"}), 0)
    assert np.isclose(oracle.expectation(1, c.gates, None, {0: "Y"}), 0)
    c = _circ(1, 1, [(C.XH, 0, 0, -1, -1)])
    assert np.isclose(oracle.expectation(1, c.gates, None, {0: "Y"}), -1)
    assert np.isclose(oracle.expectation(1, c.gates, None, {0: "Z"}), 0)
    c = _circ(1, 2, [(C.H, 0, 1, -1, -1)])
    assert np.isclose(oracle.expectation(2, c.gates, None, {0: "Z"}), 1)
    assert np.isclose(oracle.expectation(2, c.gates, None, {0: "Z", 1: "X"}), 1)


def test_pauli_algebra_of_the_oracle():
    """XY = iZ on one qubit, and O^2 = 1 for every Pauli string."""
    rng = np.random.default_rng(1)
    psi = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    xy = apply_pauli_string(3, apply_pauli_string(3, psi, {1: "Y"}), {1: "X"})
    assert np.allclose(xy, 1j * apply_pauli_string(3, psi, {1: "Z"}))
    o = {0: "X", 2: "Y"}
    assert np.allclose(apply_pauli_string(3, apply_pauli_string(3, psi, o), o), psi)


@pytest.mark.parametrize("rows,cols,depth,seed,paulis", [(2, 2, 6, 1, {0: "Z"}), (3, 3, 10, 2, {4: "X"}),
                                                         (3, 3, 8, 3, {0: "Y", 8: "Z"}),
                                                         (2, 4, 12, 4, {1: "X", 2: "Y", 5: "Z"})])
def test_light_cone_circuit_on_the_state_vector(rows, cols, depth, seed, paulis):
    """The amplitude at 0 of U_cone, O, U_cone^dag (from the oracle's state vector
    of that circuit) equals <psi|O|psi>; the cone drops gates when it can."""
    c = C.random_grid_circuit(rows, cols, depth, seed)
    e = Q.expectation_circuit(c, paulis)
    ref = oracle.expectation(c.n, c.gates, None, paulis)
    got = oracle.sv_amplitudes(c.n, e.gates, None, np.zeros(1, dtype=np.uint64))[0]
    assert abs(got - ref) < 1e-12
    assert abs(ref.imag) < 1e-12
    assert len(e.gates) <= 2 * len(c.gates) + len(paulis)


@pytest.mark.parametrize("ordering", [0, 1])
def test_expectation_plans_on_the_cpu_interpreters(ordering):
    c = C.random_grid_circuit(3, 3, 10, 5)
    for paulis in ({4: "Z"}, {0: "X", 4: "Y"}, {2: "Z", 6: "Z"}):
        e = Q.expectation_circuit(c, paulis)
        info = Q.plan(e, ordering=ordering).info(1)
        run = run_tree_plan if ordering == 1 else run_plan
        got = run(info, None, np.zeros(1, dtype=np.uint64)).reshape(-1)[0]
        assert abs(got - oracle.expectation(c.n, c.gates, None, paulis)) < 1e-12


def test_expectation_circuit_errors():
    from paper_1712_05384_amd import _native as N
    c = C.random_grid_circuit(2, 2, 4, 1)
    for bad in ({9: "Z"}, {0: "H"}):
        with pytest.raises((N.QgmError, KeyError)):
            Q.expectation_circuit(c, bad)
    with pytest.raises(N.QgmError) as e:
        Q.expectation_circuit(C.parameterised_circuit(2, 2, 4, 1), {0: "Z"})
    assert e.value.status == N.QGM_E_UNSUPPORTED
