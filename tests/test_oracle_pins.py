"""Pins of the CPU oracle against values and identities fixed by the paper and
by mathematics (not against the oracle itself).

Each test names the passage it rests on.  A plausible slip in the oracle
(a wrong gate-table entry, a transposed 2x2, a dropped gate, a wrong sign in
the CZ, a wrong bit order, a wrong adjoint) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.gates import gate_matrix
from paper_1712_05384_amd import circuits as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EULER_GAMMA = 0.5772156649015329


def test_app_d_amplitudes_and_tables():
    """App. D: <00|C|00> = 1/2; H and CZ tables; tau1, tau2 intermediate tables."""
    g = json.load(open(os.path.join(GOLDEN, "app_d.json")))
    gates = np.array(g["gates"])
    for x, (re, im) in g["amplitudes"].items():
        a = oracle.sv_amplitudes(2, gates, None, [int(x)])[0]
        assert abs(a - complex(re, im)) < 1e-14
        assert abs(oracle.path_sum_amplitude(2, gates, None, int(x)) - complex(re, im)) < 1e-14
    # tau1(b0, b1) = psi_H(0,b0) psi_CZ(b0,b1) psi_H(b0,0) psi_H(0,b1) psi_H(b1,0)
    h = gate_matrix(0, -1, None)
    tau1 = np.array([[h[0, a] * (-1) ** (a * b) * h[a, 0] * h[0, b] * h[b, 0] for b in (0, 1)]
                     for a in (0, 1)])
    assert np.allclose(tau1, np.array(g["tau1"]), atol=1e-15)
    assert np.allclose(tau1.sum(axis=1), np.array(g["tau2"]), atol=1e-15)


def test_gate_tables_against_paper():
    """H table (App. D), T = diag(1, e^{i pi/4}) (Sec. II), unitarity of all four."""
    r2 = 1 / np.sqrt(2)
    assert np.allclose(gate_matrix(0, -1, None), [[r2, r2], [r2, -r2]], atol=0)
    assert np.allclose(gate_matrix(1, -1, None), np.diag([1, np.exp(1j * np.pi / 4)]), atol=0)
    for k in range(4):
        m = gate_matrix(k, -1, None)
        assert np.allclose(m.conj().T @ m, np.eye(2), atol=1e-15)
    # X^1/2 and Y^1/2 are pi/2 rotations: squared they give X and Y up to a phase
    x2 = gate_matrix(2, -1, None) @ gate_matrix(2, -1, None)
    y2 = gate_matrix(3, -1, None) @ gate_matrix(3, -1, None)
    assert np.allclose(x2, -1j * np.array([[0, 1], [1, 0]]), atol=1e-15)
    assert np.allclose(y2, -1j * np.array([[0, -1j], [1j, 0]]), atol=1e-15)


def _rand_small(rows, cols, depth, seed):
    return C.random_grid_circuit(rows, cols, depth, seed)


@pytest.mark.parametrize("rows,cols,depth,seed", [(1, 2, 6, 1), (2, 2, 8, 2), (2, 3, 7, 3),
                                                  (1, 3, 9, 4), (3, 1, 9, 5)])
def test_ising_phase_form_matches_state_vector(rows, cols, depth, seed):
    """App. F, Eqs. (path1), (phX), (phT), (phCZ): the phase-class sum equals the
    amplitude (with the constant -i per X^1/2 of the RX(pi/2) reading).  This
    pins the relative phases of X^1/2, Y^1/2, T and CZ in the oracle's tables."""
    c = _rand_small(rows, cols, depth, seed)
    n = c.n
    psi = oracle.sv_state(n, c.gates, None)
    for x in range(2 ** n):
        assert abs(oracle.ising_amplitude(n, c.gates, x) - psi[x]) < 1e-13


@pytest.mark.parametrize("rows,cols,depth,seed", [(2, 2, 10, 11), (2, 3, 8, 12), (3, 2, 8, 13)])
def test_path_sum_matches_state_vector(rows, cols, depth, seed):
    """Eq. (psi_x) summed exhaustively over all worldline variables equals the
    state-vector amplitude of Eq. (fpath)."""
    c = _rand_small(rows, cols, depth, seed)
    n = c.n
    psi = oracle.sv_state(n, c.gates, None)
    for x in range(2 ** n):
        assert abs(oracle.path_sum_amplitude(n, c.gates, None, x) - psi[x]) < 1e-14


def test_path_sum_parameterised_gates():
    """Eq. (psi_x) with general 2x2 factors (the parameterised family)."""
    c = C.parameterised_circuit(2, 2, 6, 21)
    psi = oracle.sv_state(c.n, c.gates, c.gate_vals)
    for x in range(2 ** c.n):
        assert abs(oracle.path_sum_amplitude(c.n, c.gates, c.gate_vals, x) - psi[x]) < 1e-14


def test_hand_applied_single_qubit():
    """Closed forms: H T H |0> has <0| = (1 + e^{i pi/4})/2 and <1| = (1 - e^{i pi/4})/2;
    the bit order is bit q = qubit q."""
    g = np.array([(0, 0, 0, -1, -1), (1, 1, 0, -1, -1), (0, 2, 0, -1, -1)])
    w = np.exp(1j * np.pi / 4)
    psi = oracle.sv_state(1, g, None)
    assert abs(psi[0] - (1 + w) / 2) < 1e-15 and abs(psi[1] - (1 - w) / 2) < 1e-15
    # H on qubit 1 only of three: amplitude 1/sqrt2 on index 0 and 2
    g3 = np.array([(0, 0, 1, -1, -1)])
    psi3 = oracle.sv_state(3, g3, None)
    assert np.allclose(psi3, [2 ** -0.5, 0, 2 ** -0.5, 0, 0, 0, 0, 0], atol=1e-15)
    # CZ phase lands on index 3 (= both qubits 0 and 1 set)
    gcz = np.array([(0, 0, 0, -1, -1), (0, 0, 1, -1, -1), (4, 1, 0, 1, -1)])
    assert np.allclose(oracle.sv_state(2, gcz, None), [0.5, 0.5, 0.5, -0.5], atol=1e-15)


def test_full_unitary_is_unitary():
    """U^dagger U = I for a 6-qubit random circuit: columns obtained by
    preparing each basis input with X gates (a U slot) before the circuit."""
    c = _rand_small(2, 3, 10, 31)
    n = c.n
    xgate = np.array([[[0, 1], [1, 0]]], dtype=np.complex128)
    cols = []
    for inp in range(2 ** n):
        pre = [(5, -1, q, -1, 0) for q in range(n) if (inp >> q) & 1]
        g = np.array(pre + [tuple(r) for r in c.gates], dtype=np.int64).reshape(-1, 5)
        cols.append(oracle.sv_state(n, g, xgate))
    u = np.array(cols).T
    assert np.allclose(u.conj().T @ u, np.eye(2 ** n), atol=1e-13)


@pytest.mark.parametrize("name", ["c1_4x4_d16"])
def test_norm_and_total_probability(name):
    c, _ = C.workload(name)
    psi = oracle.sv_state(c.n, c.gates, None)
    assert abs(np.sum(np.abs(psi) ** 2) - 1) < 1e-13


def test_porter_thomas_moments_deep_circuit():
    """Sec. II and App. B: for deep random circuits N p follows the exponential
    (Porter-Thomas) law: E[Np] = 1, E[(Np)^2] = 2, E[log Np] = -gamma,
    E[Np log Np] = 1 - gamma, entropy = log N - (1 - gamma) = log N - 0.4228."""
    c = C.random_grid_circuit(4, 4, 40, 7)
    N = 2 ** c.n
    p = np.abs(oracle.sv_state(c.n, c.gates, None)) ** 2
    Np = N * p
    assert abs(Np.mean() - 1) < 1e-10
    assert abs((Np ** 2).mean() - 2 * N / (N + 1)) < 0.1 * 2
    assert abs(np.log(Np).mean() + EULER_GAMMA) < 0.05
    assert abs((Np * np.log(Np)).mean() - (1 - EULER_GAMMA)) < 0.05
    entropy = -(p * np.log(p)).sum()
    assert abs(entropy - (np.log(N) - 0.4228)) < 0.05


def test_clifford_variant_probabilities_are_dyadic():
    """App. F (end): without T gates the path phases are multiples of pi/2 and
    the circuit is Clifford; the output distribution of a stabilizer state is
    uniform on an affine subspace, so every p is 0 or 2^-k."""
    c = C.clifford_variant(C.random_grid_circuit(3, 4, 14, 41))
    p = np.abs(oracle.sv_state(c.n, c.gates, c.gate_vals)) ** 2
    nz = p[p > 1e-12]
    k = np.log2(1 / nz)
    assert np.allclose(k, np.round(k), atol=1e-9)
    assert abs(nz.sum() - 1) < 1e-12
    assert len(set(np.round(k).astype(int))) == 1


def _loss(c, bits, vals):
    a = oracle.sv_amplitudes(c.n, c.gates, vals, bits)
    return float(np.sum(np.log(np.abs(a) ** 2)))


def test_gradient_finite_differences():
    """Central finite differences on Re and Im of gate entries match the
    adjoint-state gradient of L = sum log p (the estimator of Eq. (cee))."""
    c = C.parameterised_circuit(2, 3, 8, 51)
    bits = C.random_bitstrings(c.n, 16, 51)
    _, grad = oracle.sv_log_prob_gradient(c.n, c.gates, c.gate_vals, bits)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(24):
        s, a, b = rng.integers(0, c.n_slots), rng.integers(0, 2), rng.integers(0, 2)
        for part, unit in (("re", 1.0), ("im", 1j)):
            vp = c.gate_vals.copy(); vp[s, a, b] += h * unit
            vm = c.gate_vals.copy(); vm[s, a, b] -= h * unit
            fd = (_loss(c, bits, vp) - _loss(c, bits, vm)) / (2 * h)
            an = grad[s, a, b].real if part == "re" else grad[s, a, b].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (s, a, b, part, fd, an)


def _shared_and_diagonal_slot_circuit(seed):
    """A random circuit whose T gates become diagonal value-slot gates (kind UD,
    only the diagonal of the slot is read) and whose non-diagonal gates become
    general value-slot gates (kind U), with two UD gates reading one slot and two
    U gates reading one slot."""
    base = C.random_grid_circuit(2, 3, 10, seed)
    gates = base.gates.copy()
    rng = np.random.default_rng(seed)
    vals = []
    first_ud = first_u = -1
    for i in range(len(gates)):
        kind = gates[i, 0]
        if kind == C.CZ:
            continue
        if kind == C.T:
            gates[i, 0] = C.UD
            if first_ud >= 0 and (gates[:i, 4] == first_ud).sum() == 1:
                gates[i, 4] = first_ud          # the second UD gate reuses the first one's slot
                continue
            gates[i, 4] = len(vals)
            if first_ud < 0:
                first_ud = len(vals)
            # a full 2x2 value: the off-diagonal entries are never read by a UD gate
            vals.append(np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 2))) + 0.3 * np.array([[0, 1], [1, 0]]))
        else:
            gates[i, 0] = C.U
            if first_u >= 0 and (gates[:i, 4] == first_u).sum() == 1:
                gates[i, 4] = first_u           # the second U gate reuses the first one's slot
                continue
            gates[i, 4] = len(vals)
            if first_u < 0:
                first_u = len(vals)
            z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
            q, _ = np.linalg.qr(z)
            vals.append(q)
    c = C.Circuit(base.rows, base.cols, gates, np.array(vals, dtype=np.complex128), base.name + "_slots")
    return c, first_ud, first_u


def test_gradient_finite_differences_diagonal_and_shared_slots():
    """Finite differences of L = sum log p through the state vector alone pin the
    two slot rules of the gradient: a slot read by two gates gets the sum of both
    gates' gradients (perturbing the slot moves both), and a diagonal slot gate
    reads only the diagonal, so its off-diagonal entries have gradient 0 (their
    perturbation leaves L unchanged).  Appendix B, Eq. (cee) gives the loss."""
    c, s_ud, s_u = _shared_and_diagonal_slot_circuit(52)
    assert s_ud >= 0 and s_u >= 0
    assert (c.gates[:, 4] == s_ud).sum() == 2 and (c.gates[:, 4] == s_u).sum() == 2
    bits = C.random_bitstrings(c.n, 12, 52)
    _, grad = oracle.sv_log_prob_gradient(c.n, c.gates, c.gate_vals, bits)
    h = 1e-6
    ud_slots = {int(r[4]) for r in c.gates if r[0] == C.UD}
    for s in range(c.n_slots):
        for a in range(2):
            for b in range(2):
                for part, unit in (("re", 1.0), ("im", 1j)):
                    vp = c.gate_vals.copy(); vp[s, a, b] += h * unit
                    vm = c.gate_vals.copy(); vm[s, a, b] -= h * unit
                    fd = (_loss(c, bits, vp) - _loss(c, bits, vm)) / (2 * h)
                    an = grad[s, a, b].real if part == "re" else grad[s, a, b].imag
                    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (s, a, b, part, fd, an)
                    if s in ud_slots and a != b:
                        assert fd == 0.0 and an == 0.0
    # the shared slots' gradients are not those of either gate alone
    _, per_gate = oracle.sv_vjp(c.n, c.gates, c.gate_vals, bits,
                                2.0 / np.conj(oracle.sv_amplitudes(c.n, c.gates, c.gate_vals, bits)))
    two = np.flatnonzero(c.gates[:, 4] == s_u)
    assert np.abs(grad[s_u] - per_gate[two[0]]).max() > 1e-3
    assert np.abs(grad[s_u] - per_gate[two[1]]).max() > 1e-3


def test_gradient_scale_identity():
    """A is linear in each gate matrix, so L(lambda U_g) = L + 2m log|lambda| and
    sum_ab U_g[a,b] conj(G_g[a,b]) = 2m exactly, for every gate."""
    c = C.parameterised_circuit(3, 3, 10, 61)
    m = 32
    bits = C.random_bitstrings(c.n, m, 61)
    _, grad = oracle.sv_log_prob_gradient(c.n, c.gates, c.gate_vals, bits)
    ident = np.einsum("sab,sab->s", c.gate_vals, grad.conj())
    assert np.allclose(ident, 2 * m, rtol=1e-10, atol=0)


def test_environment_reconstructs_amplitude():
    """Per bitstring, sum_ab U_g[a,b] E_g[a,b] = A_x for every gate g (linearity)."""
    c = C.parameterised_circuit(2, 3, 8, 71)
    bits = C.random_bitstrings(c.n, 1, 71)
    amps, per_gate = oracle.sv_vjp(c.n, c.gates, c.gate_vals, bits, np.ones(1, dtype=complex))
    for i, row in enumerate(c.gates):
        if row[0] == C.CZ:
            continue
        u = c.gate_vals[row[4]]
        assert abs(np.sum(u * per_gate[i].conj()) - amps[0]) < 1e-13


def test_cycle0_input_column_is_zero():
    """The input of a cycle-0 gate is |0>, so its environment has E[:,1] = 0
    (to rounding: the oracle reaches that state by uncomputing with inverses)."""
    c = C.parameterised_circuit(2, 2, 6, 81)
    bits = C.random_bitstrings(c.n, 4, 81)
    _, per_gate = oracle.sv_vjp(c.n, c.gates, c.gate_vals, bits, np.ones(4, dtype=complex))
    for i, row in enumerate(c.gates):
        if row[1] == 0:
            assert np.abs(per_gate[i][:, 1]).max() < 1e-14


@pytest.mark.parametrize("rows,cols,depth,seed", [(3, 3, 12, 91), (4, 4, 16, 92), (3, 5, 20, 93)])
def test_bucket_elimination_matches_state_vector(rows, cols, depth, seed):
    """App. A bucket elimination (own min-degree order) equals the state vector."""
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, 6, seed)
    a = oracle.bucket_amplitudes(c.n, c.gates, None, bits)
    b = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(a - b).max() < 1e-14
    cp = C.parameterised_circuit(3, 3, 8, seed)
    a = oracle.bucket_amplitudes(cp.n, cp.gates, cp.gate_vals, bits % (1 << cp.n))
    b = oracle.sv_amplitudes(cp.n, cp.gates, cp.gate_vals, bits % (1 << cp.n))
    assert np.abs(a - b).max() < 1e-14


def test_bucket_elimination_app_d():
    g = json.load(open(os.path.join(GOLDEN, "app_d.json")))
    for x, (re, im) in g["amplitudes"].items():
        assert abs(oracle.bucket_amplitude(2, np.array(g["gates"]), None, int(x)) - complex(re, im)) < 1e-15
