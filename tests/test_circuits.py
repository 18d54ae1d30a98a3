"""The seeded circuit generator follows the frozen reading of the layout rules
(Sec. II: CZ between nearest neighbours, never on neighbouring qubits at once;
single-qubit gates from {T, X^1/2, Y^1/2}; depth 1 = the Hadamard layer)."""
import numpy as np
import pytest

from paper_1712_05384_amd import circuits as C


def _neighbours(rows, cols, a, b):
    ra, ca = divmod(a, cols)
    rb, cb = divmod(b, cols)
    return abs(ra - rb) + abs(ca - cb) == 1


@pytest.mark.parametrize("rows,cols", [(4, 4), (5, 5), (5, 6), (6, 7)])
def test_patterns_cover_each_edge_once_and_never_touch(rows, cols):
    seen = {}
    for name in C.PATTERN_ORDER:
        edges = C.pattern_edges(rows, cols, name)
        qs = [q for e in edges for q in e]
        assert len(qs) == len(set(qs))
        for e in edges:
            assert _neighbours(rows, cols, *e)
            assert e not in seen
            seen[e] = name
        for i, (a, b) in enumerate(edges):
            for (c, d) in edges[i + 1:]:
                for u in (a, b):
                    for v in (c, d):
                        assert not _neighbours(rows, cols, u, v)
    n_edges = rows * (cols - 1) + (rows - 1) * cols
    assert len(seen) == n_edges


def test_single_qubit_rules():
    c = C.random_grid_circuit(5, 5, 25, 201)
    g = c.gates
    assert (g[g[:, 1] == 0][:, 0] == C.H).all() and (g[:, 1] == 0).sum() == 25
    last = {q: C.H for q in range(25)}
    for row in g[np.argsort(g[:, 1], kind="stable")]:
        kind, t, q0, q1, _ = row
        if kind in (C.T, C.XH, C.YH):
            if last[q0] == C.H:
                assert kind == C.T
            else:
                assert kind != last[q0]
            last[q0] = kind
    assert c.depth() == 25


def test_depth_one_is_hadamard_layer():
    c = C.random_grid_circuit(3, 3, 1, 0)
    assert len(c.gates) == 9 and (c.gates[:, 0] == C.H).all()


def test_seeded_determinism_and_bitstrings():
    a = C.random_grid_circuit(4, 5, 20, 501)
    b = C.random_grid_circuit(4, 5, 20, 501)
    assert np.array_equal(a.gates, b.gates)
    bits = C.random_bitstrings(20, 1024, 501)
    assert bits.dtype == np.uint64 and bits.max() < 2 ** 20
    assert np.array_equal(bits, C.random_bitstrings(20, 1024, 501))


def test_parameterised_gates_are_unitary():
    c = C.parameterised_circuit(3, 3, 8, 401)
    for m in c.gate_vals:
        assert np.allclose(m.conj().T @ m, np.eye(2), atol=1e-14)
        assert abs(np.linalg.det(m) - 1) < 1e-14
