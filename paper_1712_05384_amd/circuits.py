"""Seeded random grid circuits and bitstrings (input generators only).

This module draws the *inputs* of the amplitude computation: which gate sits
where in a 2D-lattice random circuit, the values of parameterised gates, and
the output bitstrings.  It holds none of the method's arithmetic (no gate
tables for the fixed kinds, no contraction), so both the HIP path and the
CPU oracle take their inputs from here without sharing any computation.

Circuit family (Sec. II of the paper, "Numerical results"): cycle 0 is a
Hadamard on every qubit; later cycles apply CZ gates between nearest
neighbours of the lattice, never on two neighbouring qubits at once, plus
single-qubit gates from {T, X^1/2, Y^1/2}.  The exact layout rules live in the
paper's cited companion work and are not given in the text, so this module
freezes one reading of them:

* qubit (r, c) has index q = r*cols + c;
* depth d means cycles 0..d-1 (depth 1 is the Hadamard layer alone, as the
  footnote to Fig. 1 says);
* cycle t >= 1 uses CZ pattern PATTERN_ORDER[(t-1) % 8] where
  H_a = {(r,c)-(r,c+1) : c = a + 2*(r%2) mod 4} and
  V_a = {(r,c)-(r+1,c) : r = a + 2*(c%2) mod 4};
* a single-qubit gate is placed on q at cycle t iff q was in a CZ at t-1 and
  is not in one at t; the first such gate after the Hadamard layer is T, the
  later ones are drawn uniformly from {T, X^1/2, Y^1/2} minus q's previous
  single-qubit gate (one rng.integers(0, 2) draw per non-forced gate, cycles
  ascending, then qubits ascending).
"""
from __future__ import annotations

import dataclasses
import numpy as np

# Gate kinds; the numbering is the C-ABI's (qgm_kind in include/qgm.h).
H, T, XH, YH, CZ, U, UD = 0, 1, 2, 3, 4, 5, 6
TDG, XHDG, YHDG, X, Y, Z = 7, 8, 9, 10, 11, 12   # inverses and Pauli operators (expectation values)
U2 = 13   # general two-qubit gate: rows of its 4x4 matrix in four consecutive value slots
KIND_NAMES = {H: "H", T: "T", XH: "X^1/2", YH: "Y^1/2", CZ: "CZ", U: "U", UD: "UD"}
DIAGONAL_KINDS = (T, CZ, UD)

PATTERN_ORDER = ("H0", "V0", "H2", "V2", "H1", "V1", "H3", "V3")


@dataclasses.dataclass
class Circuit:
    """A circuit on a rows x cols lattice.

    gates: int32 [n_gates, 5] with columns (kind, cycle, q0, q1, slot);
    q1 = -1 for single-qubit gates, slot = -1 unless the gate's value is
    read from gate_vals[slot] (kinds U and UD).
    gate_vals: complex128 [n_slots, 2, 2] or None.
    """

    rows: int
    cols: int
    gates: np.ndarray
    gate_vals: np.ndarray | None = None
    name: str = ""

    @property
    def n(self) -> int:
        return self.rows * self.cols

    @property
    def n_slots(self) -> int:
        return 0 if self.gate_vals is None else int(self.gate_vals.shape[0])

    def depth(self) -> int:
        return int(self.gates[:, 1].max()) + 1 if len(self.gates) else 0


def pattern_edges(rows: int, cols: int, name: str) -> list[tuple[int, int]]:
    """Edges (q0, q1) of one of the 8 CZ patterns, q0 < q1."""
    a = int(name[1])
    edges = []
    if name[0] == "H":
        for r in range(rows):
            for c in range(cols - 1):
                if c % 4 == (a + 2 * (r % 2)) % 4:
                    edges.append((r * cols + c, r * cols + c + 1))
    else:
        for r in range(rows - 1):
            for c in range(cols):
                if r % 4 == (a + 2 * (c % 2)) % 4:
                    edges.append((r * cols + c, (r + 1) * cols + c))
    return edges


def random_grid_circuit(rows: int, cols: int, depth: int, seed: int) -> Circuit:
    """The seeded random circuit of the family above (fixed-kind gates only)."""
    if rows < 1 or cols < 1 or depth < 1:
        raise ValueError("rows, cols and depth must be >= 1")
    n = rows * cols
    rng = np.random.default_rng(seed)
    gates: list[tuple[int, int, int, int, int]] = []
    for q in range(n):
        gates.append((H, 0, q, -1, -1))
    last_1q = [H] * n           # previous single-qubit gate on each qubit
    in_cz_prev = np.zeros(n, dtype=bool)
    for t in range(1, depth):
        edges = pattern_edges(rows, cols, PATTERN_ORDER[(t - 1) % 8])
        in_cz = np.zeros(n, dtype=bool)
        for q0, q1 in edges:
            in_cz[q0] = in_cz[q1] = True
        for q in range(n):
            if in_cz_prev[q] and not in_cz[q]:
                if last_1q[q] == H:
                    kind = T
                else:
                    choices = [k for k in (T, XH, YH) if k != last_1q[q]]
                    kind = choices[int(rng.integers(0, 2))]
                gates.append((kind, t, q, -1, -1))
                last_1q[q] = kind
        for q0, q1 in edges:
            gates.append((CZ, t, q0, q1, -1))
        in_cz_prev = in_cz
    g = np.array(gates, dtype=np.int32).reshape(-1, 5)
    return Circuit(rows, cols, g, None, name=f"{rows}x{cols}_d{depth}_s{seed}")


def parameterised_circuit(rows: int, cols: int, depth: int, seed: int) -> Circuit:
    """Same structure as random_grid_circuit, but every single-qubit gate
    (including the cycle-0 layer) becomes U = exp(-i theta n.sigma / 2) with
    theta ~ U(0, pi) and n uniform on the unit sphere, each in its own slot.
    The values are drawn from a generator seeded with seed + 7_000_000, in
    gate order, after the structure is fixed."""
    base = random_grid_circuit(rows, cols, depth, seed)
    gates = base.gates.copy()
    rng = np.random.default_rng(seed + 7_000_000)
    vals = []
    for i in range(len(gates)):
        if gates[i, 0] == CZ:
            continue
        theta = rng.uniform(0.0, np.pi)
        g = rng.standard_normal(3)
        nx, ny, nz = g / np.linalg.norm(g)
        c, s = np.cos(theta / 2), np.sin(theta / 2)
        # cos(theta/2) I - i sin(theta/2) (nx X + ny Y + nz Z)
        m = np.array([[c - 1j * s * nz, -1j * s * nx - s * ny],
                      [-1j * s * nx + s * ny, c + 1j * s * nz]], dtype=np.complex128)
        gates[i, 0] = U
        gates[i, 4] = len(vals)
        vals.append(m)
    return Circuit(rows, cols, gates, np.array(vals, dtype=np.complex128),
                   name=f"{rows}x{cols}_d{depth}_s{seed}_U")


def clifford_variant(c: Circuit) -> Circuit:
    """Replace every T by S = diag(1, i) through a UD slot.  S is diagonal, so
    the graphical model keeps the same variables and edges; only the factor
    values change (the circuit becomes Clifford)."""
    gates = c.gates.copy()
    vals = [] if c.gate_vals is None else list(c.gate_vals)
    s_slot = len(vals)
    vals.append(np.array([[1, 0], [0, 1j]], dtype=np.complex128))
    for i in range(len(gates)):
        if gates[i, 0] == T:
            gates[i, 0] = UD
            gates[i, 4] = s_slot
    return Circuit(c.rows, c.cols, gates, np.array(vals, dtype=np.complex128),
                   name=c.name + "_clifford")


def random_bitstrings(n: int, count: int, seed: int) -> np.ndarray:
    """count uniform n-bit strings as uint64, bit q = qubit q."""
    rng = np.random.default_rng(seed + 1_000_000)
    if n < 64:
        return rng.integers(0, 2 ** n, count, dtype=np.uint64)
    return rng.integers(0, 2 ** 63, count, dtype=np.uint64) * 2 + rng.integers(0, 2, count, dtype=np.uint64)


def random_amplitudes(n: int, count: int, seed: int, zeros: int = 0) -> np.ndarray:
    """count complex amplitudes with independent Gaussian real and imaginary
    parts of variance 2^-n / 2 (Porter-Thomas statistics for p = |a|^2), the
    first `zeros` set to 0; complex128."""
    rng = np.random.default_rng(seed + 3_000_000)
    a = (rng.standard_normal(count) + 1j * rng.standard_normal(count)) * np.sqrt(2.0 ** (-n) / 2.0)
    a[:zeros] = 0
    return a


def random_uniforms(count: int, seed: int) -> np.ndarray:
    """count uniform doubles in [0, 1) (the random numbers of a sampling step)."""
    return np.random.default_rng(seed + 4_000_000).random(count)


# The five workloads (grid, depth, seed, bitstring count).
WORKLOADS = {
    "c1_4x4_d16": dict(rows=4, cols=4, depth=16, seed=101, batch=64),
    "c2_5x5_d25": dict(rows=5, cols=5, depth=25, seed=201, batch=1024),
    "c3_5x6_d30": dict(rows=5, cols=6, depth=30, seed=301, batch=1024),
    "c4_5x5_d20_U": dict(rows=5, cols=5, depth=20, seed=401, batch=256, parameterised=True),
    "c5_4x5_d20": dict(rows=4, cols=5, depth=20, seed=501, batch=1024),
    "c5_5x5_d24": dict(rows=5, cols=5, depth=24, seed=502, batch=1024),
    "c5_6x6_d24": dict(rows=6, cols=6, depth=24, seed=503, batch=1024),
    "c5_6x7_d27": dict(rows=6, cols=7, depth=27, seed=504, batch=1024),
}


def workload(name: str) -> tuple[Circuit, np.ndarray]:
    w = WORKLOADS[name]
    make = parameterised_circuit if w.get("parameterised") else random_grid_circuit
    c = make(w["rows"], w["cols"], w["depth"], w["seed"])
    bits = random_bitstrings(c.n, w["batch"], w["seed"])
    return c, bits


def example_app_d() -> Circuit:
    """The two-qubit H-CZ-H circuit worked out in App. D of the paper."""
    g = np.array([(H, 0, 0, -1, -1), (H, 0, 1, -1, -1), (CZ, 1, 0, 1, -1),
                  (H, 2, 0, -1, -1), (H, 2, 1, -1, -1)], dtype=np.int32)
    return Circuit(1, 2, g, None, name="app_d")
