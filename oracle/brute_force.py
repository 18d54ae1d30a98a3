"""Tiny exhaustive sums (test infrastructure; circuits with <= ~22 free variables).

path_sum_amplitude: Eq. (psi_x) of Sec. III.B written out.  Each qubit j gets
  worldline variables b_j^0..b_j^{d_j}, one new variable per non-diagonal gate
  (Sec. III.A); b_j^0 = 0 and b_j^{d_j} = x_j are the delta functions of
  Eq. (psi_x).  Every gate contributes its factor psi_U (a 2x2 table on
  (new, old) variables for non-diagonal single-qubit gates, a function of the
  current variable for diagonal ones, (-1)^{b b'} for CZ).  The amplitude is the
  sum over all assignments of the remaining variables of the product of the
  factors.  Independent of the state-vector code and of variable elimination.

ising_amplitude: the Ising form of App. F, Eq. (path1): every path has the
  same magnitude 2^{-L/2} (L = number of non-diagonal gates) and a phase that
  is a sum of per-gate terms, Eqs. (phX), (phT), (phCZ), with s = 1 - 2b.
  The paper omits path-independent phases; under the X^1/2 = RX(pi/2) reading
  each X^1/2 carries the constant -i, which is restored here so the result is
  the amplitude itself.  Hadamards contribute pi*b*b' (their table in App. D);
  for the cycle-0 layer b = 0, so the phase vanishes, which is why Eq. (phX)
  has no separate Hadamard term.  Only the fixed gate set {H, X^1/2, Y^1/2, T,
  CZ} is supported.
"""
from __future__ import annotations

import itertools

import numpy as np

from .gates import gate_matrix, is_diagonal_kind, KIND_CZ, KIND_H, KIND_T, KIND_XH, KIND_YH


def _worldlines(n: int, gates: np.ndarray):
    """Walk the gates in time order and attach variable ids.  Returns
    (factors, first_var, last_var, n_vars); a factor is (gate_row, vars)."""
    order = np.argsort(gates[:, 1], kind="stable")
    cur = list(range(n))                 # variable b_j^0 of qubit j has id j
    n_vars = n
    factors = []
    for gi in order:
        kind, _cyc, q0, q1, _slot = (int(v) for v in gates[gi])
        if kind == KIND_CZ:
            factors.append((gi, (cur[q0], cur[q1])))
        elif is_diagonal_kind(kind):
            factors.append((gi, (cur[q0],)))
        else:
            new = n_vars
            n_vars += 1
            factors.append((gi, (new, cur[q0])))   # psi_U(b', b) = U[b'][b]
            cur[q0] = new
    return factors, list(range(n)), cur, n_vars


def path_sum_amplitude(n: int, gates, gate_vals, x: int) -> complex:
    """<x|U|0...0> by brute force over Eq. (psi_x)."""
    gates = np.asarray(gates, dtype=np.int64).reshape(-1, 5)
    factors, first, last, n_vars = _worldlines(n, gates)
    fixed = {}
    for j in range(n):
        fixed[first[j]] = 0
    for j in range(n):
        xj = (int(x) >> j) & 1
        if last[j] in fixed and fixed[last[j]] != xj:
            return 0j                     # qubit never flipped but x_j = 1
        fixed[last[j]] = xj
    free = [v for v in range(n_vars) if v not in fixed]
    if len(free) > 24:
        raise ValueError("too many free variables for brute force: %d" % len(free))
    tables = []
    for gi, vs in factors:
        kind, _c, _q0, _q1, slot = (int(v) for v in gates[gi])
        if kind == KIND_CZ:
            tables.append((vs, lambda a, b: -1.0 if (a and b) else 1.0))
        else:
            m = gate_matrix(kind, slot, gate_vals)
            if len(vs) == 1:
                tables.append((vs, lambda a, m=m: m[a, a]))
            else:
                tables.append((vs, lambda a, b, m=m: m[a, b]))
    total = 0j
    val = dict(fixed)
    for assign in itertools.product((0, 1), repeat=len(free)):
        for v, a in zip(free, assign):
            val[v] = a
        p = 1 + 0j
        for vs, f in tables:
            p *= f(*(val[v] for v in vs))
            if p == 0:
                break
        total += p
    return total


def ising_amplitude(n: int, gates, x: int) -> complex:
    """<x|U|0...0> from the Ising-phase form of App. F."""
    gates = np.asarray(gates, dtype=np.int64).reshape(-1, 5)
    factors, first, last, n_vars = _worldlines(n, gates)
    fixed = {first[j]: 0 for j in range(n)}
    for j in range(n):
        xj = (int(x) >> j) & 1
        if last[j] in fixed and fixed[last[j]] != xj:
            return 0j
        fixed[last[j]] = xj
    free = [v for v in range(n_vars) if v not in fixed]
    n_nondiag = 0
    const = 1 + 0j
    terms = []   # (vars, phase function in units of pi/4, of s-values)
    for gi, vs in factors:
        kind = int(gates[gi, 0])
        if kind == KIND_CZ:        # Eq. (phCZ): pi (1-s_i)/2 (1-s_j)/2
            terms.append((vs, lambda si, sj: 4 * ((1 - si) // 2) * ((1 - sj) // 2)))
        elif kind == KIND_T:       # Eq. (phT): (pi/4) (1-s)/2
            terms.append((vs, lambda s: (1 - s) // 2))
        elif kind == KIND_XH:      # Eq. (phX), alpha = 1: (pi/2) (1 + s^{k-1} s^k)/2
            n_nondiag += 1
            const *= -1j
            terms.append((vs, lambda sk, skm1: 2 * ((1 + skm1 * sk) // 2)))
        elif kind == KIND_YH:      # Eq. (phX), alpha = 0: pi (1 - s^{k-1})/2 (1 + s^k)/2
            n_nondiag += 1
            terms.append((vs, lambda sk, skm1: 4 * ((1 - skm1) // 2) * ((1 + sk) // 2)))
        elif kind == KIND_H:       # Hadamard table: pi b b'
            n_nondiag += 1
            terms.append((vs, lambda sk, skm1: 4 * ((1 - skm1) // 2) * ((1 - sk) // 2)))
        else:
            raise ValueError("ising_amplitude supports only H, X^1/2, Y^1/2, T, CZ")
    if len(free) > 24:
        raise ValueError("too many free variables for brute force: %d" % len(free))
    val = {v: 1 - 2 * b for v, b in fixed.items()}
    counts = np.zeros(8, dtype=np.int64)        # paths per phase class (units of pi/4)
    for assign in itertools.product((1, -1), repeat=len(free)):
        for v, s in zip(free, assign):
            val[v] = s
        ph = 0
        for vs, f in terms:
            ph += f(*(val[v] for v in vs))
        counts[ph % 8] += 1
    phases = np.exp(1j * np.pi / 4 * np.arange(8))
    return complex(const * 2.0 ** (-n_nondiag / 2) * np.dot(counts, phases))
