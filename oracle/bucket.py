"""Bucket (variable) elimination in FP64 -- TEST INFRASTRUCTURE (oracle).

The algorithm of Sec. IV and App. A written out plainly, for circuits whose
state vector does not fit (n > 30):

* variables b_j^k per Sec. III.A (one per non-diagonal gate, b_j^0 = 0 and
  b_j^{d_j} = x_j by the deltas of Eq. (psi_x));
* factors per Sec. III.B (2x2 table on (new, old) for non-diagonal gates,
  a function of the current variable for diagonal ones, (-1)^{b b'} for CZ),
  with the fixed variables substituted;
* an elimination order (App. A takes it as given): here a greedy min-degree
  order on the graph of the remaining variables, chosen independently of the
  HIP path's vertical order;
* buckets: each tensor goes to the bucket of its earliest variable; a bucket
  is processed by multiplying its tensors with broadcasting and summing over
  the bucket's variable; the result goes to the bucket of its earliest
  remaining variable, and rank-0 results multiply into the amplitude.

numpy.einsum serves as the broadcast product + sum of a bucket.
"""
from __future__ import annotations

import numpy as np

from .gates import gate_matrix, is_diagonal_kind, KIND_CZ

_LETTERS = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"


def _factors(n, gates, gate_vals, x):
    """Factors as (vars, table) with the fixed variables substituted."""
    gates = np.asarray(gates, dtype=np.int64).reshape(-1, 5)
    order = np.argsort(gates[:, 1], kind="stable")
    cur = list(range(n))
    n_vars = n
    raw = []
    for gi in order:
        kind, _c, q0, q1, slot = (int(v) for v in gates[gi])
        if kind == KIND_CZ:
            raw.append(((cur[q0], cur[q1]), np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128)))
        elif is_diagonal_kind(kind):
            m = gate_matrix(kind, slot, gate_vals)
            raw.append(((cur[q0],), np.array([m[0, 0], m[1, 1]], dtype=np.complex128)))
        else:
            m = gate_matrix(kind, slot, gate_vals)
            raw.append(((n_vars, cur[q0]), m.astype(np.complex128)))   # psi(b', b) = U[b'][b]
            cur[q0] = n_vars
            n_vars += 1
    fixed = {j: 0 for j in range(n)}
    scalar = 1.0 + 0j
    for j in range(n):
        xj = (int(x) >> j) & 1
        if cur[j] in fixed and fixed[cur[j]] != xj:
            return None, 0.0, n_vars        # worldline never flips but x_j = 1
        fixed[cur[j]] = xj
    out = []
    for vs, t in raw:
        idx = tuple(fixed[v] if v in fixed else slice(None) for v in vs)
        t2 = t[idx]
        free = tuple(v for v in vs if v not in fixed)
        if not free:
            scalar *= complex(t2)
        else:
            out.append((free, np.array(t2, dtype=np.complex128)))
    return out, scalar, n_vars


def _min_degree_order(factors):
    adj = {}
    for vs, _ in factors:
        for v in vs:
            adj.setdefault(v, set())
        for a in vs:
            for b in vs:
                if a != b:
                    adj[a].add(b)
    order = []
    alive = set(adj)
    while alive:
        v = min(alive, key=lambda u: (len(adj[u] & alive), u))
        nb = adj[v] & alive
        for a in nb:
            adj[a] |= nb - {a}
        alive.remove(v)
        order.append(v)
    return order


def bucket_amplitude(n: int, gates, gate_vals, x: int) -> complex:
    """<x|U|0...0> by bucket elimination (App. A)."""
    factors, scalar, _ = _factors(n, gates, gate_vals, x)
    if factors is None:
        return 0j
    order = _min_degree_order(factors)
    pos = {v: i for i, v in enumerate(order)}
    buckets = [[] for _ in order]

    def place(vs, t):
        perm = sorted(range(len(vs)), key=lambda i: pos[vs[i]])
        vs2 = tuple(vs[i] for i in perm)
        t2 = np.transpose(t, perm)
        buckets[pos[vs2[0]]].append((vs2, t2))

    for vs, t in factors:
        place(vs, t)
    result = scalar
    for i, v in enumerate(order):
        if not buckets[i]:
            continue
        allv = sorted({u for vs, _ in buckets[i] for u in vs}, key=lambda u: pos[u])
        if len(allv) > len(_LETTERS):
            raise ValueError("bucket too wide for einsum")
        letter = {u: _LETTERS[j] for j, u in enumerate(allv)}
        outv = [u for u in allv if u != v]
        spec = ",".join("".join(letter[u] for u in vs) for vs, _ in buckets[i])
        spec += "->" + "".join(letter[u] for u in outv)
        t = np.einsum(spec, *[t for _, t in buckets[i]], optimize="greedy")
        buckets[i] = []
        if outv:
            place(tuple(outv), t)
        else:
            result *= complex(t)
    return complex(result)


def bucket_amplitudes(n: int, gates, gate_vals, bits) -> np.ndarray:
    return np.array([bucket_amplitude(n, gates, gate_vals, int(x)) for x in np.asarray(bits, dtype=np.uint64)],
                    dtype=np.complex128)
