"""FP64 state-vector oracle (Eq. (fpath), Sec. III.A) over sv_oracle.c.

Test infrastructure: the HIP path never imports this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .gates import gate_matrix, gate_matrix_2q, KIND_CZ, KIND_U2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sv.so")
_lib = None


def build_library(force: bool = False) -> str:
    """Compile sv_oracle.c with gcc -O2 -fopenmp into oracle/liboracle_sv.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_library()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_sv_state.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        lib.oracle_sv_amplitudes.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int64, P]
        lib.oracle_sv_vjp.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int64, P, P, P]
        for f in (lib.oracle_sv_state, lib.oracle_sv_amplitudes, lib.oracle_sv_vjp):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ops(n: int, gates: np.ndarray, gate_vals):
    """Time-ordered op list: gates sorted by cycle (stable, so list order breaks
    ties), each single-qubit gate expanded to its 2x2 matrix."""
    gates = np.asarray(gates, dtype=np.int64).reshape(-1, 5)
    order = np.argsort(gates[:, 1], kind="stable")
    g = gates[order]
    op_q = np.empty((len(g), 2), dtype=np.int32)
    op_m = np.zeros((len(g), 2, 2, 2), dtype=np.float64)
    for i, (kind, _cyc, q0, q1, slot) in enumerate(g):
        if kind == KIND_CZ:
            op_q[i] = (q0, q1)
        else:
            op_q[i] = (q0, -1)
            m = gate_matrix(kind, slot, gate_vals)
            op_m[i, ..., 0] = m.real
            op_m[i, ..., 1] = m.imag
    return order, np.ascontiguousarray(op_q), np.ascontiguousarray(op_m)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _has_2q(gates) -> bool:
    g = np.asarray(gates, dtype=np.int64).reshape(-1, 5)
    return bool((g[:, 0] == KIND_U2).any())


def sv_state_numpy(n: int, gates, gate_vals=None) -> np.ndarray:
    """U|0...0> by plain numpy tensor contractions (every gate kind, including
    the general two-qubit gate); index = sum_q x_q 2^q."""
    g = np.asarray(gates, dtype=np.int64).reshape(-1, 5)
    g = g[np.argsort(g[:, 1], kind="stable")]
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    psi = psi.reshape([2] * n)          # axis n - 1 - q holds qubit q
    ax = lambda q: n - 1 - int(q)       # noqa: E731
    for kind, _cyc, q0, q1, slot in g:
        if kind == KIND_CZ:
            sl = [slice(None)] * n
            sl[ax(q0)] = 1
            sl[ax(q1)] = 1
            psi[tuple(sl)] *= -1.0
        elif kind == KIND_U2:
            T = gate_matrix_2q(slot, gate_vals).reshape(2, 2, 2, 2)   # (a0, a1, c0, c1)
            psi = np.tensordot(T, psi, axes=([2, 3], [ax(q0), ax(q1)]))
            psi = np.moveaxis(psi, [0, 1], [ax(q0), ax(q1)])
        else:
            m = gate_matrix(kind, slot, gate_vals)
            psi = np.moveaxis(np.tensordot(m, psi, axes=([1], [ax(q0)])), 0, ax(q0))
    return psi.reshape(-1)


def sv_state(n: int, gates, gate_vals=None) -> np.ndarray:
    """U|0...0> as complex128 [2^n]; index = sum_q x_q 2^q."""
    if _has_2q(gates):
        return sv_state_numpy(n, gates, gate_vals)
    _, op_q, op_m = _ops(n, gates, gate_vals)
    out = np.empty(2 ** n, dtype=np.complex128)
    rc = _load().oracle_sv_state(n, len(op_q), _ptr(op_q), _ptr(op_m), _ptr(out))
    if rc:
        raise ValueError("oracle_sv_state: invalid circuit (rc=%d)" % rc)
    return out


def sv_amplitudes(n: int, gates, gate_vals, bits) -> np.ndarray:
    """<x|U|0...0> for each uint64 bitstring x (bit q = qubit q)."""
    if _has_2q(gates):
        return sv_state_numpy(n, gates, gate_vals)[np.asarray(bits, dtype=np.uint64).astype(np.int64)]
    _, op_q, op_m = _ops(n, gates, gate_vals)
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    out = np.empty(len(bits), dtype=np.complex128)
    rc = _load().oracle_sv_amplitudes(n, len(op_q), _ptr(op_q), _ptr(op_m), _ptr(bits),
                                      len(bits), _ptr(out))
    if rc:
        raise ValueError("oracle_sv_amplitudes failed (rc=%d)" % rc)
    return out


def sv_vjp(n: int, gates, gate_vals, bits, grad_amps):
    """Amplitudes and, for every gate in the input order, the torch-convention
    gradient dL/dRe U + i dL/dIm U of a real loss whose gradient with respect
    to the amplitudes is grad_amps (zeros for CZ gates).  Returns
    (amps [B], per_gate [n_gates, 2, 2])."""
    order, op_q, op_m = _ops(n, gates, gate_vals)
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    gin = np.ascontiguousarray(grad_amps, dtype=np.complex128)
    amps = np.empty(len(bits), dtype=np.complex128)
    env = np.zeros((len(op_q), 2, 2), dtype=np.complex128)
    rc = _load().oracle_sv_vjp(n, len(op_q), _ptr(op_q), _ptr(op_m), _ptr(bits), len(bits),
                               _ptr(gin), _ptr(amps), _ptr(env))
    if rc:
        raise ValueError("oracle_sv_vjp failed (rc=%d)" % rc)
    per_gate = np.zeros_like(env)
    per_gate[order] = env
    return amps, per_gate


def sv_log_prob_gradient(n: int, gates, gate_vals, bits):
    """Gradient of L = sum_x log |<x|U|0>|^2 with respect to gate_vals
    (torch convention, summed over the gates that read each slot).  This loss
    is m times the negative of the cross-entropy estimator of Eq. (cee).
    Returns (amps, grad [n_slots, 2, 2])."""
    gates = np.asarray(gates, dtype=np.int64).reshape(-1, 5)
    amps0 = sv_amplitudes(n, gates, gate_vals, bits)
    grad_amps = 2.0 / np.conj(amps0)              # dL/dRe A + i dL/dIm A
    amps, per_gate = sv_vjp(n, gates, gate_vals, bits, grad_amps)
    n_slots = 0 if gate_vals is None else len(gate_vals)
    grad = np.zeros((n_slots, 2, 2), dtype=np.complex128)
    for i, (kind, _c, _q0, _q1, slot) in enumerate(gates):
        if slot >= 0 and kind != KIND_CZ:
            g = per_gate[i]
            if kind == 6:                      # diagonal slot: only the diagonal is read
                g = np.diag(np.diag(g))
            grad[slot] += g
    return amps, grad
