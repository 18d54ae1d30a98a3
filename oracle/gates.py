"""Gate matrices used by the oracle (its own table; the HIP path has another).

Matrix convention: U[row][col] = <row|U|col>, i.e. psi_U(b', b) = U[b'][b] in
the notation of Sec. III.B (row = the bit after the gate).

* H: psi_H(1,1) = -1/sqrt(2), other entries +1/sqrt(2) (Sec. III.B and the
  Hadamard table of App. D).
* T = diag(1, e^{i pi/4}) (Sec. II, gate list).
* X^1/2, Y^1/2: pi/2 rotations about X and Y (Sec. II).  The paper fixes them
  only up to a global phase; App. F, Eq. (phX) fixes the relative phases
  (no-flip/flip ratio i for X^1/2; only <0|Y^1/2|1> negative).  The reading
  used here is RX(pi/2) = (1/sqrt2)[[1,-i],[-i,1]] and
  RY(pi/2) = (1/sqrt2)[[1,-1],[1,1]].
* CZ = diag(1,1,1,-1): psi_CZ(1,1) = -1, others 1 (Sec. III.B, App. D table).
* U / UD: the value is read from gate_vals[slot].
"""
import numpy as np

KIND_H, KIND_T, KIND_XH, KIND_YH, KIND_CZ, KIND_U, KIND_UD = 0, 1, 2, 3, 4, 5, 6
KIND_TDG, KIND_XHDG, KIND_YHDG, KIND_X, KIND_Y, KIND_Z = 7, 8, 9, 10, 11, 12
KIND_U2 = 13   # general two-qubit gate; row r of its 4x4 matrix in value slot (slot + r)

_R2 = 1.0 / np.sqrt(2.0)
_FIXED = {
    KIND_H: np.array([[_R2, _R2], [_R2, -_R2]], dtype=np.complex128),
    KIND_T: np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128),
    KIND_XH: np.array([[_R2, -1j * _R2], [-1j * _R2, _R2]], dtype=np.complex128),
    KIND_YH: np.array([[_R2, -_R2], [_R2, _R2]], dtype=np.complex128),
}
# inverses of the fixed gates (conjugate transposes) and the Pauli operators
for _k, _kd in ((KIND_T, KIND_TDG), (KIND_XH, KIND_XHDG), (KIND_YH, KIND_YHDG)):
    _FIXED[_kd] = _FIXED[_k].conj().T.copy()
_FIXED[KIND_X] = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_FIXED[KIND_Y] = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_FIXED[KIND_Z] = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def gate_matrix(kind: int, slot: int, gate_vals) -> np.ndarray:
    """2x2 complex128 matrix of a single-qubit gate."""
    kind = int(kind)
    if kind in _FIXED:
        return _FIXED[kind].copy()
    if kind in (KIND_U, KIND_UD):
        m = np.asarray(gate_vals[int(slot)], dtype=np.complex128).reshape(2, 2)
        if kind == KIND_UD:
            m = np.diag(np.diag(m))
        return m.copy()
    raise ValueError(f"gate kind {kind} is not a single-qubit gate")


def is_diagonal_kind(kind: int) -> bool:
    return int(kind) in (KIND_T, KIND_CZ, KIND_UD, KIND_TDG, KIND_Z)


def gate_matrix_2q(slot: int, gate_vals) -> np.ndarray:
    """4x4 complex128 matrix of a general two-qubit gate: M[2 a0 + a1][2 c0 + c1]
    (a0, c0 on its first qubit) with row r read from gate_vals[slot + r]."""
    return np.stack([np.asarray(gate_vals[int(slot) + r], dtype=np.complex128).reshape(4) for r in range(4)])
