"""Expectation values of Pauli strings, <psi|O|psi> with psi = U|0...0>, from
the FP64 state vector -- TEST INFRASTRUCTURE (see oracle/__init__.py).  The
plain definition (Sec. III.B names the quantity <0|U^dag O U|0>)."""
import numpy as np

from .statevector import sv_state


def apply_pauli_string(n: int, psi: np.ndarray, paulis: dict) -> np.ndarray:
    """O psi for O = prod over {qubit: 'X' | 'Y' | 'Z'}; index bit q = qubit q."""
    idx = np.arange(1 << n, dtype=np.int64)
    out = psi.astype(np.complex128).copy()
    for q, k in paulis.items():
        bit = (idx >> int(q)) & 1
        k = str(k).upper()
        if k == "Z":
            out = out * np.where(bit == 1, -1.0, 1.0)
        else:
            flipped = out[idx ^ (1 << int(q))]   # (X psi)[x] = psi[x xor 2^q]
            if k == "X":
                out = flipped
            elif k == "Y":                       # Y|0> = i|1>, Y|1> = -i|0>: (Y psi)[x] = -i (-1)^{x_q} psi[x xor 2^q]
                out = -1j * np.where(bit == 1, -1.0, 1.0) * flipped
            else:
                raise ValueError(k)
    return out


def expectation(n: int, gates, gate_vals, paulis: dict) -> complex:
    psi = sv_state(n, gates, gate_vals)
    return complex(np.vdot(psi, apply_pauli_string(n, psi, paulis)))
