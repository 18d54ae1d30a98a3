"""CPU oracle for output amplitudes of circuits -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP path: it takes the circuit as a
plain gate array (kind, cycle, q0, q1, slot) and owns its own gate tables.

Contents
  gates.py        fixed gate matrices (Sec. II; tables of App. D)
  statevector.py  FP64 state vector (Eq. (fpath)) and its adjoint-state VJP,
                  over the C library sv_oracle.c
  brute_force.py  tiny exhaustive sums: Eq. (psi_x) over all worldline
                  variables, and the Ising-phase form of App. F
  bucket.py       bucket elimination of App. A in FP64 (for n > 30)
  xeb.py          cross entropy (Eq. (cee)), fidelity (Eq. (ae)), entropy and
                  sampling from a set of probabilities (App. B, App. C)
  observable.py   <psi|O|psi> of Pauli strings from the state vector
"""
from .gates import gate_matrix, KIND_H, KIND_T, KIND_XH, KIND_YH, KIND_CZ, KIND_U, KIND_UD  # noqa: F401
from .statevector import sv_state, sv_amplitudes, sv_vjp, sv_log_prob_gradient, build_library  # noqa: F401
from .brute_force import path_sum_amplitude, ising_amplitude  # noqa: F401
from .bucket import bucket_amplitude, bucket_amplitudes  # noqa: F401
from . import xeb  # noqa: F401
from .observable import expectation  # noqa: F401
