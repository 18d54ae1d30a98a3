"""Writes oracle amplitudes for workloads whose state vector is too large to
recompute inside a test (FP64 state vector, oracle/ only).

    python tests/golden/make_golden.py c3_5x6_d30

produces tests/golden/<workload>_amps.npy: complex128 [B], the oracle's
<x_b|U|0> for the workload's seeded circuit and bitstrings.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1712_05384_amd import circuits as C  # noqa: E402  (input generator only)


def main(name: str) -> None:
    c, bits = C.workload(name)
    t = time.time()
    amps = oracle.sv_amplitudes(c.n, c.gates, c.gate_vals, bits)
    path = os.path.join(HERE, f"{name}_amps.npy")
    np.save(path, amps.astype(np.complex128), allow_pickle=False)
    print(f"{name}: n={c.n}, {len(bits)} amplitudes, {time.time() - t:.1f} s -> {path}")


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        main(nm)
