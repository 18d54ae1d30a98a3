"""GPU parity of sliced bucket plans (ordering 1; Sec. V outlook: space-time
tradeoffs).  A sliced variable is fixed by a bit above the qubits of a batch
column's word, the 2^s slices of every bitstring run as batch columns in
chunks, and their amplitudes are summed in FP64 in slice order.

Tolerance as everywhere for complex64: max |A_gpu - A_oracle| <= 1e-5 * 2^{-n/2}.
The 5x9 depth-40 and 7x8 depth-30 circuits are beyond any state vector; there
the checks are properties that hold at any size: Clifford variants give
probabilities that are exact powers of 1/2 (or 0), and two plans with
different sliced variables agree.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1712_05384_amd import circuits as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _amps(p, bits, gate_vals=None):
    out = p.amplitudes(bits, None if gate_vals is None else torch.tensor(gate_vals.astype(np.complex64)))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_c3_ordering_1_two_sliced_variables():
    """5x6 depth 30, 1024 bitstrings, two sliced variables, complex128 output,
    against the stored FP64 state-vector amplitudes; the same slices one chunk
    at a time (a memory budget below the all-slices workspace) give the same
    bits."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c3_5x6_d30")
    ref = np.load(os.path.join(GOLDEN, "c3_5x6_d30_amps.npy"), allow_pickle=False)
    p = Q.plan(c, ordering=1, min_sliced_vars=2, out_c128=True)
    info = p.info(0)
    assert info["n_sliced"] == 2 and info["slice_chunk_bits"] == 2
    _say("case sliced c3 5x6 d30 B=1024 slices 2 form", "lds" if info["lds_ok"] else "levels")
    got = _amps(p, bits)[:, 0]
    err = np.abs(got - ref).max()
    _say("  max err * 2^(n/2) = %.3g" % (err * 2 ** (c.n / 2)))
    assert err <= TOL * 2 ** (-c.n / 2)
    budget = p.workspace_bytes(64) - 1
    pc = Q.plan(c, ordering=1, min_sliced_vars=2, out_c128=True, mem_budget=budget)
    ic = pc.info(0)
    assert ic["n_sliced"] == 2 and ic["slice_chunk_bits"] < 2 and pc.workspace_bytes(64) <= budget
    assert ic["sliced_qubit"] == info["sliced_qubit"] and ic["sliced_k"] == info["sliced_k"]
    _say("case sliced c3 chunks of 2^%d slices" % ic["slice_chunk_bits"])
    assert np.array_equal(_amps(pc, bits)[:, 0], got)


@pytest.mark.parametrize("mode", [1, 3])
@pytest.mark.parametrize("B", [1, 63, 130])
def test_sliced_ragged_batches(B, mode):
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(3, 4, 12, 7)
    bits = C.random_bitstrings(c.n, B, 7)
    p = Q.plan(c, ordering=1, min_sliced_vars=3, tree_exec=mode)
    _say("case sliced 3x4 d12 B=%d slices 3 tree_exec %d" % (B, mode))
    got = _amps(p, bits)[:, 0]
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)


@pytest.mark.parametrize("mode", [1, 3])
def test_sliced_gate_values_and_c2(mode):
    """Gate values (factor tables per call) with two slices; and the 5x5
    depth-25 workload (1024 bitstrings) with three slices, both launch forms."""
    import paper_1712_05384_amd as Q
    cp = C.parameterised_circuit(4, 4, 14, 8)
    bits = C.random_bitstrings(cp.n, 128, 8)
    gv = cp.gate_vals.astype(np.complex64)
    p = Q.plan(cp, ordering=1, min_sliced_vars=2, tree_exec=mode)
    _say("case sliced %s B=128 gate values tree_exec %d" % (cp.name, mode))
    got = _amps(p, bits, gv)[:, 0]
    ref = oracle.sv_amplitudes(cp.n, cp.gates, gv.astype(np.complex128), bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-cp.n / 2)
    c, bits = C.workload("c2_5x5_d25")
    p = Q.plan(c, ordering=1, min_sliced_vars=3, tree_exec=mode)
    _say("case sliced c2 5x5 d25 B=1024 slices 3 tree_exec %d" % mode)
    got = _amps(p, bits)[:, 0]
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)


def test_sliced_open_qubits():
    """Sets of amplitudes (Sec. III.A) with two sliced variables: every
    completion of the open bits against the state vector."""
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(4, 4, 14, 3)
    oq = (2, 9)
    bits = C.random_bitstrings(c.n, 64, 3)
    p = Q.plan(c, oq, ordering=1, min_sliced_vars=2)
    _say("case sliced 4x4 d14 open (2, 9) B=64")
    got = _amps(p, bits)
    psi = oracle.sv_state(c.n, c.gates, None)
    for o in range(4):
        y = bits.copy()
        for j, q in enumerate(oq):
            y = (y & ~np.uint64(1 << q)) | np.uint64(((o >> j) & 1) << q)
        assert np.abs(got[:, o] - psi[y.astype(np.int64)]).max() <= TOL * 2 ** (-c.n / 2)


@pytest.mark.parametrize("rows,cols,depth", [(5, 9, 40), (7, 8, 30)])
def test_headline_circuits(rows, cols, depth):
    """The 5x9 depth-40 and 7x8 depth-30 circuits of the Abstract, 64
    bitstrings each: the Clifford variant (every T replaced by S) gives
    probabilities that are 0 or exact powers of 1/2, and the random circuit's
    amplitudes from two plans with different sliced variables agree."""
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(rows, cols, depth, 1)
    bits = C.random_bitstrings(c.n, 64, 1)
    cl = C.clifford_variant(c)
    pcl = Q.plan(cl, ordering=1)
    _say("case headline clifford %dx%d d%d B=64 slices %d" % (rows, cols, depth, pcl.info(0)["n_sliced"]))
    a = _amps(pcl, bits, cl.gate_vals)[:, 0]
    pr = np.abs(a.astype(np.complex128)) ** 2
    nz = pr[pr > 2.0 ** (-c.n - 12)]
    assert len(nz) > 0 and np.all(pr[pr <= 2.0 ** (-c.n - 12)] < 2.0 ** (-c.n - 12))
    k = np.log2(1 / nz)
    _say("  dyadic exponents %s, max deviation %.2e" % (sorted(set(np.round(k).astype(int).tolist()))[:8],
                                                        np.abs(k - np.round(k)).max()))
    assert np.abs(k - np.round(k)).max() < 1e-4
    p1 = Q.plan(c, ordering=1)
    s1 = p1.info(0)["n_sliced"]
    p2 = Q.plan(c, ordering=1, min_sliced_vars=s1 + 1)
    _say("case headline %dx%d d%d B=64 slices %d and %d" % (rows, cols, depth, s1, s1 + 1))
    x1 = _amps(p1, bits)[:, 0]
    x2 = _amps(p2, bits)[:, 0]
    d = np.abs(x1 - x2).max() * 2 ** (c.n / 2)
    _say("  max |A1 - A2| * 2^(n/2) = %.3g, mean N p = %.3f" % (d, np.mean(np.abs(x1) ** 2) * 2.0 ** c.n))
    assert d <= 2 * TOL
