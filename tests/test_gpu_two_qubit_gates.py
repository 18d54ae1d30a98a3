"""GPU parity of circuits with non-diagonal two-qubit gates (a factor over the
four worldline variables of the two qubits, Sec. III.B) on the bucket path,
against the FP64 state vector: max |A_gpu - A_oracle| <= 1e-5 * 2^{-n/2}."""
import sys

import numpy as np
import pytest

import oracle
from paper_1712_05384_amd import circuits as C
from test_two_qubit_gates import brickwork, haar_2x2, haar_4x4, u2_slots

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("rows,cols,layers,seed,B", [(1, 2, 1, 1, 4), (2, 2, 3, 2, 16), (3, 3, 6, 3, 65),
                                                     (3, 4, 8, 4, 130), (4, 5, 8, 5, 64)])
def test_two_qubit_brickwork(rows, cols, layers, seed, B):
    import paper_1712_05384_amd as Q
    c = brickwork(rows, cols, layers, seed)
    bits = C.random_bitstrings(c.n, B, seed)
    _say("case u2 %s B=%d" % (c.name, B))
    gv0 = c.gate_vals.astype(np.complex64)
    p = Q.plan(c, ordering=1)
    got = p.amplitudes(bits, torch.tensor(gv0)).cpu().numpy()[:, 0]
    ref = oracle.sv_amplitudes(c.n, c.gates, gv0.astype(np.complex128), bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)
    # new gate values at call time, complex128 output
    rng = np.random.default_rng(seed + 100)
    gv = c.gate_vals.copy()
    for kind, _cyc, _q0, _q1, slot in c.gates:
        if kind == C.U2:
            gv[slot:slot + 4] = u2_slots(haar_4x4(rng))
        elif kind == C.U:
            gv[slot] = haar_2x2(rng)
    assert gv.shape == c.gate_vals.shape
    p2 = Q.plan(c, ordering=1, out_c128=True)
    got2 = p2.amplitudes(bits, torch.tensor(gv.astype(np.complex64))).cpu().numpy()[:, 0]
    ref2 = oracle.sv_amplitudes(c.n, c.gates, gv.astype(np.complex64).astype(np.complex128), bits)
    assert np.abs(got2 - ref2).max() <= TOL * 2 ** (-c.n / 2)


def test_two_qubit_gates_mixed_with_cz_and_fixed_gates_open_qubits():
    import paper_1712_05384_amd as Q
    base = C.random_grid_circuit(3, 4, 10, 9)
    rng = np.random.default_rng(9)
    last = int(base.gates[:, 1].max())
    g = [tuple(int(v) for v in r) for r in base.gates]
    vals = []
    for i, (a, b) in enumerate([(0, 1), (5, 9), (2, 6), (10, 11), (4, 5)]):
        g.append((C.U2, last + 1 + i, a, b, len(vals)))
        vals.extend(u2_slots(haar_4x4(rng)))
    g += [(C.T, last + 7, q, -1, -1) for q in range(0, 12, 3)] + [(C.CZ, last + 8, 1, 5, -1)]
    c = C.Circuit(3, 4, np.array(g, dtype=np.int32), np.array(vals), "u2_mixed_3x4")
    bits = C.random_bitstrings(c.n, 70, 9)
    _say("case u2 mixed open=(1, 10)")
    gv = c.gate_vals.astype(np.complex64)
    psi = oracle.sv_state(c.n, c.gates, gv.astype(np.complex128))
    got = Q.plan(c, ordering=1).amplitudes(bits, torch.tensor(gv)).cpu().numpy()[:, 0]
    assert np.abs(got - psi[bits.astype(np.int64)]).max() <= TOL * 2 ** (-c.n / 2)
    oq = (1, 10)
    out = Q.plan(c, oq, ordering=1).amplitudes(bits, torch.tensor(gv)).cpu().numpy()
    for o in range(4):
        x = bits.copy()
        for i, q in enumerate(oq):
            x = (x & ~np.uint64(1 << q)) | np.uint64(((o >> i) & 1) << q)
        assert np.abs(out[:, o] - psi[x.astype(np.int64)]).max() <= TOL * 2 ** (-c.n / 2)


def test_two_qubit_gates_backward_rejected():
    import paper_1712_05384_amd as Q
    from paper_1712_05384_amd import _native as N
    c = brickwork(2, 2, 2, 3)
    p = Q.plan(c, ordering=1)
    bits = C.random_bitstrings(c.n, 64, 3)
    gv = torch.tensor(c.gate_vals.astype(np.complex64), device="cuda")
    bd = torch.from_numpy(bits.view(np.int64)).cuda()
    with pytest.raises(N.QgmError) as e:
        p.backward(bd, torch.ones(64, 1, dtype=torch.complex64, device="cuda"), gv)
    assert e.value.status == N.QGM_E_UNSUPPORTED
