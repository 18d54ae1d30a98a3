"""FP64 normalisation checks of sets of amplitudes (Sec. III.A): with every
qubit of the 4x4 depth-16 circuit open, one call returns the whole output
distribution, entry by entry equal to the FP64 state vector, and its FP64 sum
is 1; for partial sets the sum over the open qubits is the probability that
the fixed qubits read x (at most 1), equal to the oracle's."""
import sys

import numpy as np
import pytest

import oracle
from paper_1712_05384_amd import circuits as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("ordering", [1, 0])
def test_all_qubits_open_sum_to_one(ordering):
    import paper_1712_05384_amd as Q
    c, _ = C.workload("c1_4x4_d16")
    _say("case c1 all 16 qubits open, ordering %d" % ordering)
    p = Q.plan(c, tuple(range(c.n)), ordering=ordering, out_c128=True)
    amps = p.amplitudes(np.zeros(1, dtype=np.uint64))          # [1, 2^16]
    ref = oracle.sv_state(c.n, c.gates, None)
    got = amps.cpu().numpy()[0]
    err = np.abs(got - ref).max()
    _say("  max err * 2^(n/2) = %.3g" % (err * 2 ** (c.n / 2)))
    assert err <= TOL * 2 ** (-c.n / 2)
    s = float(Q.prob_sums(amps).cpu().numpy()[0])
    _say("  sum p - 1 = %.3g" % (s - 1.0))
    assert abs(s - 1.0) <= 1e-6
    # the same sums from complex64 output
    p32 = Q.plan(c, tuple(range(c.n)), ordering=ordering)
    s32 = float(Q.prob_sums(p32.amplitudes(np.zeros(1, dtype=np.uint64))).cpu().numpy()[0])
    assert abs(s32 - 1.0) <= 1e-6


@pytest.mark.parametrize("open_qubits", [(0, 6, 12, 18), (0, 3, 6, 9, 12, 15, 18, 21)])
def test_set_probabilities_at_most_one(open_qubits):
    """5x5 depth 25 with 4 and 8 open qubits, 256 bitstrings (bucket order):
    sum_o |A(x, o)|^2 <= 1 and equal to the FP64 state vector's marginal."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c2_5x5_d25")
    bits = bits[:256]
    _say("case c2 open %s" % (open_qubits,))
    amps = Q.plan(c, open_qubits, ordering=1).amplitudes(bits)
    sums = Q.prob_sums(amps).cpu().numpy()
    psi = oracle.sv_state(c.n, c.gates, None)
    mask = 0
    for q in open_qubits:
        mask |= 1 << q
    ref = np.zeros(len(bits))
    for o in range(1 << len(open_qubits)):
        x = bits & np.uint64(~mask & ((1 << c.n) - 1))
        for i, q in enumerate(open_qubits):
            if (o >> i) & 1:
                x = x | np.uint64(1 << q)
        ref += np.abs(psi[x.astype(np.int64)]) ** 2
    rel = np.abs(sums - ref) / ref
    _say("  max rel err of the set sums %.3g, max sum %.3g" % (rel.max(), sums.max()))
    assert rel.max() <= 1e-4
    assert sums.max() <= 1.0
    assert np.all(sums > 0)


def test_prob_sums_rejects_bad_arguments():
    import paper_1712_05384_amd as Q
    from paper_1712_05384_amd import _native as N
    a = torch.zeros((2, 3), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        Q.prob_sums(a)
    with pytest.raises(N.QgmError):
        N.check(N.lib().qgm_prob_sums(None, 0, 4, 2, None, None))
