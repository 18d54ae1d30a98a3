"""GPU parity of the persistent bucket-elimination launch (ordering 1,
tree_exec 2: every level and the amplitude product in one launch, each
64-bitstring group pinned to one accelerator complex, tasks started by
completion flags) against the FP64 oracle and against the per-level launches.

Tolerance: max |A_gpu - A_oracle| <= 1e-5 * 2^{-n/2}.  Group counts cover
one group (a single complex busy), counts that do not divide by the eight
complexes, and full batches.
"""
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


def _plan(c, mode, **kw):
    import paper_1712_05384_amd as Q
    return Q.plan(c, ordering=1, tree_exec=mode, **kw)


def _amps(p, bits, gate_vals=None):
    out = p.amplitudes(bits, gate_vals)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:, 0]


@pytest.mark.parametrize("rows,cols,depth,seed,B", [(3, 4, 12, 7, 1), (3, 4, 12, 7, 64), (3, 4, 12, 7, 300),
                                                    (4, 4, 16, 3, 700), (4, 5, 16, 6, 1024), (2, 2, 1, 2, 513),
                                                    (1, 1, 3, 1, 600), (5, 4, 30, 16, 1100)])
def test_persistent_matches_oracle_and_level_launches(rows, cols, depth, seed, B):
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, B, seed + 100)
    _say("case persistent %s B=%d" % (c.name, B))
    got = _amps(_plan(c, 2), bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    bound = TOL * 2 ** (-c.n / 2)
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= bound
    lev = _amps(_plan(c, 1), bits)
    assert np.abs(got - lev).max() <= bound


def test_persistent_gate_values_c128_and_repeat():
    c = C.parameterised_circuit(4, 4, 14, 8)
    bits = C.random_bitstrings(c.n, 640, 8)
    gv = c.gate_vals.astype(np.complex64)
    _say("case persistent %s B=640 (gate_vals, complex128 out)" % c.name)
    p = _plan(c, 2, out_c128=True)
    got = _amps(p, bits, torch.tensor(gv))
    assert got.dtype == np.complex128
    ref = oracle.sv_amplitudes(c.n, c.gates, gv.astype(np.complex128), bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)
    for _ in range(3):
        assert np.array_equal(_amps(p, bits, torch.tensor(gv)), got)


def test_persistent_c2_full_size():
    """5x5 depth 25, 1024 bitstrings in one persistent launch against the 2^25 state vector."""
    c, bits = C.workload("c2_5x5_d25")
    _say("case persistent c2_5x5_d25 B=1024")
    got = _amps(_plan(c, 2), bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    err = np.abs(got - ref).max()
    _say("  persistent c2 max err * 2^(n/2) = %.3g" % (err * 2 ** (c.n / 2)))
    assert err <= TOL * 2 ** (-c.n / 2)


def test_persistent_give_up_is_reported():
    """A spin limit of one poll, set from the host, makes the launch's own
    bounded waits give up (every wave still ends): the call itself returns,
    qgm_plan_check reports QGM_E_INTERNAL once and then clears the record, and
    a plan with the default limit reports nothing."""
    import paper_1712_05384_amd as Q
    from paper_1712_05384_amd import _native as N
    c, bits = C.workload("c2_5x5_d25")
    _say("case persistent give-up c2_5x5_d25 B=1024 spin limit 1")
    p = _plan(c, 2, persist_spin=1)
    p.amplitudes(bits)
    with pytest.raises(N.QgmError) as ei:
        p.check()
    assert ei.value.status == N.QGM_E_INTERNAL
    p.check()                      # the record was cleared by the first check
    q = _plan(c, 2)
    got = _amps(q, bits)
    q.check()
    assert np.isfinite(got).all()


def test_persistent_graph_branches_and_replays():
    """A HIP graph with two persistent branches and a per-level branch replays to the eager results."""
    import paper_1712_05384_amd as Q
    c1 = C.random_grid_circuit(4, 4, 16, 2)
    c2 = C.random_grid_circuit(3, 5, 14, 4)
    plans = [_plan(c1, 2), _plan(c2, 2), _plan(c2, 1)]
    bits = [C.random_bitstrings(c1.n, 1024, 1), C.random_bitstrings(c2.n, 520, 2), C.random_bitstrings(c2.n, 520, 2)]
    eager = [p.amplitudes(b).cpu().numpy() for p, b in zip(plans, bits)]
    g = Q.Graph(plans, bits, [None] * 3)
    for rep in range(3):
        outs = [o.cpu().numpy() for o in g.launch()]
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(outs, eager)):
            assert np.array_equal(a, b), (rep, i, int(np.isnan(a).sum()), int(np.isnan(b).sum()),
                                          float(np.nanmax(np.abs(a - b))), int((a != b).sum()))
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
    for p in plans:
        p.check()
    ref = oracle.sv_amplitudes(c1.n, c1.gates, None, bits[0])
    assert np.abs(eager[0][:, 0] - ref).max() <= TOL * 2 ** (-c1.n / 2)
    assert np.abs(eager[2] - eager[1]).max() <= TOL * 2 ** (-c2.n / 2)

