"""Full-size workloads on the GPU: the 5x6 depth-30 circuit (sliced, FP64 slice
sum) against stored oracle amplitudes, and the uneven four-circuit batch run
as one HIP graph, against the state vector (n <= 25) or the FP64 bucket
elimination oracle (n = 36, 42) plus Porter-Thomas statistics."""
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
EULER_GAMMA = 0.5772156649015329
C5 = ("c5_4x5_d20", "c5_5x5_d24", "c5_6x6_d24", "c5_6x7_d27")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_c3_sliced_against_stored_oracle():
    """5x6 depth 30, 1024 bitstrings, 2 sliced variables summed in FP64 on the
    GPU, complex128 output; the stored values come from the FP64 state vector
    (tests/golden/make_golden.py)."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c3_5x6_d30")
    ref = np.load(os.path.join(GOLDEN, "c3_5x6_d30_amps.npy"), allow_pickle=False)
    _say("case c3 5x6 d30 B=1024 slices=2")
    p = Q.plan(c, min_sliced_vars=2, out_c128=True)
    assert p.info(0)["n_sliced"] == 2
    got = p.amplitudes(bits).cpu().numpy()[:, 0]
    err = np.abs(got - ref).max()
    _say("  c3 max err * 2^(n/2) = %.3g" % (err * 2 ** (c.n / 2)))
    assert err <= TOL * 2 ** (-c.n / 2)
    # unsliced plan agrees with the sliced one to rounding
    got0 = Q.plan(c).amplitudes(bits).cpu().numpy()[:, 0]
    assert np.abs(got0 - got).max() <= TOL * 2 ** (-c.n / 2)


@pytest.mark.parametrize("B,chunked", [(100, False), (1024, False), (1024, True)])
def test_c3_bucket_quad_tiles_against_stored_oracle(B, chunked):
    """5x6 depth 30 on the bucket path (level launches), whose two-input
    32-row tile buckets run as quad tiles (four tasks per work-group sharing
    one input's rows through LDS): a ragged batch of 100 (2 groups of 64, one
    work-group per block of tasks), the full 1024 (8 and more groups, blocks
    dealt by accelerator complex), and the full batch with 2 sliced variables
    as batch columns; against the stored FP64 state-vector amplitudes."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c3_5x6_d30")
    ref = np.load(os.path.join(GOLDEN, "c3_5x6_d30_amps.npy"), allow_pickle=False)[:B]
    _say("case c3 5x6 d30 ordering 1 level launches B=%d sliced=%d" % (B, 2 if chunked else 0))
    kw = dict(min_sliced_vars=2) if chunked else {}
    p = Q.plan(c, ordering=1, tree_exec=1, out_c128=True, **kw)
    info = p.info(1)
    assert sum(bk["quad"] for bk in info["buckets"]) >= 2 and sum(info["level_quad"]) > 0
    got = p.amplitudes(bits[:B]).cpu().numpy()[:, 0]
    err = np.abs(got - ref).max() * 2 ** (c.n / 2)
    _say("  max err * 2^(n/2) = %.3g" % err)
    assert err <= TOL


def test_6x7_quad_tile_forms_agree_across_batches():
    """6x7 depth 27 on the bucket path: its largest level runs the quad tiles
    with two bitstrings per lane (results beyond the last-level cache) at a
    pitch of 1024, including a batch of 900 (15 groups of 64: the last pair of
    groups half past the batch), and with one bitstring per lane at a pitch
    of 64.  Each bitstring's amplitude is the same bits whatever the batch (the
    same products in the same order)."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c5_6x7_d27")
    p = Q.plan(c, ordering=1, tree_exec=1)
    info = p.info(0)
    assert max(info["level_quad"]) * 32 * 1024 * 8 > 256 << 20
    _say("case 6x7 d27 ordering 1 B=1024, 900, 64")
    full = p.amplitudes(bits).cpu().numpy()[:, 0]
    assert np.isfinite(full).all()
    for B in (900, 64):
        part = p.amplitudes(bits[:B]).cpu().numpy()[:, 0]
        _say("  B=%d: max |diff| = %.3g" % (B, np.abs(part - full[:B]).max()))
        assert np.array_equal(part, full[:B])


BF16X3_TOL = 1e-4   # BF16x3 split precision, max |A - A_oracle| * 2^(n/2); frozen from the 5x6 depth-30 run (2.7e-5)


@pytest.mark.parametrize("policy,kind,tol", [(2, "mfma_f32", TOL), (4, "mfma_bf16x3", BF16X3_TOL)])
def test_c3_matrix_core_precisions_against_stored_oracle(policy, kind, tol):
    """5x6 depth 30, 1024 bitstrings, vertical order with 2 sliced variables
    summed in FP64: the steps the matrix-core kernel supports run on FP32 MFMA
    (policy 2, complex64 bound) or in BF16x3 split precision (policy 4, three
    bf16 products accumulated in FP32), against the stored FP64 state vector."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c3_5x6_d30")
    ref = np.load(os.path.join(GOLDEN, "c3_5x6_d30_amps.npy"), allow_pickle=False)
    _say("case c3 5x6 d30 B=1024 slices=2 policy %d" % policy)
    p = Q.plan(c, min_sliced_vars=2, out_c128=True, kernel_policy=policy)
    info = p.info(0)
    kinds = [s["kernel"] for s in info["steps"]]
    assert info["n_sliced"] == 2 and kinds.count(kind) >= 10
    got = p.amplitudes(bits).cpu().numpy()[:, 0]
    err = np.abs(got - ref) * 2 ** (c.n / 2)
    _say("  c3 %s (%d of %d steps): max err * 2^(n/2) = %.3g, median %.3g"
         % (kind, kinds.count(kind), len(kinds), err.max(), np.median(err)))
    assert err.max() <= tol


def test_graph_replays_match_eager():
    """Several circuits in one graph; every replay (with eager work and
    synchronisation in between) equals the eager result bit for bit."""
    import paper_1712_05384_amd as Q
    circs = [C.random_grid_circuit(3, 4, 12, 1), C.random_grid_circuit(4, 4, 16, 2),
             C.parameterised_circuit(3, 3, 10, 3), C.random_grid_circuit(2, 3, 8, 4)]
    opens = [(), (1, 5), (), (0,)]
    plans = [Q.plan(c, o) for c, o in zip(circs, opens)]
    bits = [C.random_bitstrings(c.n, B, i) for i, (c, B) in enumerate(zip(circs, (64, 130, 50, 1)))]
    gvs = [None if c.gate_vals is None else c.gate_vals.astype(np.complex64) for c in circs]
    eager = [p.amplitudes(b, g).cpu().numpy() for p, b, g in zip(plans, bits, gvs)]
    g = Q.Graph(plans, bits, gvs)
    for rep in range(3):
        outs = [o.cpu().numpy() for o in g.launch()]
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert np.array_equal(o, e), rep
        plans[1].amplitudes(bits[1])          # eager work between replays
        torch.cuda.synchronize()


def _pt_checks(amps, n, name):
    """E_x[N p(x)] = sum_x p(x) = 1 over uniform x holds for any circuit (Sec. II:
    probabilities of uniformly chosen bitstrings); the higher Porter-Thomas
    moments E[(Np)^2] = 2, E[log Np] = -gamma hold only once the circuit is deep
    enough for its size (App. B), so they are reported, not asserted."""
    m = len(amps)
    Np = (2.0 ** n) * np.abs(amps).astype(np.float64) ** 2
    assert abs(Np.mean() - 1) <= 5 * Np.std() / np.sqrt(m)
    _say("  %s: mean Np %.3f, mean (Np)^2 %.3f (PT 2), mean log Np %.3f (PT %.3f)"
         % (name, Np.mean(), (Np ** 2).mean(), np.log(Np).mean(), -EULER_GAMMA))


@pytest.mark.parametrize("kw,tol", [({}, TOL), ({"ordering": 1}, TOL), ({"precision": 1}, BF16X3_TOL)])
def test_c5_uneven_batch_in_one_graph(kw, tol):
    """4x5 d20, 5x5 d24, 6x6 d24, 6x7 d27 with 1024 bitstrings each, one graph, on the vertical order (complex64
    and BF16x3 steps) and the bucket path; the two larger circuits against the bucket oracle on 128 bitstrings
    spread over the batch."""
    import paper_1712_05384_amd as Q
    cs, bs = zip(*[C.workload(nm) for nm in C5])
    plans = [Q.plan(c, **kw) for c in cs]
    _say("case c5 graph of 4 circuits x 1024 %s" % kw)
    g = Q.Graph(plans, list(bs))
    outs = [o.cpu().numpy()[:, 0] for o in g.launch()]
    torch.cuda.synchronize()
    for nm, c, b, a in zip(C5, cs, bs, outs):
        if c.n <= 25:
            ref = oracle.sv_amplitudes(c.n, c.gates, None, b)
            err = np.abs(a - ref).max()
        else:
            idx = np.arange(0, len(b), len(b) // 128)[:128]
            ref = oracle.bucket_amplitudes(c.n, c.gates, None, b[idx])
            err = np.abs(a[idx] - ref).max()
        _say("  %s n=%d max err * 2^(n/2) = %.3g" % (nm, c.n, err * 2 ** (c.n / 2)))
        assert err <= tol * 2 ** (-c.n / 2)
        _pt_checks(a, c.n, nm)


def test_clifford_42_qubits_dyadic():
    """6x7 depth 27 with T -> S: same plan structure as the benchmark circuit,
    probabilities are 0 or 2^-k (App. F, end)."""
    import paper_1712_05384_amd as Q
    c, b = C.workload("c5_6x7_d27")
    k = C.clifford_variant(c)
    _say("case clifford 6x7 d27")
    a = Q.plan(k).amplitudes(b[:256], k.gate_vals.astype(np.complex64)).cpu().numpy()[:, 0]
    p = np.abs(a) ** 2
    nz = p[p > 2.0 ** (-k.n - 10)]
    assert len(nz) > 0
    e = np.log2(1 / nz)
    assert np.abs(e - np.round(e)).max() < 1e-3
