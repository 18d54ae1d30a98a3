"""GPU parity of the bucket-elimination path (ordering 1: greedy treewidth
order) against the FP64 oracle, in both of its launch forms: one launch per
elimination-tree level (tree_exec 1) and one work-group per bitstring with
every result in LDS (tree_exec 3, the default when the plan fits).

Same tolerance as the vertical path: max |A_gpu - A_oracle| <= 1e-5 * 2^{-n/2}.
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


def _tree(c, **kw):
    import paper_1712_05384_amd as Q
    return Q.plan(c, ordering=1, **kw)


def _amps(p, bits, gate_vals=None):
    out = p.amplitudes(bits, gate_vals)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:, 0]


def test_app_d_tree():
    d = C.example_app_d()
    got = _amps(_tree(d), np.arange(4, dtype=np.uint64))
    assert np.allclose(got, [0.5, 0.5, 0.5, -0.5], atol=1e-7)


def test_tree_c1_full_batch():
    """4x4 depth 16, 64 bitstrings, with the chosen plan and with the first order's
    plan among 16 restarts per criterion (order_restarts = 16, order_finalists = 1),
    whose tail runs a tile bucket from LDS."""
    c, bits = C.workload("c1_4x4_d16")
    _say("case tree c1_4x4_d16 B=64")
    got = _amps(_tree(c), bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)
    p1 = _tree(c, order_restarts=16, order_finalists=1, compose=False)   # (composed leaves take that bucket)
    info = p1.info(1)
    assert any(bk["tile"] and bk["level"] >= info["tail_start"] for bk in info["buckets"])
    _say("case tree c1_4x4_d16 B=64 order_finalists=1")
    got1 = _amps(p1, bits)
    assert np.abs(got1 - ref).max() <= TOL * 2 ** (-c.n / 2)


@pytest.mark.parametrize("mode", [1, 3])
@pytest.mark.parametrize("B", [1, 5, 63, 64, 65, 130])
def test_tree_ragged_batches(B, mode):
    c = C.random_grid_circuit(3, 4, 12, 7)
    bits = C.random_bitstrings(c.n, B, 7)
    _say("case tree 3x4_d12 B=%d tree_exec %d" % (B, mode))
    got = _amps(_tree(c, tree_exec=mode), bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)


_RANDOM = [(1, 1, 3, 1), (2, 2, 1, 2), (1, 5, 12, 3), (4, 4, 24, 4), (3, 5, 20, 5), (4, 5, 16, 6), (5, 4, 30, 16)]


# the 5x4 depth-30 plan's factor tables exceed a work-group's LDS: level launches only
@pytest.mark.parametrize("rows,cols,depth,seed,mode", [r + (m,) for r in _RANDOM for m in (1, 3)
                                                       if not (m == 3 and r == (5, 4, 30, 16))])
def test_tree_random_circuits(rows, cols, depth, seed, mode):
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, 256, seed)
    _say("case tree %s B=256 tree_exec %d" % (c.name, mode))
    got = _amps(_tree(c, tree_exec=mode), bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)


@pytest.mark.parametrize("mode", [1, 3])
def test_tree_gate_values_and_c128(mode):
    c = C.parameterised_circuit(4, 4, 14, 8)
    bits = C.random_bitstrings(c.n, 128, 8)
    gv = c.gate_vals.astype(np.complex64)
    _say("case tree %s B=128 (gate_vals, complex128 out) tree_exec %d" % (c.name, mode))
    got = _amps(_tree(c, out_c128=True, tree_exec=mode), bits, torch.tensor(gv))
    assert got.dtype == np.complex128
    ref = oracle.sv_amplitudes(c.n, c.gates, gv.astype(np.complex128), bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)


def test_tree_qubit_without_non_diagonal_gates():
    """b^0 = b^d = 0 on a worldline without non-diagonal gates: amplitude 0 when x_q = 1."""
    g = np.array([(C.H, 0, 0, -1, -1), (C.CZ, 1, 0, 1, -1), (C.T, 2, 1, -1, -1), (C.H, 3, 0, -1, -1),
                  (C.H, 0, 2, -1, -1), (C.CZ, 4, 1, 2, -1), (C.XH, 5, 2, -1, -1)])
    c = C.Circuit(1, 3, g)
    bits = np.arange(8, dtype=np.uint64)
    got = _amps(_tree(c), bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    assert np.abs(got - ref).max() <= 1e-7


def test_tree_clifford_probabilities_dyadic_36_qubits():
    c = C.clifford_variant(C.random_grid_circuit(6, 6, 12, 11))
    bits = C.random_bitstrings(c.n, 256, 11)
    _say("case tree clifford 6x6_d12")
    got = _amps(_tree(c), bits, torch.tensor(c.gate_vals.astype(np.complex64)))
    p = np.abs(got) ** 2
    nz = p[p > 2.0 ** (-c.n - 8)]
    assert len(nz) > 0
    k = np.log2(1 / nz)
    assert np.abs(k - np.round(k)).max() < 1e-4


def test_tree_c2_full_size_and_vertical_agreement():
    """5x5 depth 25, 1024 bitstrings: the bucket path against the 2^25 state
    vector, and against the vertical path; the plan of the first order by
    symbolic cost among 16 restarts per criterion (which has a three-input tile)
    against the same state vector."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c2_5x5_d25")
    _say("case tree c2_5x5_d25 B=1024")
    got = _amps(_tree(c), bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    err = np.abs(got - ref).max()
    _say("  tree c2 max err * 2^(n/2) = %.3g" % (err * 2 ** (c.n / 2)))
    assert err <= TOL * 2 ** (-c.n / 2)
    vert = _amps(Q.plan(c), bits)
    assert np.abs(vert - got).max() <= TOL * 2 ** (-c.n / 2)
    p1 = _tree(c, order_restarts=16, order_finalists=1, compose=False)   # (composed leaves take the tile)
    assert any(bk["tile"] == 2 for bk in p1.info(1)["buckets"])
    _say("case tree c2_5x5_d25 B=1024 order_finalists=1")
    got1 = _amps(p1, bits)
    assert np.abs(got1 - ref).max() <= TOL * 2 ** (-c.n / 2)


def test_tree_c3_against_stored_oracle():
    """5x6 depth 30, 1024 bitstrings, no slicing needed (largest bucket result
    rank 16), complex128 output, against the stored FP64 state-vector values."""
    c, bits = C.workload("c3_5x6_d30")
    ref = np.load(os.path.join(GOLDEN, "c3_5x6_d30_amps.npy"), allow_pickle=False)
    _say("case tree c3 5x6 d30 B=1024")
    got = _amps(_tree(c, out_c128=True), bits)
    err = np.abs(got - ref).max()
    _say("  tree c3 max err * 2^(n/2) = %.3g" % (err * 2 ** (c.n / 2)))
    assert err <= TOL * 2 ** (-c.n / 2)


def test_tree_c4_parameterised_workload():
    c, bits = C.workload("c4_5x5_d20_U")
    gv = c.gate_vals.astype(np.complex64)
    _say("case tree c4 5x5 d20 U B=256")
    got = _amps(_tree(c), bits, torch.tensor(gv))
    ref = oracle.sv_amplitudes(c.n, c.gates, gv.astype(np.complex128), bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)


def test_tree_repeat_calls_bitwise_identical():
    c, bits = C.workload("c1_4x4_d16")
    p = _tree(c)
    a = _amps(p, bits)
    for _ in range(3):
        assert np.array_equal(_amps(p, bits), a)


def test_tree_graph_mixed_with_vertical():
    """A HIP graph holding a bucket plan and a vertical plan replays to the eager results."""
    import paper_1712_05384_amd as Q
    c1 = C.random_grid_circuit(4, 4, 16, 2)
    c2 = C.parameterised_circuit(3, 3, 10, 3)
    plans = [_tree(c1), Q.plan(c2), _tree(c2)]
    bits = [C.random_bitstrings(c1.n, 130, 1), C.random_bitstrings(c2.n, 64, 2), C.random_bitstrings(c2.n, 64, 2)]
    gv2 = c2.gate_vals.astype(np.complex64)
    gvs = [None, gv2, gv2]
    eager = [p.amplitudes(b, g).cpu().numpy() for p, b, g in zip(plans, bits, gvs)]
    g = Q.Graph(plans, bits, gvs)
    for rep in range(3):
        outs = [o.cpu().numpy() for o in g.launch()]
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert np.array_equal(a, b), rep
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
    ref = oracle.sv_amplitudes(c1.n, c1.gates, None, bits[0])
    assert np.abs(eager[0][:, 0] - ref).max() <= TOL * 2 ** (-c1.n / 2)
    assert np.abs(eager[2] - eager[1]).max() <= TOL * 2 ** (-c2.n / 2)


def _oracle_open(c, bits, open_qubits, gate_vals=None):
    psi = oracle.sv_state(c.n, c.gates, gate_vals)
    out = np.zeros((len(bits), 1 << len(open_qubits)), dtype=np.complex128)
    for o in range(1 << len(open_qubits)):
        x = np.asarray(bits, dtype=np.uint64).copy()
        for i, q in enumerate(open_qubits):
            x = (x & ~np.uint64(1 << q)) | np.uint64(((o >> i) & 1) << q)
        out[:, o] = psi[x.astype(np.int64)]
    return out


@pytest.mark.parametrize("rows,cols,depth,seed,open_qubits,B", [(3, 4, 12, 7, (0,), 64), (3, 4, 12, 7, (5, 2), 130),
                                                               (4, 4, 16, 3, (11, 3, 7), 70),
                                                               (4, 5, 16, 6, (0, 4, 8, 12, 16, 19), 100),
                                                               (3, 3, 10, 2, tuple(range(9)), 5)])
def test_tree_open_qubits(rows, cols, depth, seed, open_qubits, B):
    """Sets of amplitudes on the bucket path: every completion of the open qubits,
    against the state vector and against the vertical path."""
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, B, seed)
    _say("case tree open %s open=%s B=%d" % (c.name, open_qubits, B))
    out = Q.plan(c, open_qubits, ordering=1).amplitudes(bits)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = _oracle_open(c, bits, open_qubits)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)
    vert = Q.plan(c, open_qubits).amplitudes(bits).cpu().numpy()
    assert np.abs(vert - got).max() <= TOL * 2 ** (-c.n / 2)


def test_tree_open_qubits_gate_values_c128_chain_and_zero_bit():
    import paper_1712_05384_amd as Q
    # gate values and complex128 output
    c = C.parameterised_circuit(4, 4, 14, 8)
    bits = C.random_bitstrings(c.n, 66, 8)
    gv = c.gate_vals.astype(np.complex64)
    got = Q.plan(c, (3, 12), ordering=1, out_c128=True).amplitudes(bits, torch.tensor(gv)).cpu().numpy()
    assert got.dtype == np.complex128
    assert np.abs(got - _oracle_open(c, bits, (3, 12), gv.astype(np.complex128))).max() <= TOL * 2 ** (-c.n / 2)
    # more than 8 results on the open qubits: a chain of buckets over them
    n = 18
    g = [(C.H, 0, q, -1, -1) for q in range(n)] + [(C.CZ, 1, 2 * i, 2 * i + 1, -1) for i in range(9)] + \
        [(C.XH, 2, q, -1, -1) for q in range(n)]
    c2 = C.Circuit(1, n, np.array(g))
    oq = tuple(range(0, n, 2))
    bits2 = C.random_bitstrings(n, 64, 5)
    got2 = Q.plan(c2, oq, ordering=1).amplitudes(bits2).cpu().numpy()
    assert np.abs(got2 - _oracle_open(c2, bits2, oq)).max() <= TOL * 2 ** (-n / 2)
    # an open qubit without non-diagonal gates: amplitude 0 when its output bit is set
    g3 = np.array([(C.H, 0, 0, -1, -1), (C.CZ, 1, 0, 1, -1), (C.T, 2, 1, -1, -1), (C.H, 3, 0, -1, -1),
                   (C.H, 0, 2, -1, -1), (C.CZ, 4, 1, 2, -1), (C.XH, 5, 2, -1, -1)])
    c3 = C.Circuit(1, 3, g3)
    bits3 = np.arange(8, dtype=np.uint64)
    got3 = Q.plan(c3, (2, 1), ordering=1).amplitudes(bits3).cpu().numpy()
    assert np.abs(got3 - _oracle_open(c3, bits3, (2, 1))).max() <= 1e-7


def test_tree_open_qubits_backward_rejected():
    import paper_1712_05384_amd as Q
    from paper_1712_05384_amd import _native as N
    c = C.parameterised_circuit(3, 3, 8, 1)
    p = Q.plan(c, (0,), ordering=1)
    bits = C.random_bitstrings(c.n, 64, 1)
    gv = torch.tensor(c.gate_vals.astype(np.complex64), device="cuda")
    bd = torch.from_numpy(bits.view(np.int64)).cuda()
    with pytest.raises(N.QgmError) as e:
        p.backward(bd, torch.ones(64, 2, dtype=torch.complex64, device="cuda"), gv)
    assert e.value.status == N.QGM_E_UNSUPPORTED


def _shifted(c, off):
    return [(int(r[0]), int(r[1]), int(r[2]) + off, int(r[3]) + off if r[3] >= 0 else -1, int(r[4])) for r in c.gates]


def _tail_table_inputs(info):
    maker = {bk["out_tensor"]: bk for bk in info["buckets"]}
    return sum(1 for bk in info["buckets"] if bk["level"] >= info["tail_start"]
               for t in bk["in_tensors"] if maker.get(t, {}).get("table_leaf"))


@pytest.mark.parametrize("rows,cols,depth,seed", [(3, 4, 16, 2), (4, 4, 16, 4)])
def test_tree_tail_reads_leaf_tables(rows, cols, depth, seed):
    """Buckets of the last levels (run from LDS in one work-group per group)
    whose inputs include leaf tables read from the table area."""
    c = C.random_grid_circuit(rows, cols, depth, seed)
    p = _tree(c, tree_exec=1, compose=False)   # (composed leaves take those buckets)
    assert _tail_table_inputs(p.info(1)) > 0
    bits = C.random_bitstrings(c.n, 130, seed)
    _say("case tree tail leaf tables %s" % c.name)
    got = _amps(p, bits)
    assert np.abs(got - oracle.sv_amplitudes(c.n, c.gates, None, bits)).max() <= TOL * 2 ** (-c.n / 2)


def test_tree_tail_many_phase_factors_60_qubits():
    """More factors without free variables than the tail stages in LDS (the rest
    are evaluated from their records): a 3x4 block on qubits 0..11 and H then T
    on qubits 12..59, whose amplitude factor is <x|TH|0> = (1, e^{i pi/4})[x] / sqrt 2."""
    blk = C.random_grid_circuit(3, 4, 12, 3)
    n = 60
    g = _shifted(blk, 0) + [(C.H, 0, q, -1, -1) for q in range(12, n)] + [(C.T, 1, q, -1, -1) for q in range(12, n)]
    c = C.Circuit(1, n, np.array(g, dtype=np.int32))
    p = _tree(c, order_restarts=16, order_finalists=1, tree_exec=1)   # this plan has tail levels
    info = p.info(0)
    assert info["n_phase"] > 64 and info["tail_levels"] > 0
    bits = C.random_bitstrings(n, 200, 11)
    _say("case tree tail 60 qubits, %d phase factors" % info["n_phase"])
    got = _amps(p, bits)
    psi = oracle.sv_state(12, blk.gates, None)
    ref = psi[(bits & np.uint64(0xFFF)).astype(np.int64)].copy()
    for q in range(12, n):
        xq = ((bits >> np.uint64(q)) & np.uint64(1)).astype(bool)
        ref *= np.where(xq, np.exp(1j * np.pi / 4), 1.0) / np.sqrt(2.0)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-n / 2)


def test_tree_tail_with_final_from_the_arena():
    """Two components: the shallow one's rank-0 result is made before the tail
    (the tail reads it from the arena), the deep one's in the tail (LDS)."""
    a = C.random_grid_circuit(2, 2, 6, 5)
    b = C.random_grid_circuit(4, 4, 16, 6)
    c = C.Circuit(1, 20, np.array(_shifted(a, 0) + _shifted(b, 4), dtype=np.int32))
    p = _tree(c, tree_exec=1)
    info = p.info(1)
    made = {bk["out_tensor"]: bk["level"] for bk in info["buckets"]}
    levels = [made[f] for f in info["finals"]]
    assert info["tail_levels"] > 0 and min(levels) < info["tail_start"] <= max(levels)
    bits = C.random_bitstrings(20, 100, 12)
    _say("case tree tail final from arena")
    got = _amps(p, bits)
    assert np.abs(got - oracle.sv_amplitudes(20, c.gates, None, bits)).max() <= TOL * 2 ** (-20 / 2)


@pytest.mark.parametrize("rows,cols,depth,seed,B", [(4, 4, 16, 3, 130), (5, 5, 20, 8, 64), (4, 5, 20, 2, 200)])
def test_tree_tile_units(rows, cols, depth, seed, B):
    """Tile units (two-input buckets, 8 rows per unit from 4 + 2 input rows) against
    the oracle, and the same plan without them."""
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(rows, cols, depth, seed)
    p = Q.plan(c, ordering=1, tree_exec=1)
    n_tiles = sum(1 for bk in p.info(1)["buckets"] if bk["tile"])
    bits = C.random_bitstrings(c.n, B, seed)
    _say("case tree tiles %s (%d tile buckets) B=%d" % (c.name, n_tiles, B))
    got = _amps(p, bits)
    assert np.abs(got - oracle.sv_amplitudes(c.n, c.gates, None, bits)).max() <= TOL * 2 ** (-c.n / 2)
    plain = _amps(Q.plan(c, ordering=1, tile=False, tree_exec=1), bits)
    assert np.abs(got - plain).max() <= TOL * 2 ** (-c.n / 2)


def test_tree_tile_units_c3_and_parameterised():
    """5x6 depth 30 (six tile buckets) against the stored oracle amplitudes, and
    a circuit with gate values whose plan has tiles."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c3_5x6_d30")
    p = Q.plan(c, ordering=1)
    assert sum(1 for bk in p.info(1)["buckets"] if bk["tile"]) >= 3
    ref = np.load(os.path.join(GOLDEN, "c3_5x6_d30_amps.npy"), allow_pickle=False)
    got = _amps(p, bits)
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)
    cp, _ = C.workload("c4_5x5_d20_U")
    pp = Q.plan(cp, ordering=1, tree_exec=1)
    assert sum(1 for bk in pp.info(1)["buckets"] if bk["tile"]) >= 1
    bits2 = C.random_bitstrings(cp.n, 70, 8)
    gv = cp.gate_vals.astype(np.complex64)
    got2 = _amps(pp, bits2, torch.tensor(gv))
    ref2 = oracle.sv_amplitudes(cp.n, cp.gates, gv.astype(np.complex128), bits2)
    assert np.abs(got2 - ref2).max() <= TOL * 2 ** (-cp.n / 2)


@pytest.mark.parametrize("B", [1, 65, 200])
def test_tree_tile_units_ragged_batches_c128(B):
    """Tile plans at batches that do not fill the arena's power-of-two pitch, with
    complex128 output, and a circuit with gate values whose plan has tiles."""
    import paper_1712_05384_amd as Q
    c = C.random_grid_circuit(4, 5, 20, 2)
    p = Q.plan(c, ordering=1, out_c128=True, tree_exec=1, compose=False)   # (composed leaves take the tiles)
    assert any(bk["tile"] for bk in p.info(1)["buckets"])
    bits = C.random_bitstrings(c.n, B, 40 + B)
    _say("case tree tiles ragged B=%d c128" % B)
    got = p.amplitudes(bits).cpu().numpy()[:, 0]
    assert got.dtype == np.complex128
    assert np.abs(got - oracle.sv_amplitudes(c.n, c.gates, None, bits)).max() <= TOL * 2 ** (-c.n / 2)
    cp, _ = C.workload("c4_5x5_d20_U")
    pp = Q.plan(cp, ordering=1, tree_exec=1)
    gv = cp.gate_vals.astype(np.complex64)
    bits2 = C.random_bitstrings(cp.n, B, 50 + B)
    got2 = _amps(pp, bits2, torch.tensor(gv))
    ref2 = oracle.sv_amplitudes(cp.n, cp.gates, gv.astype(np.complex128), bits2)
    assert np.abs(got2 - ref2).max() <= TOL * 2 ** (-cp.n / 2)


@pytest.mark.parametrize("name", ["c2_5x5_d25", "c5_4x5_d20", "c5_5x5_d24"])
def test_tree_lds_workloads_against_state_vector(name):
    """Full-size workloads (1024 bitstrings) in the LDS-resident launch against
    the FP64 state vector, and against the level launches of the same plan."""
    c, bits = C.workload(name)
    p = _tree(c, tree_exec=3)
    assert p.info(0)["lds_ok"] == 1
    _say("case tree lds %s B=%d" % (name, len(bits)))
    got = _amps(p, bits)
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits)
    err = np.abs(got - ref).max()
    _say("  lds %s max err * 2^(n/2) = %.3g" % (name, err * 2 ** (c.n / 2)))
    assert err <= TOL * 2 ** (-c.n / 2)
    lev = _amps(_tree(c, tree_exec=1), bits)
    assert np.abs(got - lev).max() <= TOL * 2 ** (-c.n / 2)


def test_tree_lds_36_qubits_and_gradient_workload():
    """6x6 depth 24 (44 KiB of LDS per work-group) against the level launches and
    the FP64 bucket oracle on 8 bitstrings; the parameterised 5x5 depth-20
    circuit (tables from gate values each call) against the state vector."""
    c, bits = C.workload("c5_6x6_d24")
    p = _tree(c, tree_exec=3)
    assert p.info(0)["lds_ok"] == 1
    _say("case tree lds c5_6x6_d24 B=%d" % len(bits))
    got = _amps(p, bits)
    lev = _amps(_tree(c, tree_exec=1), bits)
    assert np.abs(got - lev).max() <= TOL * 2 ** (-c.n / 2)
    ref = oracle.bucket_amplitudes(c.n, c.gates, None, bits[:8])
    assert np.abs(got[:8] - ref).max() <= TOL * 2 ** (-c.n / 2)
    cp, bp = C.workload("c4_5x5_d20_U")
    gv = cp.gate_vals.astype(np.complex64)
    _say("case tree lds c4 B=%d" % len(bp))
    got2 = _amps(_tree(cp, tree_exec=3, out_c128=True), bp, torch.tensor(gv))
    ref2 = oracle.sv_amplitudes(cp.n, cp.gates, gv.astype(np.complex128), bp)
    assert np.abs(got2 - ref2).max() <= TOL * 2 ** (-cp.n / 2)


@pytest.mark.parametrize("B", [0, 1, 3, 65, 2051])
def test_tree_lds_edge_batches(B):
    """Empty, ragged and multi-round batches in the LDS-resident launch of the
    composed 5x5 depth-25 plan: no launch and an empty result for 0
    bitstrings; otherwise the amplitudes of the FP64 state vector, and each
    bitstring's amplitude equal to its amplitude in a batch of 1024 (2051
    work-groups take more than one round of the GPU, so the launch reads its
    job records from memory instead of LDS)."""
    c, bits = C.workload("c2_5x5_d25")
    if B > len(bits):
        bits = np.concatenate([bits, C.random_bitstrings(c.n, B - len(bits), 5)])
    p = _tree(c, tree_exec=3)
    _say("case tree lds edge B=%d" % B)
    got = _amps(p, bits[:B])
    assert got.shape[0] == B
    if B == 0:
        return
    ref = oracle.sv_amplitudes(c.n, c.gates, None, bits[:B])
    assert np.abs(got - ref).max() <= TOL * 2 ** (-c.n / 2)
    assert np.array_equal(got[:min(B, 1024)], _amps(p, bits[:1024])[:min(B, 1024)])


def test_tree_lds_repeat_and_graph():
    """The LDS launch gives the same bits on repeated calls and in a graph replay."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c2_5x5_d25")
    p = _tree(c, tree_exec=3)
    a = p.amplitudes(bits).cpu().numpy()
    for _ in range(2):
        assert np.array_equal(p.amplitudes(bits).cpu().numpy(), a)
    g = Q.Graph([p], [bits], [None])
    for _ in range(3):
        out = g.launch()[0].cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(out, a)


@pytest.mark.gpu
def test_tree_lds_null_workspace():
    """A circuit without gate values needs no workspace in the LDS launch: the C-ABI takes NULL for it and gives
    the same amplitudes; a plan that needs a workspace rejects NULL with QGM_E_INVALID."""
    import ctypes
    from paper_1712_05384_amd import _native as N
    c, bits = C.workload("c2_5x5_d25")
    p = _tree(c, tree_exec=3)
    assert p.workspace_bytes(len(bits)) == 0
    a = p.amplitudes(bits).cpu().numpy()
    bd = torch.from_numpy(bits.view(np.int64)).cuda()
    out = torch.empty((len(bits), 1), dtype=torch.complex64, device="cuda")
    s = torch.cuda.current_stream()
    L = N.lib()
    N.check(L.qgm_amplitudes(p._h, None, bd.data_ptr(), len(bits), out.data_ptr(), None, 0,
                             ctypes.c_void_p(s.cuda_stream)))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), a)
    p1 = _tree(c, tree_exec=1)
    assert p1.workspace_bytes(len(bits)) > 0
    st = L.qgm_amplitudes(p1._h, None, bd.data_ptr(), len(bits), out.data_ptr(), None, 0,
                          ctypes.c_void_p(s.cuda_stream))
    assert st == N.QGM_E_INVALID
