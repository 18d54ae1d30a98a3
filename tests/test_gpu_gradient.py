"""GPU gradients (adjoint of the elimination steps) against the FP64 oracle's
adjoint-state gradient, the exact per-gate scaling identity, and finite
differences.  Loss: L = sum_x log |A_x|^2 (m times the negative cross-entropy
estimator of App. B, Eq. (cee)); torch convention dL/dRe U + i dL/dIm U."""
import sys

import numpy as np
import pytest

import oracle
from paper_1712_05384_amd import circuits as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GTOL = 1e-4   # per entry, relative to the largest gate gradient (and the Frobenius error over all gates)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_grad(got, ref, tol=GTOL):
    """Entry by entry: |G - G_ref| <= tol * max_g ||G_ref,g||_F for every entry of
    every gate (one gate off by more than that fails, however many gates there
    are); the relative Frobenius error over all gates is printed as a summary."""
    scale = np.sqrt((np.abs(ref) ** 2).sum(axis=(1, 2))).max()
    err = np.abs(got - ref)
    worst = int(np.unravel_index(np.argmax(err), err.shape)[0])
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say("  worst gate %d: max |dG| / max ||G_ref|| = %.3g (frobenius over all gates %.3g)"
         % (worst, err.max() / scale, rel))
    assert err.max() <= tol * scale, (worst, got[worst], ref[worst])
    assert rel <= tol


def _gpu_grad(c, bits, **kw):
    import paper_1712_05384_amd as Q
    p = Q.plan(c, **kw)
    gv = torch.tensor(c.gate_vals.astype(np.complex64), device="cuda")
    amps = p.amplitudes(bits, gv)
    g_amps = 2.0 / torch.conj(amps)
    a2, grads = p.backward(bits, g_amps, gv)
    torch.cuda.synchronize()
    return amps.cpu().numpy()[:, 0], a2.cpu().numpy()[:, 0], grads.cpu().numpy()


@pytest.mark.parametrize("rows,cols,depth,seed,kw", [
    (2, 2, 6, 1, {}), (3, 3, 10, 2, {}), (3, 4, 12, 3, {"checkpoint_every": 2}),
    (4, 4, 12, 4, {"checkpoint_every": 1}), (3, 4, 10, 5, {"min_sliced_vars": 2}),
    (4, 4, 16, 6, {"kernel_policy": 2}), (4, 3, 14, 7, {})])
def test_gradient_matches_oracle(rows, cols, depth, seed, kw):
    c = C.parameterised_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, 100, seed)
    _say("case %s %s" % (c.name, kw))
    amps, amps2, got = _gpu_grad(c, bits, **kw)
    vals = c.gate_vals.astype(np.complex64).astype(np.complex128)
    _, ref = oracle.sv_log_prob_gradient(c.n, c.gates, vals, bits)
    assert np.array_equal(amps, amps2)
    _check_grad(got, ref)
    # exact identity: sum_ab U[a,b] conj(G[a,b]) = 2m for every gate (A is linear in U)
    ident = np.einsum("sab,sab->s", vals, got.conj())
    assert np.abs(ident - 2 * len(bits)).max() <= 1e-3 * 2 * len(bits)


def test_c4_workload_gradient():
    """5x5 depth 20, every single-qubit gate U(theta, n), 256 bitstrings."""
    c, bits = C.workload("c4_5x5_d20_U")
    _say("case c4 5x5 d20 B=256")
    amps, _, got = _gpu_grad(c, bits)
    vals = c.gate_vals.astype(np.complex64).astype(np.complex128)
    ref_amps, ref = oracle.sv_log_prob_gradient(c.n, c.gates, vals, bits)
    assert np.abs(amps - ref_amps).max() <= 1e-5 * 2 ** (-c.n / 2)
    _check_grad(got, ref)


def test_autograd_function_and_finite_difference():
    import paper_1712_05384_amd as Q
    c = C.parameterised_circuit(3, 3, 10, 9)
    bits = torch.from_numpy(C.random_bitstrings(c.n, 64, 9).view(np.int64)).cuda()
    p = Q.plan(c)
    gv = torch.tensor(c.gate_vals.astype(np.complex64), device="cuda", requires_grad=True)
    amps = Q.amplitudes_autograd(gv, bits, p)
    loss = torch.log(amps.abs() ** 2).sum()
    loss.backward()
    g = gv.grad.detach().cpu().numpy()
    # coarse finite difference in complex64 (smoke level, h = 1e-2)
    rng = np.random.default_rng(0)
    for _ in range(6):
        s, a, b = rng.integers(0, c.n_slots), rng.integers(0, 2), rng.integers(0, 2)
        for unit in (1.0, 1j):
            vp = gv.detach().clone(); vp[s, a, b] += 1e-2 * unit
            vm = gv.detach().clone(); vm[s, a, b] -= 1e-2 * unit
            lp = torch.log(p.amplitudes(bits, vp).abs() ** 2).sum().item()
            lm = torch.log(p.amplitudes(bits, vm).abs() ** 2).sum().item()
            fd = (lp - lm) / 2e-2
            an = g[s, a, b].real if unit == 1.0 else g[s, a, b].imag
            assert abs(fd - an) <= 0.05 * max(1.0, abs(an)), (s, a, b, unit, fd, an)


# --- adjoint of the bucket path (ordering 1) -------------------------------------------------


@pytest.mark.parametrize("rows,cols,depth,seed,kw", [
    (1, 1, 4, 11, {}), (2, 2, 6, 1, {}), (3, 3, 10, 2, {}), (3, 4, 12, 3, {}), (4, 4, 12, 4, {}),
    (4, 3, 14, 7, {"chain_merge": False}), (4, 4, 16, 6, {"out_c128": True}), (3, 4, 12, 5, {"B": 130})])
def test_tree_gradient_matches_oracle(rows, cols, depth, seed, kw):
    """Adjoint through the buckets (merged chains, absorbed buckets, tail
    levels) against the FP64 adjoint-state gradient; the identity
    sum_ab U conj(G) = 2m; amplitudes of the backward call equal the forward's.
    B = 130: three groups of 64 in an arena of row pitch 256."""
    kw = dict(kw)
    B = kw.pop("B", 100)
    c = C.parameterised_circuit(rows, cols, depth, seed)
    bits = C.random_bitstrings(c.n, B, seed)
    _say("case tree %s %s" % (c.name, kw))
    amps, amps2, got = _gpu_grad(c, bits, ordering=1, **kw)
    vals = c.gate_vals.astype(np.complex64).astype(np.complex128)
    ref_amps, ref = oracle.sv_log_prob_gradient(c.n, c.gates, vals, bits)
    assert np.abs(amps2 - ref_amps).max() <= 1e-5 * 2 ** (-c.n / 2)
    assert np.abs(amps2 - amps).max() <= 1e-5 * 2 ** (-c.n / 2)
    _check_grad(got, ref)
    ident = np.einsum("sab,sab->s", vals, got.conj())
    assert np.abs(ident - 2 * len(bits)).max() <= 1e-3 * 2 * len(bits)


def test_tree_c4_workload_gradient_and_vertical_agreement():
    """5x5 depth 20, every single-qubit gate U(theta, n), 256 bitstrings: the
    bucket-path gradient against the oracle and against the vertical path."""
    c, bits = C.workload("c4_5x5_d20_U")
    _say("case tree c4 5x5 d20 B=256")
    _, amps, got = _gpu_grad(c, bits, ordering=1)
    vals = c.gate_vals.astype(np.complex64).astype(np.complex128)
    ref_amps, ref = oracle.sv_log_prob_gradient(c.n, c.gates, vals, bits)
    assert np.abs(amps - ref_amps).max() <= 1e-5 * 2 ** (-c.n / 2)
    _check_grad(got, ref)
    _, _, vert = _gpu_grad(c, bits)
    _check_grad(got, vert)


def test_tree_gradient_diagonal_gates_and_autograd():
    """Diagonal parameterised gates (UD: every T of a random circuit becomes
    diag(1, e^{i phi}) with its own slot, the first two sharing one) on the
    bucket path, through the autograd function."""
    import paper_1712_05384_amd as Q
    base = C.random_grid_circuit(3, 3, 12, 21)
    gates = base.gates.copy()
    rng = np.random.default_rng(5)
    vals = []
    n_t = 0
    for i in range(len(gates)):
        if gates[i, 0] == C.T:
            gates[i, 0] = C.UD
            if n_t == 1:
                gates[i, 4] = 0   # the second diagonal gate shares the first one's slot
            else:
                gates[i, 4] = len(vals)
                vals.append(np.diag([1.0, np.exp(1j * rng.uniform(0, 2 * np.pi))]))
            n_t += 1
    kk = C.Circuit(base.rows, base.cols, gates, np.array(vals, dtype=np.complex128), base.name + "_ud")
    assert kk.n_slots >= 3 and (gates[:, 4] == 0).sum() >= 2
    bits = C.random_bitstrings(kk.n, 64, 21)
    _say("case tree diagonal slots %s (%d slots)" % (kk.name, kk.n_slots))
    _, amps, got = _gpu_grad(kk, bits, ordering=1)
    v128 = kk.gate_vals.astype(np.complex64).astype(np.complex128)
    ref_amps, ref = oracle.sv_log_prob_gradient(kk.n, kk.gates, v128, bits)
    assert np.abs(amps - ref_amps).max() <= 1e-5 * 2 ** (-kk.n / 2)
    _check_grad(got, ref)
    p = Q.plan(kk, ordering=1)
    gv = torch.tensor(kk.gate_vals.astype(np.complex64), device="cuda", requires_grad=True)
    bt = torch.from_numpy(bits.view(np.int64)).cuda()
    a = Q.amplitudes_autograd(gv, bt, p)
    torch.log(a.abs() ** 2).sum().backward()
    _check_grad(gv.grad.cpu().numpy(), got)


@pytest.mark.parametrize("ordering", [1, 0])
def test_backward_is_bitwise_repeatable(ordering):
    """Every sum of the adjoint runs in a fixed order (no floating-point
    atomics), so repeated qgm_backward calls on the same inputs give the same
    bits, including the phase factors' and the shared slots' sums."""
    import paper_1712_05384_amd as Q
    c, bits = C.workload("c4_5x5_d20_U")
    _say("case repeat backward ordering %d" % ordering)
    p = Q.plan(c, ordering=ordering)
    gv = torch.tensor(c.gate_vals.astype(np.complex64), device="cuda")
    amps = p.amplitudes(bits, gv)
    g_amps = 2.0 / torch.conj(amps)
    first = None
    for _ in range(4):
        a2, grads = p.backward(bits, g_amps, gv)
        torch.cuda.synchronize()
        cur = (a2.cpu().numpy().copy(), grads.cpu().numpy().copy())
        if first is None:
            first = cur
        else:
            assert np.array_equal(cur[0].view(np.uint32), first[0].view(np.uint32))
            assert np.array_equal(cur[1].view(np.uint32), first[1].view(np.uint32))
