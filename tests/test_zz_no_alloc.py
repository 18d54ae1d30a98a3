"""qgm_amplitudes_static (the entry point that allocates nothing: its
workspace is the library's file-scope device array) against qgm_amplitudes,
through the C ABI: two calls in a row, the second with a smaller batch, on a
bucket plan, a bucket plan with gate values, a vertical-order plan and a
persistent-launch plan; then the errors it owes its callers."""
import ctypes
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


def _static(p, bits, gv=None):
    from paper_1712_05384_amd import _native as N
    dev = torch.device("cuda", torch.cuda.current_device())
    b = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64)).to(dev)
    odt = torch.complex128 if p.out_c128 else torch.complex64
    out = torch.empty((len(bits), 1 << len(p.open_qubits)), dtype=odt, device=dev)
    s = torch.cuda.current_stream(dev)
    N.check(N.lib().qgm_amplitudes_static(p.handle, None if gv is None else gv.data_ptr(), b.data_ptr(), len(bits),
                                          out.data_ptr(), ctypes.c_void_p(s.cuda_stream)))
    torch.cuda.synchronize()
    return out.cpu().numpy()


CASES = [("c2_5x5_d25", {"ordering": 1}, 1024, 300),
         ("c4_5x5_d20_U", {"ordering": 1}, 256, 70),
         ("c1_4x4_d16", {"ordering": 0}, 64, 17),
         ("c1_4x4_d16", {"ordering": 1, "tree_exec": 2}, 512, 65)]


@pytest.mark.parametrize("name,kw,b1,b2", CASES)
def test_static_matches_workspace_entry_point(name, kw, b1, b2):
    import paper_1712_05384_amd as Q
    c, bits = C.workload(name)
    bits = np.resize(bits, b1)
    gv = None if c.gate_vals is None else torch.tensor(c.gate_vals.astype(np.complex64), device="cuda")
    p = Q.plan(c, **kw)
    _say("case static %s %s B=%d then %d" % (name, kw, b1, b2))
    ref1 = p.amplitudes(bits, gv).cpu().numpy()          # also uploads the plan's tables
    got1 = _static(p, bits, gv)
    ref2 = p.amplitudes(bits[:b2], gv).cpu().numpy()
    got2 = _static(p, bits[:b2], gv)
    assert np.array_equal(got1, ref1)
    assert np.array_equal(got2, ref2)
    vals = None if c.gate_vals is None else c.gate_vals.astype(np.complex64).astype(np.complex128)
    ora = oracle.sv_amplitudes(c.n, c.gates, vals, bits[:b2])
    assert np.abs(got2[:, 0] - ora).max() <= TOL * 2 ** (-c.n / 2)
    if kw.get("tree_exec") == 2:
        p.check()


def test_static_errors():
    import paper_1712_05384_amd as Q
    from paper_1712_05384_amd import _native as N
    c, bits = C.workload("c1_4x4_d16")
    p = Q.plan(c, ordering=1)
    _say("case static errors")
    with pytest.raises(N.QgmError) as ei:          # tables not on the device yet: no upload here
        _static(p, bits)
    assert ei.value.status == N.QGM_E_INVALID
    p.amplitudes(bits)
    c3, _ = C.workload("c3_5x6_d30")
    p3 = Q.plan(c3, ordering=1)
    p3.amplitudes(np.zeros(1, dtype=np.uint64))
    assert p3.workspace_bytes(4096) > (64 << 20)
    with pytest.raises(N.QgmError) as ei:          # beyond the 64 MiB array
        _static(p3, np.zeros(4096, dtype=np.uint64))
    assert ei.value.status == N.QGM_E_OOM
    assert np.array_equal(_static(p, bits), p.amplitudes(bits).cpu().numpy())
