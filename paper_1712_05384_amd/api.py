"""Python binding of the C ABI (argument marshalling only; every step of the
amplitude path runs in the HIP kernels of libqgm.so)."""
from __future__ import annotations

import ctypes
import json

import numpy as np

from . import _native as N


def _circuit_struct(rows: int, cols: int, gates: np.ndarray, n_slots: int):
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 5))
    arr = (N.QgmGate * max(1, len(g)))()
    ctypes.memmove(arr, g.ctypes.data, g.nbytes)
    c = N.QgmCircuit(rows, cols, len(g), n_slots, ctypes.cast(arr, ctypes.POINTER(N.QgmGate)))
    return c, arr


class Plan:
    """A contraction plan (qgm_plan).  `circuit` is anything with rows, cols,
    gates (int32 [n_gates, 5]: kind, cycle, q0, q1, slot) and n_slots."""

    def __init__(self, circuit, open_qubits=(), *, min_sliced_vars: int = 0, max_rank: int = 0,
                 out_c128: bool = False, kernel_policy: int = 0, checkpoint_every: int = 0, ordering: int = 0,
                 chain_merge: bool = True, tree_exec: int = 0, tile: bool = True, order_finalists: int = 0,
                 order_restarts: int = 0, order_pick: int = 0, persist_spin: int = 0, precision: int = 0,
                 mem_budget: int = 0, checkpoint_budget: int = 0, compose: bool = True):
        L = N.lib()
        self._lib = L
        self._h = None
        self.n = int(circuit.rows * circuit.cols)
        self.n_slots = int(getattr(circuit, "n_slots", 0))
        self.open_qubits = [int(q) for q in open_qubits]
        self.out_c128 = bool(out_c128)
        cs, self._keep = _circuit_struct(circuit.rows, circuit.cols, circuit.gates, self.n_slots)
        opts = N.QgmPlanOpts()
        L.qgm_default_opts(ctypes.byref(opts))
        opts.min_sliced_vars = int(min_sliced_vars)
        opts.max_rank = int(max_rank)
        opts.out_c128 = 1 if out_c128 else 0
        opts.kernel_policy = int(kernel_policy)
        opts.checkpoint_every = int(checkpoint_every)
        opts.ordering = int(ordering)
        opts.no_chain_merge = 0 if chain_merge else 1
        opts.tree_exec = int(tree_exec)
        opts.no_tile = 0 if tile else 1
        opts.order_finalists = int(order_finalists)
        opts.order_restarts = int(order_restarts)
        opts.order_pick = int(order_pick)
        opts.persist_spin = int(persist_spin)
        opts.precision = int(precision)
        opts.mem_budget = int(mem_budget)
        opts.checkpoint_budget = int(checkpoint_budget)
        opts.no_compose = 0 if compose else 1
        self.ordering = int(ordering)
        op = (ctypes.c_int32 * max(1, len(self.open_qubits)))(*self.open_qubits)
        h = ctypes.c_void_p()
        N.check(L.qgm_plan(ctypes.byref(cs), op, len(self.open_qubits), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def info(self, detail: int = 0) -> dict:
        need = ctypes.c_size_t()
        self._lib.qgm_plan_info(self._h, detail, None, 0, ctypes.byref(need))
        buf = ctypes.create_string_buffer(need.value)
        N.check(self._lib.qgm_plan_info(self._h, detail, buf, need.value, None))
        return json.loads(buf.value.decode())

    def workspace_bytes(self, B: int) -> int:
        out = ctypes.c_uint64()
        N.check(self._lib.qgm_workspace_bytes(self._h, int(B), ctypes.byref(out)))
        return int(out.value)

    def amplitudes(self, bits, gate_vals=None, *, out=None, workspace=None, stream=None):
        """Amplitudes for a batch of bitstrings on the current CUDA/HIP device.

        bits: torch tensor (int64 or uint64 bit patterns) or numpy uint64 array.
        gate_vals: complex64 tensor [n_slots, 2, 2] (moved to the device), or None.
        Returns complex64 (or complex128) tensor [B, 2^n_open]."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if isinstance(bits, np.ndarray):
            bits = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64))
        if bits.dtype not in (torch.int64, torch.uint64):
            raise TypeError("bits must be a 64-bit integer tensor")
        bits = bits.to(dev).contiguous()
        B = int(bits.shape[0])
        n_out = 1 << len(self.open_qubits)
        odt = torch.complex128 if self.out_c128 else torch.complex64
        if out is None:
            out = torch.empty((B, n_out), dtype=odt, device=dev)
        elif out.dtype != odt or tuple(out.shape) != (B, n_out) or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, shape or layout")
        gv = None
        if self.n_slots:
            if gate_vals is None:
                raise ValueError("this circuit reads gate_vals")
            gv = torch.as_tensor(gate_vals).to(dev, torch.complex64).contiguous()
            if tuple(gv.shape) != (self.n_slots, 2, 2):
                raise ValueError("gate_vals must be [n_slots, 2, 2]")
        need = self.workspace_bytes(B)
        if workspace is None:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        if workspace.numel() < need:
            raise ValueError("workspace too small")
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        N.check(self._lib.qgm_amplitudes(self._h, None if gv is None else gv.data_ptr(), bits.data_ptr(), B,
                                         out.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                         ctypes.c_void_p(stream.cuda_stream)))
        return out

    def check(self, stream=None) -> None:
        """qgm_plan_check: synchronise the stream and raise QgmError if a
        persistent launch of this plan gave up since the last check."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        N.check(self._lib.qgm_plan_check(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def backward_workspace_bytes(self, B: int) -> int:
        out = ctypes.c_uint64()
        N.check(self._lib.qgm_backward_workspace_bytes(self._h, int(B), ctypes.byref(out)))
        return int(out.value)

    def backward(self, bits, grad_amps, gate_vals=None, *, workspace=None, stream=None, want_amps=True,
                 gate_grads=None, amps_out=None):
        """Gradient with respect to gate_vals of a real loss whose torch gradient
        with respect to the amplitudes is grad_amps ([B, 2^n_open] complex).
        Returns (amps or None, gate_grads [n_slots, 2, 2] complex64); gate_grads
        and amps_out, when given, are device tensors the call writes instead of
        allocating."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if isinstance(bits, np.ndarray):
            bits = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64))
        bits = bits.to(dev).contiguous()
        B = int(bits.shape[0])
        n_out = 1 << len(self.open_qubits)
        g = torch.as_tensor(grad_amps).to(dev, torch.complex64).reshape(B, n_out).contiguous()
        gv = None
        if self.n_slots:
            if gate_vals is None:
                raise ValueError("this circuit reads gate_vals")
            gv = torch.as_tensor(gate_vals).to(dev, torch.complex64).contiguous()
            if tuple(gv.shape) != (self.n_slots, 2, 2):
                raise ValueError("gate_vals must be [n_slots, 2, 2]")
        if gate_grads is not None:
            if tuple(gate_grads.shape) != (self.n_slots, 2, 2) or gate_grads.dtype != torch.complex64 \
                    or not gate_grads.is_contiguous():
                raise ValueError("gate_grads must be a contiguous complex64 [n_slots, 2, 2] tensor")
            grads = gate_grads
        else:
            grads = torch.zeros((max(self.n_slots, 1), 2, 2), dtype=torch.complex64, device=dev)
        odt = torch.complex128 if self.out_c128 else torch.complex64
        if amps_out is not None:
            if tuple(amps_out.shape) != (B, n_out) or amps_out.dtype != odt or not amps_out.is_contiguous():
                raise ValueError("amps_out must be a contiguous [B, 2^n_open] tensor of the plan's output type")
            amps = amps_out
        else:
            amps = torch.empty((B, n_out), dtype=odt, device=dev) if want_amps else None
        need = self.backward_workspace_bytes(B)
        if workspace is None:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        if workspace.numel() < need:
            raise ValueError("workspace too small")
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        N.check(self._lib.qgm_backward(self._h, None if gv is None else gv.data_ptr(), bits.data_ptr(), B,
                                       g.data_ptr(), None if amps is None else amps.data_ptr(),
                                       grads.data_ptr() if self.n_slots else None,
                                       workspace.data_ptr(), workspace.numel(), ctypes.c_void_p(stream.cuda_stream)))
        return amps, grads[:self.n_slots]

    def autotune(self, bits, gate_vals=None, *, allow_bf16x3: bool = False, cache_path=None, stream=None):
        """Times the candidate kernels of every step on this device and keeps
        the fastest (qgm_autotune).  Returns the per-step kernel names."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if isinstance(bits, np.ndarray):
            bits = torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint64).view(np.int64))
        bits = bits.to(dev).contiguous()
        B = int(bits.shape[0])
        gv = None
        if self.n_slots:
            gv = torch.as_tensor(gate_vals).to(dev, torch.complex64).contiguous()
        ws = torch.empty(max(self.workspace_bytes(B), 256), dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        N.check(self._lib.qgm_autotune(self._h, None if gv is None else gv.data_ptr(), bits.data_ptr(), B,
                                       ws.data_ptr(), ws.numel(), ctypes.c_void_p(stream.cuda_stream),
                                       1 if allow_bf16x3 else 0,
                                       None if cache_path is None else str(cache_path).encode()))
        return [s["kernel"] for s in self.info(0)["steps"]]

    def set_timing(self, enable: bool) -> None:
        N.check(self._lib.qgm_plan_set_timing(self._h, 1 if enable else 0))

    def timings(self) -> tuple[list[float], int]:
        """Accumulated ms of [boundary, G build, elimination steps, output] and the call count."""
        ms = (ctypes.c_double * 4)()
        n = ctypes.c_int64()
        N.check(self._lib.qgm_plan_timings(self._h, ms, ctypes.byref(n)))
        return list(ms), int(n.value)

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.qgm_plan_destroy(self._h)
            self._h = None


class Graph:
    """One HIP graph replaying the amplitude computation of several
    (plan, bits, gate_vals) batches, one concurrent branch per circuit
    (qgm_graph_create).  Buffers are allocated here and fixed for the graph's
    life; launch() recomputes self.outs[i] from self.bits[i]."""

    def __init__(self, plans, bits_list, gate_vals_list=None):
        import torch
        self._lib = N.lib()
        self._h = None
        dev = torch.device("cuda", torch.cuda.current_device())
        n = len(plans)
        self.plans = list(plans)
        self.bits, self.outs, self.workspaces, self.gate_vals = [], [], [], []
        for i, p in enumerate(self.plans):
            b = bits_list[i]
            if isinstance(b, np.ndarray):
                b = torch.from_numpy(np.ascontiguousarray(b, dtype=np.uint64).view(np.int64))
            b = b.to(dev).contiguous()
            self.bits.append(b)
            B = int(b.shape[0])
            odt = torch.complex128 if p.out_c128 else torch.complex64
            self.outs.append(torch.empty((B, 1 << len(p.open_qubits)), dtype=odt, device=dev))
            self.workspaces.append(torch.empty(max(p.workspace_bytes(B), 256), dtype=torch.uint8, device=dev))
            gv = None if gate_vals_list is None else gate_vals_list[i]
            self.gate_vals.append(None if gv is None else torch.as_tensor(gv).to(dev, torch.complex64).contiguous())
        VP = ctypes.c_void_p * n
        ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        hp = VP(*[p.handle.value for p in self.plans])
        gp = VP(*[ptr(g) for g in self.gate_vals])
        bp = VP(*[ptr(b) for b in self.bits])
        Bs = (ctypes.c_int64 * n)(*[int(b.shape[0]) for b in self.bits])
        op = VP(*[ptr(o) for o in self.outs])
        wp = VP(*[ptr(w) for w in self.workspaces])
        wb = (ctypes.c_uint64 * n)(*[w.numel() for w in self.workspaces])
        h = ctypes.c_void_p()
        N.check(self._lib.qgm_graph_create(n, hp, gp, bp, Bs, op, wp, wb, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        N.check(self._lib.qgm_graph_launch(self._h, ctypes.c_void_p(stream.cuda_stream)))
        return self.outs

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.qgm_graph_destroy(self._h)
            self._h = None


_PAULI = {"X": 10, "Y": 11, "Z": 12}


def expectation_circuit(circuit, paulis):
    """The circuit whose amplitude at bitstring 0 is <0|U^dag O U|0> for the
    Pauli string O = {qubit: "X" | "Y" | "Z"} (qgm_expectation_circuit: U on
    O's backward light cone, O, the inverses in reverse order)."""
    from .circuits import Circuit
    items = sorted(paulis.items())
    qs = (ctypes.c_int32 * len(items))(*[int(q) for q, _ in items])
    ks = (ctypes.c_int32 * len(items))(*[_PAULI[str(k).upper()] for _, k in items])
    cs, keep = _circuit_struct(circuit.rows, circuit.cols, circuit.gates, int(getattr(circuit, "n_slots", 0)))
    L = N.lib()
    n = ctypes.c_int32()
    st = L.qgm_expectation_circuit(ctypes.byref(cs), len(items), qs, ks, None, 0, ctypes.byref(n))
    if st != N.QGM_E_OOM or n.value == 0:
        N.check(st)
    out = (N.QgmGate * max(1, n.value))()
    N.check(L.qgm_expectation_circuit(ctypes.byref(cs), len(items), qs, ks, out, n.value, ctypes.byref(n)))
    g = np.array([(x.kind, x.cycle, x.q0, x.q1, x.slot) for x in out[:n.value]], dtype=np.int32).reshape(-1, 5)
    return Circuit(circuit.rows, circuit.cols, g, None, f"{getattr(circuit, 'name', '')}<O>")


def expectation(circuit, paulis, *, ordering: int = 1, **plan_opts):
    """<0|U^dag O U|0> (complex; real up to rounding) on the GPU: the amplitude at
    bitstring 0 of expectation_circuit(circuit, paulis)."""
    c2 = expectation_circuit(circuit, paulis)
    p = plan(c2, ordering=ordering, **plan_opts)
    return p.amplitudes(np.zeros(1, dtype=np.uint64)).reshape(-1)[0]


def xeb_workspace(B: int, device=None):
    """A device workspace for xeb / sample_from_set over B amplitudes (allocate once, pass to every call)."""
    import torch
    wsb = ctypes.c_uint64()
    N.check(N.lib().qgm_xeb_workspace_bytes(int(B), ctypes.byref(wsb)))
    return torch.empty(max(int(wsb.value), 256), dtype=torch.uint8, device=device or "cuda")


def xeb(amps, n_qubits: int, *, stream=None, workspace=None, out=None):
    """Cross-entropy statistics of a batch of amplitudes (qgm_xeb, App. B): a
    float64 device tensor [sum log p, sum p, sum p log p, zeros, cross entropy
    (Eq. (cee)), fidelity (Eq. (ae), Porter-Thomas H_0 and H), entropy from a
    uniform set (App. C), (2^n / B) sum p]."""
    import torch
    a = amps.reshape(-1)
    if a.dtype not in (torch.complex64, torch.complex128) or not a.is_cuda:
        raise TypeError("amps must be a complex64 or complex128 CUDA tensor")
    a = a.contiguous()
    L = N.lib()
    B = int(a.numel())
    ws = workspace if workspace is not None else xeb_workspace(B, a.device)
    if out is None:
        out = torch.empty(8, dtype=torch.float64, device=a.device)
    s = stream if stream is not None else torch.cuda.current_stream(a.device)
    N.check(L.qgm_xeb(a.data_ptr(), 1 if a.dtype == torch.complex128 else 0, B, int(n_qubits), out.data_ptr(),
                      ws.data_ptr(), ws.numel(), ctypes.c_void_p(s.cuda_stream)))
    return out


def prob_sums(amps, *, out=None, stream=None):
    """FP64 sum over each row of |amps|^2 (qgm_prob_sums, Sec. III.A): amps is
    the [B, 2^n_open] complex64/complex128 device tensor of a set of amplitudes
    per bitstring; returns float64 [B] (each at most 1; exactly 1 with every
    qubit open)."""
    import torch
    if amps.dim() != 2 or amps.dtype not in (torch.complex64, torch.complex128) or not amps.is_cuda:
        raise TypeError("amps must be a [B, 2^n_open] complex64 or complex128 CUDA tensor")
    B, n_out = int(amps.shape[0]), int(amps.shape[1])
    n_open = n_out.bit_length() - 1
    if n_out != 1 << n_open:
        raise ValueError("the second dimension of amps must be a power of two")
    a = amps.contiguous()
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=a.device)
    elif out.dtype != torch.float64 or out.numel() != B or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of B entries")
    s = stream if stream is not None else torch.cuda.current_stream(a.device)
    N.check(N.lib().qgm_prob_sums(a.data_ptr(), 1 if a.dtype == torch.complex128 else 0, B, n_open, out.data_ptr(),
                                  ctypes.c_void_p(s.cuda_stream)))
    return out


def sample_from_set(amps, uniforms, *, stream=None, workspace=None, out=None):
    """Indices drawn from a set of bitstrings with probability p_j / sum p
    (qgm_sample_set, App. C); uniforms: float64 device tensor in [0, 1), one
    per draw (the caller's random numbers)."""
    import torch
    a = amps.reshape(-1).contiguous()
    if a.dtype not in (torch.complex64, torch.complex128) or not a.is_cuda:
        raise TypeError("amps must be a complex64 or complex128 CUDA tensor")
    u = uniforms.reshape(-1).to(a.device, torch.float64).contiguous()
    L = N.lib()
    B, m = int(a.numel()), int(u.numel())
    ws = workspace if workspace is not None else xeb_workspace(B, a.device)
    idx = out if out is not None else torch.empty(max(m, 1), dtype=torch.int64, device=a.device)
    s = stream if stream is not None else torch.cuda.current_stream(a.device)
    N.check(L.qgm_sample_set(a.data_ptr(), 1 if a.dtype == torch.complex128 else 0, B, u.data_ptr(), m,
                             idx.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.c_void_p(s.cuda_stream)))
    return idx[:m]


def plan(circuit, open_qubits=(), **opts) -> Plan:
    return Plan(circuit, open_qubits, **opts)


def amplitudes(p: Plan, bits, gate_vals=None, **kw):
    return p.amplitudes(bits, gate_vals, **kw)


def sync_check(stream=None) -> None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    N.check(N.lib().qgm_sync_check(ctypes.c_void_p(stream.cuda_stream)))


def _autograd_function():
    import torch

    class QGMAmplitudes(torch.autograd.Function):
        """amps = QGMAmplitudes.apply(gate_vals, bits, plan): complex64 [B, 2^n_open]
        differentiable with respect to gate_vals [n_slots, 2, 2] (complex64).
        The backward pass calls qgm_backward, which recomputes the forward with
        checkpoints instead of keeping the frontier tensors alive in between."""

        @staticmethod
        def forward(ctx, gate_vals, bits, plan):
            ctx.plan = plan
            ctx.save_for_backward(gate_vals, bits)
            return plan.amplitudes(bits, gate_vals.detach())

        @staticmethod
        def backward(ctx, grad_out):
            gate_vals, bits = ctx.saved_tensors
            _, grads = ctx.plan.backward(bits, grad_out, gate_vals.detach(), want_amps=False)
            return grads.to(gate_vals.dtype), None, None

    return QGMAmplitudes


_QGM_FN = None


def amplitudes_autograd(gate_vals, bits, p: Plan):
    """Differentiable amplitudes (see QGMAmplitudes)."""
    global _QGM_FN
    if _QGM_FN is None:
        _QGM_FN = _autograd_function()
    return _QGM_FN.apply(gate_vals, bits, p)
