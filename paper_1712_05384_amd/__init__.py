"""MI355X (gfx950) amplitude engine for random grid circuits viewed as complex
undirected graphical models (arXiv:1712.05384), behind the C ABI of
include/qgm.h.

    from paper_1712_05384_amd import circuits, plan
    c, bits = circuits.workload("c2_5x5_d25")
    p = plan(c)                       # host-side planner
    amps = p.amplitudes(bits)         # HIP kernels on the current device

Importing the package does not load the native library; the first plan()
does, and raises if libqgm.so has not been built.
"""
from .api import Plan, Graph, plan, amplitudes, amplitudes_autograd, sync_check, xeb, sample_from_set, prob_sums, expectation_circuit, expectation  # noqa: F401
from . import circuits  # noqa: F401
