"""ctypes declarations of libqgm.so (include/qgm.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqgm.so")

QGM_OK, QGM_E_INVALID, QGM_E_UNSUPPORTED, QGM_E_OOM, QGM_E_HIP, QGM_E_INTERNAL = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "QGM_OK", -1: "QGM_E_INVALID", -2: "QGM_E_UNSUPPORTED", -3: "QGM_E_OOM",
                -4: "QGM_E_HIP", -5: "QGM_E_INTERNAL"}

# Every symbol include/qgm.h declares.
EXPORTED = ("qgm_default_opts", "qgm_plan", "qgm_plan_info", "qgm_workspace_bytes", "qgm_amplitudes",
            "qgm_backward_workspace_bytes", "qgm_backward", "qgm_graph_create", "qgm_graph_launch",
            "qgm_graph_destroy", "qgm_autotune", "qgm_plan_set_timing", "qgm_plan_timings", "qgm_plan_destroy", "qgm_last_error",
            "qgm_sync_check", "qgm_xeb_workspace_bytes", "qgm_xeb", "qgm_sample_set", "qgm_expectation_circuit",
            "qgm_prob_sums", "qgm_plan_check", "qgm_amplitudes_static")


class QgmGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("cycle", ctypes.c_int32), ("q0", ctypes.c_int32),
                ("q1", ctypes.c_int32), ("slot", ctypes.c_int32)]


class QgmCircuit(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("n_slots", ctypes.c_int32), ("gates", ctypes.POINTER(QgmGate))]


class QgmPlanOpts(ctypes.Structure):
    _fields_ = [("ordering", ctypes.c_int32), ("precision", ctypes.c_int32), ("kernel_policy", ctypes.c_int32),
                ("min_sliced_vars", ctypes.c_int32), ("out_c128", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("checkpoint_every", ctypes.c_int32), ("no_chain_merge", ctypes.c_int32),
                ("tree_exec", ctypes.c_int32), ("no_tile", ctypes.c_int32),
                ("order_finalists", ctypes.c_int32), ("order_restarts", ctypes.c_int32),
                ("order_pick", ctypes.c_int32), ("persist_spin", ctypes.c_int32),
                ("mem_budget", ctypes.c_uint64), ("checkpoint_budget", ctypes.c_uint64),
                ("no_compose", ctypes.c_int32), ("reserved0", ctypes.c_int32)]
QGM_PREC_C64, QGM_PREC_BF16X3 = 0, 1


class QgmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Loads libqgm.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1712_05384_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.qgm_default_opts.argtypes = [ctypes.POINTER(QgmPlanOpts)]
        L.qgm_default_opts.restype = None
        L.qgm_plan.argtypes = [ctypes.POINTER(QgmCircuit), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                               ctypes.POINTER(QgmPlanOpts), ctypes.POINTER(P)]
        L.qgm_plan_info.argtypes = [P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t,
                                    ctypes.POINTER(ctypes.c_size_t)]
        L.qgm_workspace_bytes.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
        L.qgm_amplitudes.argtypes = [P, P, P, ctypes.c_int64, P, P, ctypes.c_uint64, P]
        L.qgm_backward_workspace_bytes.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
        L.qgm_backward.argtypes = [P, P, P, ctypes.c_int64, P, P, P, P, ctypes.c_uint64, P]
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.qgm_graph_create.argtypes = [ctypes.c_int32, PP, PP, PP, ctypes.POINTER(ctypes.c_int64), PP, PP,
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(P)]
        L.qgm_graph_launch.argtypes = [P, P]
        L.qgm_graph_destroy.argtypes = [P]
        L.qgm_graph_destroy.restype = None
        L.qgm_autotune.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_uint64, P, ctypes.c_int32, ctypes.c_char_p]
        L.qgm_plan_set_timing.argtypes = [P, ctypes.c_int32]
        L.qgm_plan_timings.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.qgm_plan_destroy.argtypes = [P]
        L.qgm_plan_destroy.restype = None
        L.qgm_last_error.argtypes = []
        L.qgm_last_error.restype = ctypes.c_char_p
        L.qgm_sync_check.argtypes = [P]
        L.qgm_xeb_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
        L.qgm_xeb.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_uint64, P]
        L.qgm_sample_set.argtypes = [P, ctypes.c_int32, ctypes.c_int64, P, ctypes.c_int64, P, P, ctypes.c_uint64, P]
        L.qgm_prob_sums.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P, P]
        L.qgm_plan_check.argtypes = [P, P]
        L.qgm_amplitudes_static.argtypes = [P, P, P, ctypes.c_int64, P, P]
        I32P = ctypes.POINTER(ctypes.c_int32)
        L.qgm_expectation_circuit.argtypes = [ctypes.POINTER(QgmCircuit), ctypes.c_int32, I32P, I32P,
                                              ctypes.POINTER(QgmGate), ctypes.c_int32, I32P]
        for f in (L.qgm_plan, L.qgm_plan_info, L.qgm_workspace_bytes, L.qgm_amplitudes, L.qgm_sync_check,
                  L.qgm_plan_set_timing, L.qgm_plan_timings, L.qgm_backward_workspace_bytes, L.qgm_backward,
                  L.qgm_graph_create, L.qgm_graph_launch, L.qgm_autotune, L.qgm_xeb_workspace_bytes, L.qgm_xeb,
                  L.qgm_sample_set, L.qgm_expectation_circuit, L.qgm_prob_sums,
                  L.qgm_plan_check, L.qgm_amplitudes_static):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != QGM_OK:
        raise QgmError(status, lib().qgm_last_error().decode(errors="replace"))
