"""ctypes binding of liblooporbit.so: the C-ABI entry points under their own names.

Functions here marshal arguments only (tensors to device pointers, the current stream) and
raise LoopOrbitError on a non-zero status. All arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblooporbit.so")

LOOP_OK = 0
LOOP_EINVAL = -1
LOOP_ENOTSUP = -2
LOOP_EHIP = -3
LOOP_ENONFINITE = -4
LOOP_EWORKSPACE = -5
LOOP_EHANG = -6
EXPLICIT = 0
IMEX = 1
LAYOUT_RFFT = 0
LAYOUT_BAND = 1

# every symbol include/looporbit.h and include/ks_initial_loops.h declare
EXPORTS = [
    "loop_init", "loop_shutdown", "loop_workspace_bytes", "loop_workspace_init", "loop_residual",
    "loop_cost", "loop_adjoint_grad", "loop_cost_grad", "loop_to_band", "loop_from_band", "loop_cost_fwd",
    "loop_cost_bwd", "loop_update_grad", "loop_step", "loop_step_noalloc", "loop_set_resident",
    "loop_resident_supported", "loop_step_form", "loop_extrapolate", "loop_converge", "loop_step_xi",
    "loop_step_xi_workspace_bytes", "loop_expanded_grad", "loop_step_expanded", "loop_update", "loop_batch_create", "loop_batch_set_schedule", "loop_batch_set_streams", "loop_batch_set_wait_limit",
    "loop_batch_destroy",
    "loop_batch_info", "loop_batch_workspace_init", "loop_batch_step", "loop_batch_load", "loop_batch_pass",
    "loop_batch_store", "loop_batch_set_variant", "loop_batch_get_config", "loop_batch_autotune",
    "loop_status_sync", "loop_status_string", "loop_trace_start", "loop_trace_stop", "loop_trace_count",
    "loop_trace_get",
    "ks_integrate", "ks_recurrences", "ks_segments_to_loops",
]


class LoopOrbitError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_p = ctypes.c_void_p
_sz = ctypes.c_size_t

_SIGS = {
    "loop_init": ([], _i),
    "loop_shutdown": ([], _i),
    "loop_workspace_bytes": ([_i, _i, _i, ctypes.POINTER(_sz)], _i),
    "loop_workspace_init": ([_p, _sz, _p], _i),
    "loop_residual": ([_d, _i, _i, _i, _p, _p, _p, _p, _sz, _p], _i),
    "loop_cost": ([_d, _i, _i, _i, _p, _p, _p, _p, _sz, _p], _i),
    "loop_adjoint_grad": ([_d, _i, _i, _i, _p, _p, _p, _p, _p, _p, _sz, _p], _i),
    "loop_cost_grad": ([_d, _i, _i, _i, _p, _p, _p, _p, _p, _p, _sz, _p], _i),
    "loop_to_band": ([_i, _i, _i, _p, _p, _p], _i),
    "loop_from_band": ([_i, _i, _i, _p, _p, _p], _i),
    "loop_cost_fwd": ([_d, _i, _i, _i, _i, _p, _p, _p, _p, _p, _p, _p, _sz, _p], _i),
    "loop_cost_bwd": ([_d, _i, _i, _i, _i, _p, _p, _p, _p, _p, _p, _p, _p, _p, _sz, _p], _i),
    "loop_update_grad": ([_d, _i, _i, _i, _i, _p, _p, _p, _p, _d, _i, _p], _i),
    "loop_step": ([_d, _i, _i, _i, _p, _p, _d, _i, _i, _p, _p, _sz, _p], _i),
    "loop_step_noalloc": ([_d, _i, _i, _i, _p, _p, _d, _i, _i, _p, _p, _p], _i),
    "loop_update": ([_d, _i, _i, _i, _p, _p, _p, _p, _d, _i, _p], _i),
    "loop_batch_create": ([_i, ctypes.POINTER(_d), ctypes.POINTER(_i), ctypes.POINTER(_i),
                           ctypes.POINTER(_p)], _i),
    "loop_set_resident": ([_i], _i),
    "loop_resident_supported": ([_i, _i], _i),
    "loop_step_form": ([_i, _i, _i], _i),
    "loop_extrapolate": ([_i, _i, _i, _p, _p, _p, _p, _p, _p], _i),
    "loop_step_xi": ([_d, _i, _i, _i, _p, _p, _d, _i, _i, _p, _p, _sz, _p], _i),
    "loop_step_xi_workspace_bytes": ([_i, _i, _i, ctypes.POINTER(_sz)], _i),
    "loop_expanded_grad": ([_d, _i, _i, _i, _p, _p, _p, _p, _p, _p, _sz, _p], _i),
    "loop_step_expanded": ([_d, _i, _i, _i, _p, _p, _d, _i, _i, _p, _p, _sz, _p], _i),
    "loop_converge": ([_d, _i, _i, _i, _p, _p, _d, _i, _d, _i, ctypes.c_longlong, _i, _d,
                       ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_i), ctypes.POINTER(_d), _p, _sz, _p], _i),
    "loop_batch_set_schedule": ([_p, _i], _i),
    "loop_batch_set_streams": ([_p, _i], _i),
    "loop_batch_set_wait_limit": ([_p, _d], _i),
    "loop_batch_destroy": ([_p], _i),
    "loop_batch_info": ([_p, ctypes.POINTER(_sz), ctypes.POINTER(_sz), ctypes.POINTER(ctypes.c_longlong)], _i),
    "loop_batch_workspace_init": ([_p, _p, _sz, _p], _i),
    "loop_batch_step": ([_p, _p, _p, _d, _i, _i, _p, _p, _sz, _p], _i),
    "loop_batch_load": ([_p, _p, _p, _sz, _p], _i),
    "loop_batch_pass": ([_p, _i, _i, _i, _p, _d, _i, _p, _p, _sz, _p], _i),
    "loop_batch_store": ([_p, _p, _p, _sz, _p], _i),
    "loop_batch_set_variant": ([_p, _i, _i], _i),
    "loop_batch_get_config": ([_p, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)], _i),
    "loop_batch_autotune": ([_p, _p, _p, _i, ctypes.POINTER(_d), _p, _sz, _p], _i),
    "loop_status_sync": ([_p, _p], _i),
    "loop_trace_start": ([], _i),
    "loop_trace_stop": ([], _i),
    "loop_trace_count": ([], _i),
    "loop_trace_get": ([_i, ctypes.c_char_p, _i, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_d),
                        ctypes.POINTER(_d), ctypes.POINTER(_d)], _i),
    "loop_status_string": ([_i], ctypes.c_char_p),
    "ks_integrate": ([_d, _i, _i, _i, _d, _i, _i, _p, _p, _p, _i, _p], _i),
    "ks_recurrences": ([_i, _i, _p, _i, _d, _d, _d, _d, _i, _p, _p, _p], _i),
    "ks_segments_to_loops": ([_i, _i, _i, _p, _i, _i, _p, _d, _i, _i, _p, _p, _p], _i),
}


def lib():
    """Load liblooporbit.so (built in-tree). Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2007_06427_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().loop_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != LOOP_OK:
        raise LoopOrbitError(status, where)
