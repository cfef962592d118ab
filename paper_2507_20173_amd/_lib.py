"""ctypes declarations of libfsb's C ABI (include/fsb.h).

Loading fails loudly if the library has not been built: there is no CPU or
PyTorch fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PKG, "libfsb.so")

FSB_OK = 0
FSB_ERR_INVALID_ARG = -1
FSB_ERR_HIP = -2
FSB_ERR_UNSUPPORTED = -3
FSB_ERR_STATE = -4
FSB_ERR_DEVICE = -5

FSB_REDUCE_COMPENSATED = 0
FSB_REDUCE_NAIVE_F32 = 1
FSB_REDUCE_CRITICAL_F32 = 2
FSB_SWIM_GREEDY = 1
FSB_SWIM_WEIGHTED = 2
FSB_SCHED_STATIC = 0
FSB_SCHED_DYNAMIC = 1
FSB_SCHED_GUIDED = 2
FSB_RUN_PLAIN = 0
FSB_RUN_FUSED = 1
FSB_RUN_FUSED_PREV = 2
FSB_RUN_FUSED_LEAN = 3
FSB_RUN_FUSED_REGS = 4
FSB_RUN_FUSED_DEEP = 5
FSB_RUN_PLAIN_SPLIT = 6

FSB_KERNEL_SWIM_EVAL = 0
FSB_KERNEL_FEED_BARY = 1
FSB_KERNEL_FUSED = 2
FSB_KERNEL_INIT = 3
FSB_KERNEL_FEED_SWIM = 4
FSB_KERNEL_KINDS = 5
FSB_PROBE_FMA = 0
FSB_PROBE_PHILOX = 1
FSB_PROBE_MIXED = 2
FSB_PROBE_KINDS = 3


class fsb_config(ctypes.Structure):
    _fields_ = [("n_fish", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("pond_half", ctypes.c_float), ("swim_step", ctypes.c_float),
                ("w_init_lo", ctypes.c_float), ("w_init_hi", ctypes.c_float),
                ("w_min", ctypes.c_float), ("w_max", ctypes.c_float),
                ("reduce_mode", ctypes.c_uint32), ("history_len", ctypes.c_uint32),
                ("swim_rule", ctypes.c_uint32)]


class fsb_state(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("prev", ctypes.c_void_p), ("cur", ctypes.c_void_p)]


class fsb_record(ctypes.Structure):
    _fields_ = [("sum_w", ctypes.c_double), ("sum_wx", ctypes.c_double),
                ("sum_wy", ctypes.c_double), ("max_delta", ctypes.c_float),
                ("step_lo", ctypes.c_uint32)]


class fsb_tuning(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_uint32), ("fish_per_thread", ctypes.c_uint32),
                ("steps_per_launch", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("variant", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32),
                ("chunk_tiles", ctypes.c_uint32)]


class FsbError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} [code {code}]")
        self.code = code


_P = ctypes.c_void_p
_U32, _U64, _I = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_DP = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes)
PROTOTYPES = {
    "fsb_strerror": (ctypes.c_char_p, [_I]),
    "fsb_last_error": (ctypes.c_char_p, []),
    "fsb_abi_version": (_I, []),
    "fsb_workspace_bytes": (_I, [ctypes.POINTER(fsb_config), ctypes.POINTER(ctypes.c_size_t)]),
    "fsb_init": (_I, [ctypes.POINTER(fsb_config), fsb_state, _P, ctypes.c_size_t, _P,
                      ctypes.POINTER(_P)]),
    "fsb_attach": (_I, [ctypes.POINTER(fsb_config), fsb_state, _P, ctypes.c_size_t, _P, _U64,
                        ctypes.POINTER(_P)]),
    "fsb_step": (_I, [_P]),
    "fsb_run": (_I, [_P, _U64, _U32]),
    "fsb_step_displaced": (_I, [_P, _P, _P]),
    "fsb_barycentre": (_I, [_P, _DP, _DP]),
    "fsb_max_delta": (_I, [_P, ctypes.POINTER(ctypes.c_float)]),
    "fsb_history": (_I, [_P, _U64, _U64, ctypes.POINTER(fsb_record)]),
    "fsb_sync": (_I, [_P]),
    "fsb_step_index": (_I, [_P, ctypes.POINTER(_U64)]),
    "fsb_set_step_index": (_I, [_P, _U64]),
    "fsb_destroy": (_I, [_P]),
    "fsb_run_static": (_I, [ctypes.POINTER(fsb_config), fsb_state, _U64, _U64, _U32, _P, _P,
                            _P]),
    "fsb_profile_enable": (_I, [_P, _I]),
    "fsb_kernel_times": (_I, [_P, ctypes.POINTER(_U64), _DP]),
    "fsb_batch_workspace_bytes": (_I, [ctypes.POINTER(fsb_config), _U32, _P, _P,
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "fsb_batch_init": (_I, [ctypes.POINTER(fsb_config), _U32, _P, _P, _P, fsb_state, _U64, _P,
                            ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "fsb_batch_run": (_I, [_P, _U64, ctypes.POINTER(fsb_tuning)]),
    "fsb_batch_results": (_I, [_P, _DP, _DP, ctypes.POINTER(ctypes.c_float)]),
    "fsb_batch_barycentre": (_I, [_P, _DP, _DP]),
    "fsb_batch_history": (_I, [_P, _U64, ctypes.POINTER(fsb_record)]),
    "fsb_autotune": (_I, [_P, _U64, ctypes.POINTER(fsb_tuning)]),
    "fsb_batch_get_tuning": (_I, [_P, ctypes.POINTER(fsb_tuning)]),
    "fsb_batch_step_index": (_I, [_P, ctypes.POINTER(_U64)]),
    "fsb_batch_sync": (_I, [_P]),
    "fsb_batch_destroy": (_I, [_P]),
    "fsb_batch_profile_enable": (_I, [_P, _I]),
    "fsb_barrier_probe": (_I, [_P, _U32, _U32, _DP, ctypes.POINTER(_U32)]),
    "fsb_eval_sqrt": (_I, [_P, _P, _U64, _P]),
    "fsb_valu_probe": (_I, [_U32, _U32, _U32, _P, ctypes.c_size_t, _P, _DP,
                           ctypes.POINTER(_U64)]),
    "fsb_sweep_probe": (_I, [ctypes.POINTER(_P), _U64, _U32, _U32, _P, _DP]),
    "fsb_batch_kernel_times": (_I, [_P, ctypes.POINTER(_U64), _DP]),
}

_lib: ctypes.CDLL | None = None


def lib() -> ctypes.CDLL:
    """The loaded libfsb.so (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            raise ImportError(
                f"{LIBRARY} is missing: build it with `python -m paper_2507_20173_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIBRARY)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != FSB_OK:
        msg = lib().fsb_last_error().decode() or lib().fsb_strerror(rc).decode()
        raise FsbError(rc, msg)
