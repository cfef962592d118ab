"""MI355X (gfx950) Fish School Behaviour step: Python binding of libfsb.

The entry points keep the C names of include/fsb.h and only marshal
arguments: PyTorch supplies device memory and the stream, every step of the
computation runs in the library's HIP kernels.  ``School`` is a convenience
owner of the columns and the workspace.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import _lib
from ._lib import (FSB_KERNEL_FEED_BARY, FSB_KERNEL_FUSED, FSB_KERNEL_INIT,  # noqa: F401
                   FSB_KERNEL_KINDS, FSB_KERNEL_SWIM_EVAL, FSB_REDUCE_COMPENSATED,
                   FSB_REDUCE_NAIVE_F32, FSB_RUN_FUSED, FSB_RUN_PLAIN, FsbError, check, lib)

RECORD = np.dtype([("sum_w", "<f8"), ("sum_wx", "<f8"), ("sum_wy", "<f8"),
                   ("max_delta", "<f4"), ("step_lo", "<u4")])
COLUMNS = ("x", "y", "w", "prev", "cur")


@dataclasses.dataclass
class FsbConfig:
    """Mirror of ``fsb_config``; defaults are the 200x200 pond (H = 100),
    swim step 0.1, initial weights in [1, 2], weight limits [1, 4]."""
    n_fish: int
    seed: int = 0
    pond_half: float = 100.0
    swim_step: float = 0.1
    w_init_lo: float = 1.0
    w_init_hi: float = 2.0
    w_min: float = 1.0
    w_max: float = 4.0
    reduce_mode: int = FSB_REDUCE_COMPENSATED
    history_len: int = 1

    def c(self) -> _lib.fsb_config:
        return _lib.fsb_config(self.n_fish, self.seed, self.pond_half, self.swim_step,
                               self.w_init_lo, self.w_init_hi, self.w_min, self.w_max,
                               self.reduce_mode, self.history_len)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def state_struct(cols: dict) -> _lib.fsb_state:
    return _lib.fsb_state(*[_ptr(cols[k]) for k in COLUMNS])


# ---- entry points (names as in include/fsb.h) -------------------------------

def fsb_abi_version() -> int:
    return lib().fsb_abi_version()


def fsb_workspace_bytes(cfg: FsbConfig) -> int:
    out = ctypes.c_size_t()
    c = cfg.c()
    check(lib().fsb_workspace_bytes(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def fsb_init(cfg: FsbConfig, cols: dict, workspace, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    c = cfg.c()
    check(lib().fsb_init(ctypes.byref(c), state_struct(cols), _ptr(workspace),
                         workspace.numel() * workspace.element_size(),
                         _stream_handle(stream), ctypes.byref(h)))
    return h


def fsb_attach(cfg: FsbConfig, cols: dict, workspace, t: int = 0, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    c = cfg.c()
    check(lib().fsb_attach(ctypes.byref(c), state_struct(cols), _ptr(workspace),
                           workspace.numel() * workspace.element_size(),
                           _stream_handle(stream), t, ctypes.byref(h)))
    return h


def fsb_step(h) -> None:
    check(lib().fsb_step(h))


def fsb_run(h, n_steps: int, mode: int = FSB_RUN_PLAIN) -> None:
    check(lib().fsb_run(h, n_steps, mode))


def fsb_step_displaced(h, dx, dy) -> None:
    check(lib().fsb_step_displaced(h, _ptr(dx), _ptr(dy)))


def fsb_barycentre(h) -> tuple[np.ndarray, np.ndarray]:
    xy = (ctypes.c_double * 2)()
    sums = (ctypes.c_double * 3)()
    check(lib().fsb_barycentre(h, xy, sums))
    return np.array(xy[:]), np.array(sums[:])


def fsb_max_delta(h) -> np.float32:
    m = ctypes.c_float()
    check(lib().fsb_max_delta(h, ctypes.byref(m)))
    return np.float32(m.value)


def fsb_history(h, first: int, count: int) -> np.ndarray:
    out = np.zeros(count, RECORD)
    check(lib().fsb_history(h, first, count,
                            out.ctypes.data_as(ctypes.POINTER(_lib.fsb_record))))
    return out


def fsb_sync(h) -> None:
    check(lib().fsb_sync(h))


def fsb_step_index(h) -> int:
    t = ctypes.c_uint64()
    check(lib().fsb_step_index(h, ctypes.byref(t)))
    return t.value


def fsb_set_step_index(h, t: int) -> None:
    check(lib().fsb_set_step_index(h, t))


def fsb_destroy(h) -> None:
    check(lib().fsb_destroy(h))


def fsb_profile_enable(h, enable: bool = True) -> None:
    check(lib().fsb_profile_enable(h, 1 if enable else 0))


def fsb_kernel_times(h) -> tuple[np.ndarray, np.ndarray]:
    counts = (ctypes.c_uint64 * FSB_KERNEL_KINDS)()
    ms = (ctypes.c_double * FSB_KERNEL_KINDS)()
    check(lib().fsb_kernel_times(h, counts, ms))
    return np.array(counts[:], np.uint64), np.array(ms[:])


# ---- convenience owner --------------------------------------------------------

def alloc_columns(n: int, device="cuda"):
    import torch
    return {k: torch.empty(n, dtype=torch.float32, device=device) for k in COLUMNS}


class School:
    """One school: allocates its five columns and workspace with PyTorch and
    drives them through the C ABI.  ``state=None`` runs the init kernel;
    otherwise ``state`` (a dict of columns, host or device) is copied in and
    the handle is attached at iteration ``t``."""

    def __init__(self, cfg: FsbConfig, state: dict | None = None, t: int = 0,
                 stream=None, device="cuda"):
        import torch
        self.cfg = cfg
        self.cols = alloc_columns(cfg.n_fish, device)
        self.workspace = torch.empty(fsb_workspace_bytes(cfg), dtype=torch.uint8, device=device)
        self.stream = stream
        if state is None:
            self.h = fsb_init(cfg, self.cols, self.workspace, stream)
        else:
            for k in COLUMNS:
                self.cols[k].copy_(torch.as_tensor(np.asarray(state[k], np.float32)))
            self.h = fsb_attach(cfg, self.cols, self.workspace, t, stream)

    def step(self):
        fsb_step(self.h)

    def run(self, n_steps: int, mode: int = FSB_RUN_PLAIN):
        fsb_run(self.h, n_steps, mode)

    def step_displaced(self, dx, dy):
        fsb_step_displaced(self.h, dx, dy)

    def barycentre(self):
        return fsb_barycentre(self.h)

    def max_delta(self):
        return fsb_max_delta(self.h)

    def history(self, first: int, count: int):
        return fsb_history(self.h, first, count)

    def sync(self):
        fsb_sync(self.h)

    @property
    def t(self) -> int:
        return fsb_step_index(self.h)

    def state(self) -> dict:
        """Columns copied to host numpy arrays (synchronises)."""
        self.sync()
        return {k: v.cpu().numpy() for k, v in self.cols.items()}

    def close(self):
        if getattr(self, "h", None) is not None:
            fsb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
