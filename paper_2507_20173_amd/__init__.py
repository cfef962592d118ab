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
from ._lib import (FSB_KERNEL_FEED_BARY, FSB_KERNEL_FEED_SWIM, FSB_KERNEL_FUSED,  # noqa: F401
                   FSB_KERNEL_INIT, FSB_KERNEL_KINDS, FSB_KERNEL_SWIM_EVAL, FSB_REDUCE_COMPENSATED,
                   FSB_REDUCE_CRITICAL_F32, FSB_REDUCE_NAIVE_F32, FSB_RUN_FUSED,
                   FSB_RUN_FUSED_DEEP, FSB_RUN_FUSED_LEAN, FSB_RUN_FUSED_PREV,
                   FSB_RUN_FUSED_REGS, FSB_RUN_PLAIN, FSB_RUN_PLAIN_SPLIT,
                   FSB_PROBE_FMA, FSB_PROBE_KINDS, FSB_PROBE_MIXED, FSB_PROBE_PHILOX,
                   FSB_SCHED_DYNAMIC, FSB_SCHED_GUIDED, FSB_SCHED_STATIC, FSB_SWIM_GREEDY,
                   FSB_SWIM_WEIGHTED,
                   FsbError, check, lib)

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
    swim_rule: int = 0

    def c(self) -> _lib.fsb_config:
        return _lib.fsb_config(self.n_fish, self.seed, self.pond_half, self.swim_step,
                               self.w_init_lo, self.w_init_hi, self.w_min, self.w_max,
                               self.reduce_mode, self.history_len, self.swim_rule)


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


def fsb_run_static(cfg: FsbConfig, cols: dict, t: int, n_steps: int, mode: int, records,
                   status=None, stream=None) -> None:
    """Iterations t .. t + n_steps - 1 of the school in ``cols`` with the
    library's static scratch (no workspace): ``records`` is a device uint8
    tensor of cfg.history_len records, ``status`` an optional device int32
    word for the kernels' failure flags."""
    assert records.numel() * records.element_size() >= cfg.history_len * RECORD.itemsize
    c = cfg.c()
    check(lib().fsb_run_static(ctypes.byref(c), state_struct(cols), t, n_steps, mode,
                               _ptr(records), _ptr(status), _stream_handle(stream)))


def fsb_profile_enable(h, every: int = 1) -> None:
    """Time every `every`-th launch of each kernel kind (0 = off)."""
    check(lib().fsb_profile_enable(h, int(every)))


def fsb_kernel_times(h) -> tuple[np.ndarray, np.ndarray]:
    counts = (ctypes.c_uint64 * FSB_KERNEL_KINDS)()
    ms = (ctypes.c_double * FSB_KERNEL_KINDS)()
    check(lib().fsb_kernel_times(h, counts, ms))
    return np.array(counts[:], np.uint64), np.array(ms[:])


# ---- batch entry points ---------------------------------------------------------

def _u64_array(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.uint64))


def fsb_batch_workspace_bytes(common: FsbConfig, starts, sizes) -> int:
    st, sz = _u64_array(starts), _u64_array(sizes)
    out = ctypes.c_size_t()
    c = common.c()
    check(lib().fsb_batch_workspace_bytes(ctypes.byref(c), sz.size, st.ctypes.data,
                                          sz.ctypes.data, ctypes.byref(out)))
    return out.value


def fsb_batch_init(common: FsbConfig, starts, sizes, seeds, cols: dict, workspace,
                   stream=None) -> ctypes.c_void_p:
    st, sz, sd = _u64_array(starts), _u64_array(sizes), _u64_array(seeds)
    h = ctypes.c_void_p()
    c = common.c()
    check(lib().fsb_batch_init(ctypes.byref(c), sz.size, st.ctypes.data, sz.ctypes.data,
                               sd.ctypes.data, state_struct(cols), cols["x"].numel(),
                               _ptr(workspace), workspace.numel() * workspace.element_size(),
                               _stream_handle(stream), ctypes.byref(h)))
    return h


def tuning(block_size=1024, fish_per_thread=8, steps_per_launch=100, blocks_per_cu=0, variant=0,
           schedule=FSB_SCHED_STATIC, chunk_tiles=0):
    return _lib.fsb_tuning(block_size, fish_per_thread, steps_per_launch, blocks_per_cu, variant,
                           schedule, chunk_tiles)


def tuning_dict(t: _lib.fsb_tuning) -> dict:
    return {k: getattr(t, k) for k, _ in _lib.fsb_tuning._fields_}


def fsb_batch_run(b, n_steps: int, tune: _lib.fsb_tuning | None = None) -> None:
    check(lib().fsb_batch_run(b, n_steps, ctypes.byref(tune) if tune is not None else None))


def fsb_batch_results(b, n_schools: int):
    xy = np.zeros((n_schools, 2), np.float64)
    sums = np.zeros((n_schools, 3), np.float64)
    mx = np.zeros(n_schools, np.float32)
    check(lib().fsb_batch_results(b, xy.ctypes.data_as(_lib._DP), sums.ctypes.data_as(_lib._DP),
                                  mx.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return xy, sums, mx


def fsb_batch_barycentre(b, n_schools: int) -> tuple[np.ndarray, np.ndarray]:
    """Per-school barycentres (n_schools, 2) and sums (n_schools, 3) of the
    last completed iteration."""
    xy = np.zeros((n_schools, 2), np.float64)
    sums = np.zeros((n_schools, 3), np.float64)
    check(lib().fsb_batch_barycentre(b, xy.ctypes.data_as(_lib._DP),
                                     sums.ctypes.data_as(_lib._DP)))
    return xy, sums


def fsb_batch_history(b, step: int, n_schools: int) -> np.ndarray:
    out = np.zeros(n_schools, RECORD)
    check(lib().fsb_batch_history(b, step, out.ctypes.data_as(ctypes.POINTER(_lib.fsb_record))))
    return out


def fsb_autotune(b, probe_steps: int) -> _lib.fsb_tuning:
    t = _lib.fsb_tuning()
    check(lib().fsb_autotune(b, probe_steps, ctypes.byref(t)))
    return t


def fsb_batch_get_tuning(b) -> _lib.fsb_tuning:
    t = _lib.fsb_tuning()
    check(lib().fsb_batch_get_tuning(b, ctypes.byref(t)))
    return t


def fsb_batch_step_index(b) -> int:
    t = ctypes.c_uint64()
    check(lib().fsb_batch_step_index(b, ctypes.byref(t)))
    return t.value


def fsb_batch_sync(b) -> None:
    check(lib().fsb_batch_sync(b))


def fsb_batch_destroy(b) -> None:
    check(lib().fsb_batch_destroy(b))


def fsb_barrier_probe(h, grid: int = 0, n_barriers: int = 1000) -> tuple[float, int]:
    """Microseconds per grid barrier of the persistent kind (grid 0 = the grid
    fsb_run(FSB_RUN_FUSED) uses for this school), and the max the last
    barrier published."""
    us = ctypes.c_double()
    mx = ctypes.c_uint32()
    check(lib().fsb_barrier_probe(h, grid, n_barriers, ctypes.byref(us), ctypes.byref(mx)))
    return us.value, mx.value


def fsb_eval_sqrt(inp, out, stream=None) -> None:
    """out = the kernels' binary32 square root of inp (device float32 tensors
    of equal length)."""
    import torch
    assert inp.dtype == torch.float32 and out.dtype == torch.float32
    assert inp.numel() == out.numel() and inp.is_contiguous() and out.is_contiguous()
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    check(lib().fsb_eval_sqrt(_ptr(inp), _ptr(out), inp.numel(), s))


def fsb_valu_probe(kind: int, blocks: int, iters: int, out, stream=None) -> tuple[float, int]:
    """(milliseconds, lane instructions) of one VALU ceiling probe launch;
    out: a device tensor of at least blocks x 256 4-byte words."""
    import torch
    assert out.is_contiguous() and out.element_size() * out.numel() >= blocks * 256 * 4
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    ms = ctypes.c_double()
    lanes = ctypes.c_uint64()
    check(lib().fsb_valu_probe(kind, blocks, iters, _ptr(out), out.element_size() * out.numel(),
                               s, ctypes.byref(ms), ctypes.byref(lanes)))
    return ms.value, lanes.value


def fsb_sweep_probe(cols, grid: int = 0, streamed: bool = False, stream=None) -> float:
    """Milliseconds of one streaming probe launch over four equal float32
    device tensors (read and written in place; each element gains 1)."""
    import torch
    assert len(cols) == 4 and all(c.dtype == torch.float32 and c.is_contiguous() for c in cols)
    n = cols[0].numel()
    assert all(c.numel() == n for c in cols)
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    arr = (ctypes.c_void_p * 4)(*[_ptr(c) for c in cols])
    ms = ctypes.c_double()
    check(lib().fsb_sweep_probe(arr, n, grid, int(streamed), s, ctypes.byref(ms)))
    return ms.value


def fsb_batch_profile_enable(b, every: int = 1) -> None:
    """Time every `every`-th launch (0 = off)."""
    check(lib().fsb_batch_profile_enable(b, int(every)))


def fsb_batch_kernel_times(b) -> tuple[int, float]:
    n = ctypes.c_uint64()
    ms = ctypes.c_double()
    check(lib().fsb_batch_kernel_times(b, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ---- convenience owners ---------------------------------------------------------

def alloc_columns(n: int, device="cuda", zero: bool = False):
    import torch
    make = torch.zeros if zero else torch.empty
    return {k: make(n, dtype=torch.float32, device=device) for k in COLUMNS}


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


class Batch:
    """Independent schools of the given sizes and seeds, packed back to back
    (each start rounded up to a multiple of 4 fish) in five columns
    allocated with PyTorch, plus the workspace."""

    def __init__(self, common: FsbConfig, sizes, seeds, starts=None, stream=None,
                 device="cuda"):
        import torch

        from .workloads import packed_starts
        self.sizes = _u64_array(sizes)
        self.seeds = _u64_array(seeds)
        self.starts = _u64_array(packed_starts(self.sizes) if starts is None else starts)
        self.n = int(self.sizes.size)
        self.common = common
        length = int(self.starts[-1] + self.sizes[-1])
        length = (length + 3) // 4 * 4
        self.cols = alloc_columns(length, device, zero=True)  # padding between schools is 0
        self.workspace = torch.empty(fsb_batch_workspace_bytes(common, self.starts, self.sizes),
                                     dtype=torch.uint8, device=device)
        self.h = fsb_batch_init(common, self.starts, self.sizes, self.seeds, self.cols,
                                self.workspace, stream)

    def run(self, n_steps: int, tune=None):
        fsb_batch_run(self.h, n_steps, tune)

    def results(self):
        return fsb_batch_results(self.h, self.n)

    def barycentre(self):
        return fsb_batch_barycentre(self.h, self.n)

    def history(self, step: int):
        return fsb_batch_history(self.h, step, self.n)

    def autotune(self, probe_steps: int):
        return fsb_autotune(self.h, probe_steps)

    @property
    def tuning(self):
        return fsb_batch_get_tuning(self.h)

    @property
    def t(self) -> int:
        return fsb_batch_step_index(self.h)

    def sync(self):
        fsb_batch_sync(self.h)

    def school_state(self, s: int) -> dict:
        """Columns of school s copied to host numpy arrays (synchronises)."""
        self.sync()
        a, n = int(self.starts[s]), int(self.sizes[s])
        return {k: v[a:a + n].cpu().numpy() for k, v in self.cols.items()}

    def close(self):
        if getattr(self, "h", None) is not None:
            fsb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
