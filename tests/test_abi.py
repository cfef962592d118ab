"""The C ABI library loads on the CPU, exports every entry point the public
header declares, and rejects bad arguments on the host before any HIP call.
Every call here carries at least one invalid argument, so no kernel is ever
launched (these tests also run safely where a GPU is present)."""
import ctypes
import os
import re

import pytest

from paper_2507_20173_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsb.h")

DECL = re.compile(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fsb_\w+)\s*\(", re.M)


def declared():
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(DECL.findall(text)))


# The boundary's calls: one school (init, step, run, barycentre, max |diff|,
# sync, step index, resume, destroy, error text) and the batch (init, run,
# per-school barycentres, autotune, destroy).
BOUNDARY = ("fsb_workspace_bytes", "fsb_init", "fsb_step", "fsb_run", "fsb_barycentre",
            "fsb_max_delta", "fsb_sync", "fsb_step_index", "fsb_set_step_index", "fsb_destroy",
            "fsb_strerror", "fsb_batch_init", "fsb_batch_run", "fsb_batch_barycentre",
            "fsb_autotune", "fsb_batch_destroy")


def test_header_declares_entry_points():
    names = declared()
    missing = [n for n in BOUNDARY if n not in names]
    assert not missing, f"boundary calls not declared: {missing}"


def test_batch_barycentre_rejects_null_arguments():
    lib = _lib.lib()
    xy = (ctypes.c_double * 2)()
    assert lib.fsb_batch_barycentre(None, xy, None) == _lib.FSB_ERR_INVALID_ARG
    assert lib.fsb_batch_barycentre(ctypes.c_void_p(8), None, None) == _lib.FSB_ERR_INVALID_ARG


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_every_declared_symbol():
    assert set(declared()) <= set(_lib.PROTOTYPES)


def test_binding_constants_match_the_header():
    with open(HEADER) as fh:
        text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
    consts = {m.group(1): int(m.group(2).strip("()").rstrip("u"), 0)
              for m in re.finditer(r"^#define (FSB_\w+) (\(?-?\w+\)?)\s*$", text, re.M)
              if not m.group(1).endswith("_H")}
    assert "FSB_RUN_PLAIN_SPLIT" in consts and "FSB_KERNEL_FEED_SWIM" in consts
    for name, value in consts.items():
        if name == "FSB_ABI_VERSION":
            assert _lib.lib().fsb_abi_version() == value
        else:
            assert getattr(_lib, name) == value, name


def test_abi_version_and_strerror():
    lib = _lib.lib()
    assert lib.fsb_abi_version() == 2
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.fsb_strerror(code)
    assert lib.fsb_strerror(-99) == b"unknown error code"


def cfg(**kw):
    base = dict(n_fish=1000, seed=0, pond_half=100.0, swim_step=0.1, w_init_lo=1.0,
                w_init_hi=2.0, w_min=1.0, w_max=4.0, reduce_mode=0, history_len=1, swim_rule=0)
    base.update(kw)
    return _lib.fsb_config(*base.values())


def ws_bytes(c):
    out = ctypes.c_size_t()
    rc = _lib.lib().fsb_workspace_bytes(ctypes.byref(c), ctypes.byref(out))
    return rc, out.value


def test_workspace_bytes_pure_host():
    rc, b1 = ws_bytes(cfg(history_len=1))
    assert rc == 0 and b1 % 256 == 0 and b1 > 0
    rc, b2 = ws_bytes(cfg(history_len=1000))
    assert rc == 0 and b2 >= b1 + 999 * ctypes.sizeof(_lib.fsb_record) - 256


@pytest.mark.parametrize("bad", [
    dict(pond_half=0.0), dict(pond_half=float("nan")), dict(pond_half=-1.0),
    dict(swim_step=-0.1), dict(swim_step=float("inf")), dict(swim_step=1e-35),
    dict(w_init_lo=2.0, w_init_hi=1.0), dict(w_min=5.0, w_max=4.0),
    dict(w_max=float("nan")), dict(reduce_mode=3), dict(reduce_mode=7), dict(history_len=0),
    dict(swim_rule=4), dict(swim_rule=2, w_min=0.0), dict(swim_rule=3, w_init_lo=0.0, w_min=0.0),
    dict(swim_rule=2, w_init_lo=-1.0),
    dict(pond_half=2.0 ** 63 * (1 + 2.0 ** -23)), dict(pond_half=3e38),
    dict(w_max=2.0 ** 24 * (1 + 2.0 ** -23)), dict(w_min=-(2.0 ** 25)),
    dict(w_init_lo=-(2.0 ** 24) * 2, w_init_hi=1.0),
    dict(n_fish=(1 << 40) + 1)])
def test_bad_config_rejected(bad):
    rc, _ = ws_bytes(cfg(**bad))
    assert rc == _lib.FSB_ERR_INVALID_ARG


@pytest.mark.parametrize("edge", [
    dict(pond_half=2.0 ** 63), dict(pond_half=2.0 ** -126), dict(swim_step=2.0 ** -103),
    dict(w_min=-(2.0 ** 24), w_max=2.0 ** 24, w_init_lo=-(2.0 ** 24), w_init_hi=2.0 ** 24)])
def test_edge_configs_accepted(edge):
    # a failing call first: its message is the thread's last error, which a
    # later success leaves in place ("the last failing call")
    assert ws_bytes(cfg(history_len=0))[0] == _lib.FSB_ERR_INVALID_ARG
    before = _lib.lib().fsb_last_error()
    assert before
    rc, _ = ws_bytes(cfg(**edge))
    assert rc == 0
    assert _lib.lib().fsb_last_error() == before


FAKE = 1 << 40  # an aligned address that is never dereferenced


def cols(**over):
    base = dict(x=FAKE, y=FAKE + (1 << 20), w=FAKE + (2 << 20), prev=FAKE + (3 << 20),
                cur=FAKE + (4 << 20))
    base.update(over)
    return _lib.fsb_state(*base.values())


def init(c, st, ws, nbytes):
    h = ctypes.c_void_p()
    return _lib.lib().fsb_init(ctypes.byref(c), st, ws, nbytes, None, ctypes.byref(h))


@pytest.mark.parametrize("case", ["n0", "null_col", "misaligned_col", "overlap",
                                  "null_ws", "misaligned_ws", "small_ws"])
def test_init_rejects_before_any_hip_call(case):
    c = cfg()
    _, need = ws_bytes(c)
    st, ws, nbytes = cols(), FAKE + (8 << 20), need
    if case == "n0":
        c = cfg(n_fish=0)
    elif case == "null_col":
        st = cols(w=0)
    elif case == "misaligned_col":
        st = cols(prev=FAKE + (3 << 20) + 4)
    elif case == "overlap":
        st = cols(y=FAKE + 400)
    elif case == "null_ws":
        ws = 0
    elif case == "misaligned_ws":
        ws = FAKE + (8 << 20) + 64
    elif case == "small_ws":
        nbytes = need - 1
    assert init(c, st, ws, nbytes) == _lib.FSB_ERR_INVALID_ARG
    assert _lib.lib().fsb_last_error()


def test_null_handles_rejected():
    L = _lib.lib()
    assert L.fsb_step(None) == _lib.FSB_ERR_INVALID_ARG
    assert L.fsb_run(None, 1, 0) == _lib.FSB_ERR_INVALID_ARG
    assert L.fsb_sync(None) == _lib.FSB_ERR_INVALID_ARG
    assert L.fsb_destroy(None) == _lib.FSB_ERR_INVALID_ARG
    xy = (ctypes.c_double * 2)()
    assert L.fsb_barycentre(None, xy, None) == _lib.FSB_ERR_INVALID_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIBRARY", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError, match="no fallback"):
        _lib.lib()


def batch_ws(c, starts, sizes):
    import numpy as np
    st = np.asarray(starts, np.uint64)
    sz = np.asarray(sizes, np.uint64)
    out = ctypes.c_size_t()
    rc = _lib.lib().fsb_batch_workspace_bytes(ctypes.byref(c), len(sizes), st.ctypes.data,
                                              sz.ctypes.data, ctypes.byref(out))
    return rc, out.value


def test_batch_workspace_bytes_pure_host():
    rc, b = batch_ws(cfg(), [0, 1000, 3000], [1000, 2000, 5])
    assert rc == 0 and b % 256 == 0
    rc2, b2 = batch_ws(cfg(), [0, 1000, 3000, 4000], [1000, 2000, 5, 70000])
    assert rc2 == 0 and b2 > b


@pytest.mark.parametrize("starts,sizes", [
    ([0, 10], [8, 4]),          # start not a multiple of 4
    ([0, 4], [8, 4]),           # overlap
    ([8, 0], [4, 4]),           # decreasing
    ([0, 8], [4, 0]),           # empty school
    ([], []),                   # no schools
])
def test_batch_bad_schools_rejected(starts, sizes):
    rc, _ = batch_ws(cfg(), starts, sizes)
    assert rc == _lib.FSB_ERR_INVALID_ARG
    assert _lib.lib().fsb_last_error()


def test_batch_init_rejects_before_any_hip_call():
    import numpy as np
    c = cfg()
    st = np.asarray([0, 8], np.uint64)
    sz = np.asarray([8, 8], np.uint64)
    seeds = np.asarray([1, 2], np.uint64)
    h = ctypes.c_void_p()
    L = _lib.lib()
    # packed columns shorter than the last school
    rc = L.fsb_batch_init(ctypes.byref(c), 2, st.ctypes.data, sz.ctypes.data, seeds.ctypes.data,
                          cols(), 15, FAKE + (8 << 20), 1 << 30, None, ctypes.byref(h))
    assert rc == _lib.FSB_ERR_INVALID_ARG
    # NULL seeds
    rc = L.fsb_batch_init(ctypes.byref(c), 2, st.ctypes.data, sz.ctypes.data, None, cols(), 16,
                          FAKE + (8 << 20), 1 << 30, None, ctypes.byref(h))
    assert rc == _lib.FSB_ERR_INVALID_ARG
    # workspace too small
    rc = L.fsb_batch_init(ctypes.byref(c), 2, st.ctypes.data, sz.ctypes.data, seeds.ctypes.data,
                          cols(), 16, FAKE + (8 << 20), 64, None, ctypes.byref(h))
    assert rc == _lib.FSB_ERR_INVALID_ARG
    # the critical reduction is a plain-path ablation: batches refuse it
    crit = cfg(reduce_mode=_lib.FSB_REDUCE_CRITICAL_F32)
    rc = L.fsb_batch_init(ctypes.byref(crit), 2, st.ctypes.data, sz.ctypes.data,
                          seeds.ctypes.data, cols(), 16, FAKE + (8 << 20), 1 << 30, None,
                          ctypes.byref(h))
    assert rc == _lib.FSB_ERR_UNSUPPORTED
    assert L.fsb_batch_run(None, 1, None) == _lib.FSB_ERR_INVALID_ARG
    assert L.fsb_batch_destroy(None) == _lib.FSB_ERR_INVALID_ARG


def test_every_swim_rule_is_accepted():
    for rule in range(4):
        rc, b = ws_bytes(cfg(swim_rule=rule))
        assert rc == 0 and b > 0, rule


def test_every_reduce_mode_has_a_workspace():
    for mode in (_lib.FSB_REDUCE_COMPENSATED, _lib.FSB_REDUCE_NAIVE_F32,
                 _lib.FSB_REDUCE_CRITICAL_F32):
        rc, b = ws_bytes(cfg(reduce_mode=mode))
        assert rc == 0 and b > 0


def run_static(c, st, t=0, n=1, mode=0, records=FAKE + (16 << 20), status=0):
    return _lib.lib().fsb_run_static(ctypes.byref(c), st, t, n, mode, records, status, None)


@pytest.mark.parametrize("case", ["null_records", "misaligned_records", "misaligned_status",
                                  "bad_mode", "t_limit", "steps_limit", "bad_config",
                                  "null_col"])
def test_run_static_rejects_before_any_hip_call(case):
    c, st, kw = cfg(), cols(), {}
    if case == "null_records":
        kw["records"] = 0
    elif case == "misaligned_records":
        kw["records"] = FAKE + (16 << 20) + 4
    elif case == "misaligned_status":
        kw["status"] = FAKE + (17 << 20) + 2
    elif case == "bad_mode":
        kw["mode"] = _lib.FSB_RUN_PLAIN_SPLIT + 1
    elif case == "t_limit":
        kw["t"] = 1 << 32
    elif case == "steps_limit":
        kw.update(t=(1 << 32) - 5, n=6)
    elif case == "bad_config":
        c = cfg(history_len=0)
    elif case == "null_col":
        st = cols(cur=0)
    assert run_static(c, st, **kw) == _lib.FSB_ERR_INVALID_ARG
    assert _lib.lib().fsb_last_error()


@pytest.mark.parametrize("case", ["kind", "blocks", "iters", "null_out", "small_out",
                                  "misaligned_out", "null_results"])
def test_valu_probe_rejects_before_any_hip_call(case):
    """Every argument check of fsb_valu_probe runs on the host first."""
    lib = _lib.lib()
    ms, lanes = ctypes.c_double(), ctypes.c_uint64()
    args = dict(kind=0, blocks=2, iters=1, out=FAKE, out_bytes=2 * 256 * 4,
                ms=ctypes.byref(ms), lanes=ctypes.byref(lanes))
    if case == "kind":
        args["kind"] = _lib.FSB_PROBE_KINDS
    elif case == "blocks":
        args["blocks"] = 0
    elif case == "iters":
        args["iters"] = 0
    elif case == "null_out":
        args["out"] = None
    elif case == "small_out":
        args["out_bytes"] = 2 * 256 * 4 - 1
    elif case == "misaligned_out":
        args["out"] = FAKE + 2
    elif case == "null_results":
        args["ms"] = None
    rc = lib.fsb_valu_probe(args["kind"], args["blocks"], args["iters"], args["out"],
                            args["out_bytes"], None, args["ms"], args["lanes"])
    assert rc == _lib.FSB_ERR_INVALID_ARG


@pytest.mark.parametrize("case", ["null_cols", "null_col", "misaligned", "n_zero", "n_ragged",
                                  "null_ms"])
def test_sweep_probe_rejects_before_any_hip_call(case):
    lib = _lib.lib()
    ms = ctypes.c_double()
    ptrs = [FAKE + k * (1 << 20) for k in range(4)]
    n, out = 1024, ctypes.byref(ms)
    if case == "null_col":
        ptrs[2] = 0
    elif case == "misaligned":
        ptrs[1] += 4
    elif case == "n_zero":
        n = 0
    elif case == "n_ragged":
        n = 1026
    elif case == "null_ms":
        out = None
    cols = None if case == "null_cols" else (ctypes.c_void_p * 4)(*ptrs)
    assert lib.fsb_sweep_probe(cols, n, 0, 0, None, out) == _lib.FSB_ERR_INVALID_ARG
