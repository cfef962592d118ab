"""Persistent (fused) mode: one cooperative launch per fsb_run, a grid
barrier per iteration.  Columns and maxima must equal the oracle's (and the
plain path's) bit for bit; sums within the 1e-6 gate."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default
from parity_util import assert_columns_equal, assert_sums_close, oracle_config

pytestmark = pytest.mark.gpu
FUSED, PLAIN = fsb.FSB_RUN_FUSED, fsb.FSB_RUN_PLAIN


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[fused] {msg}", flush=True)


def history_sums(h):
    return np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)


VARIANTS = [fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN]


@pytest.mark.parametrize("variant", VARIANTS, ids=["prev", "lean"])
@pytest.mark.parametrize("n,steps", [(1, 5), (2, 3), (3, 1), (5, 7), (64, 4), (1001, 6),
                                     (4097, 5), (65539, 4), ((1 << 20) + 3, 3),
                                     ((1 << 23) + 6, 2), ((1 << 24) + 7, 2)])
def test_fused_matches_oracle(torch_cuda, O, n, steps, variant):
    announce(f"n={n} steps={steps} variant={variant}")
    cfg = fsb.FsbConfig(n_fish=n, seed=4242 + n, history_len=steps)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, steps)
    sch = fsb.School(cfg)
    sch.run(steps, variant)
    h = sch.history(0, steps)
    assert np.array_equal(h["step_lo"], np.arange(steps))
    assert np.array_equal(h["max_delta"], m), f"maxima {h['max_delta']} vs {m}"
    assert_sums_close(history_sums(h), s, a, what=f"fused n={n}")
    assert_columns_equal(sch.state(), school, f"fused n={n}")
    sch.close()


def test_fused_plain_interleaved(torch_cuda, O):
    """plain 2 + prev 3 + plain 1 + lean 1 + lean 2 + prev 2 == oracle 11."""
    announce("interleaved")
    n = 30_011
    cfg = fsb.FsbConfig(n_fish=n, seed=5, history_len=11)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, 11)
    sch = fsb.School(cfg)
    for k, mode in ((2, PLAIN), (3, VARIANTS[0]), (1, PLAIN), (1, VARIANTS[1]), (2, VARIANTS[1]),
                    (2, VARIANTS[0])):
        sch.run(k, mode)
    h = sch.history(0, 11)
    assert np.array_equal(h["max_delta"], m)
    assert_sums_close(history_sums(h), s, a, what="interleaved")
    assert_columns_equal(sch.state(), school, "interleaved")


@pytest.mark.parametrize("variant", VARIANTS, ids=["prev", "lean"])
def test_fused_naive_reduction(torch_cuda, O, variant):
    announce(f"naive variant={variant}")
    n = 100_003
    cfg = fsb.FsbConfig(n_fish=n, seed=6, reduce_mode=fsb.FSB_REDUCE_NAIVE_F32, history_len=4)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, 4)
    sch = fsb.School(cfg)
    sch.run(4, variant)
    h = sch.history(0, 4)
    assert np.array_equal(h["max_delta"], m)
    assert_sums_close(history_sums(h), s, a, tol=1e-3, what="fused naive")
    assert_columns_equal(sch.state(), school, "fused naive")


@pytest.mark.parametrize("variant", VARIANTS, ids=["prev", "lean"])
def test_fused_zero_swim(torch_cuda, variant):
    announce("zero swim")
    cfg = fsb.FsbConfig(n_fish=7777, seed=3, swim_step=0.0, history_len=5)
    sch = fsb.School(cfg)
    before = sch.state()
    sch.run(5, variant)
    assert (sch.history(0, 5)["max_delta"] == 0).all()
    after = sch.state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k


def test_fused_is_deterministic(torch_cuda):
    """Same launch shape, same sums to the last bit."""
    announce("determinism")
    cfg = fsb.FsbConfig(n_fish=(1 << 20) + 1, seed=9, history_len=6)
    runs = []
    for _ in range(2):
        sch = fsb.School(cfg)
        sch.run(6, FUSED)
        runs.append(sch.history(0, 6).tobytes())
        sch.close()
    assert runs[0] == runs[1]


@pytest.mark.parametrize("variant", [fsb.FSB_RUN_FUSED] + VARIANTS, ids=["auto", "prev", "lean"])
def test_cfg4_full_size_prefix(torch_cuda, O, variant):
    """N = 2^26 (the persistent-form workload) for the first iterations,
    every fish bit-exact."""
    n, steps = 1 << 26, 2
    announce(f"cfg4 N={n} prefix {steps} variant={variant}")
    cfg = fsb.FsbConfig(n_fish=n, seed=0, history_len=steps)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, steps)
    sch = fsb.School(cfg)
    sch.run(steps, variant)
    h = sch.history(0, steps)
    assert np.array_equal(h["max_delta"], m)
    assert_sums_close(history_sums(h), s, a, what="cfg4 prefix")
    assert_columns_equal(sch.state(), school, "cfg4 prefix")
    sch.close()


CHILD = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
import paper_2507_20173_amd as fsb
s = fsb.School(fsb.FsbConfig(n_fish=50_003, seed=31, history_len=4))
s.run(4, fsb.FSB_RUN_FUSED)
st = s.state()
b = fsb.Batch(fsb.FsbConfig(n_fish=0), [5, 1000, 4099], [1, 2, 3])
b.run(3)
bs = [b.school_state(i) for i in range(3)]
np.savez(sys.argv[2], *[st[k] for k in fsb.COLUMNS], *[x[k] for x in bs for k in fsb.COLUMNS])
"""


def test_regular_launch_matches_cooperative(torch_cuda, tmp_path):
    """FSB_PERSISTENT_LAUNCH=regular (for tools that cannot follow cooperative
    launches) runs the same kernels with an ordinary launch: identical bits."""
    import os
    import subprocess
    import sys
    announce("regular launch in a child process")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = tmp_path / "regular.npz"
    env = dict(os.environ, FSB_PERSISTENT_LAUNCH="regular")
    subprocess.run([sys.executable, "-c", CHILD, root, str(out)], env=env, check=True,
                   timeout=240)
    got = np.load(out)
    s = fsb.School(fsb.FsbConfig(n_fish=50_003, seed=31, history_len=4))
    s.run(4, FUSED)
    st = s.state()
    b = fsb.Batch(fsb.FsbConfig(n_fish=0), [5, 1000, 4099], [1, 2, 3])
    b.run(3)
    want = [st[k] for k in fsb.COLUMNS] + [b.school_state(i)[k] for i in range(3)
                                           for k in fsb.COLUMNS]
    for i, w in enumerate(want):
        assert np.array_equal(got[f"arr_{i}"].view(np.uint32), w.view(np.uint32)), i


CHILD_TIMEOUT = r"""
import sys
sys.path.insert(0, sys.argv[1])
import paper_2507_20173_amd as fsb
out = []
for mode in (fsb.FSB_RUN_FUSED_REGS, fsb.FSB_RUN_FUSED_LEAN, fsb.FSB_RUN_FUSED_DEEP):
    s = fsb.School(fsb.FsbConfig(n_fish=1 << 20, seed=1))
    s.run(20, mode)
    try:
        s.sync()
        out.append("fused ok")
    except fsb.FsbError as e:
        out.append(f"fused {e.code} {e}")
    s.close()
for tune in (fsb.tuning(1024, 8, 20), fsb.tuning(256, 8, 20, variant=fsb.FSB_RUN_FUSED_DEEP)):
    b = fsb.Batch(fsb.FsbConfig(n_fish=0), [1000] * 64, list(range(64)))
    b.run(20, tune)
    try:
        b.sync()
        out.append("batch ok")
    except fsb.FsbError as e:
        out.append(f"batch {e.code} {e}")
    b.close()
print("|".join(out), flush=True)
"""


def test_barrier_timeout_is_reported(torch_cuda):
    """The persistent kernels' bounded barrier wait, forced to give up from
    the host (FSB_BARRIER_SPIN_LIMIT=1 in a child process): every block
    leaves its kernel normally and the host reports FSB_ERR_DEVICE naming the
    time-out, for one school and for a batch.  The child launches the
    persistent kernels ordinarily (a cooperative launch from a second process
    while this one holds the GPU was refused with hipErrorIllegalState); the
    time-out path is the same either way."""
    import os
    import subprocess
    import sys
    announce("forced barrier time-out in a child process")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, FSB_BARRIER_SPIN_LIMIT="1", FSB_PERSISTENT_LAUNCH="regular")
    r = subprocess.run([sys.executable, "-c", CHILD_TIMEOUT, root], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    parts = r.stdout.strip().splitlines()[-1].split("|")
    code = str(fsb._lib.FSB_ERR_DEVICE)
    assert len(parts) == 5  # register-resident, lean, deep; batches lean and deep
    for p in parts[:3]:
        assert p.startswith(f"fused {code}") and "timed out" in p, p
    for p in parts[3:]:
        assert p.startswith(f"batch {code}") and "timed out" in p, p


@pytest.mark.parametrize("grid", [1, 2, 16, 17, 100, 0])
def test_barrier_probe(torch_cuda, O, grid):
    """The barrier-only probe: each barrier publishes max(block + k) over the
    grid, so the last of n carries (grid - 1) + (n - 1); the school is left
    untouched (its next iterations still match the oracle)."""
    n, k = (1 << 20) + 3, 200
    announce(f"barrier probe grid={grid}")
    cfg = fsb.FsbConfig(n_fish=n, seed=13, history_len=3)
    sch = fsb.School(cfg)
    sch.run(1, FUSED)
    us, mx = fsb.fsb_barrier_probe(sch.h, grid, k)
    g = grid or 256
    assert mx == (g - 1) + (k - 1), (mx, g)
    assert 0.0 < us < 1000.0
    sch.run(2, FUSED)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, 3)
    h = sch.history(0, 3)
    assert np.array_equal(h["max_delta"], m)
    assert_columns_equal(sch.state(), school, "after probe")
    with pytest.raises(fsb.FsbError) as e:
        fsb.fsb_barrier_probe(sch.h, 1 << 20, 10)
    assert e.value.code == fsb._lib.FSB_ERR_INVALID_ARG
    sch.close()
