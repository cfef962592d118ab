"""Deep persistent mode (FSB_RUN_FUSED_DEEP): several iterations per grid
barrier, their differences formed ahead of their maxima.  Columns, every
iteration's M and record must equal the oracle's (bit for bit; sums within
the 1e-6 gate), for iteration counts that fill the last superstep and for
counts that leave it short, and across launches interleaved with the other
modes."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default
from parity_util import assert_columns_equal, assert_sampled_fish, assert_sums_close, oracle_config

pytestmark = pytest.mark.gpu
DEEP = fsb.FSB_RUN_FUSED_DEEP


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[deep] {msg}", flush=True)


def history_sums(h):
    return np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)


def check_run(O, cfg, runs, what):
    steps = sum(k for k, _ in runs)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, steps)
    sch = fsb.School(cfg)
    for k, mode in runs:
        sch.run(k, mode)
    h = sch.history(0, steps)
    assert np.array_equal(h["step_lo"], np.arange(steps))
    assert np.array_equal(h["max_delta"].view(np.uint32), m.view(np.uint32)), (h["max_delta"], m)
    assert_sums_close(history_sums(h), s, a, what=what)
    assert sch.max_delta() == m[-1]
    assert_columns_equal(sch.state(), school, what)
    sch.close()


@pytest.mark.parametrize("n,steps", [(1, 5), (3, 3), (5, 9), (64, 4), (1001, 6), (4097, 8),
                                     (65539, 7), ((1 << 20) + 3, 5), ((1 << 22) + 1, 4),
                                     ((1 << 24) + 7, 3)])
def test_deep_matches_oracle(torch_cuda, O, n, steps):
    announce(f"n={n} steps={steps}")
    check_run(O, fsb.FsbConfig(n_fish=n, seed=606 + n, history_len=steps), [(steps, DEEP)],
              f"deep n={n}")


@pytest.mark.parametrize("steps", [1, 2, 3, 4, 5, 8, 9, 17])
def test_deep_every_superstep_length(torch_cuda, O, steps):
    """Full and short last supersteps, and a launch shorter than one."""
    announce(f"steps={steps}")
    check_run(O, fsb.FsbConfig(n_fish=20_011, seed=5, history_len=steps), [(steps, DEEP)],
              f"deep steps={steps}")


def test_deep_interleaved_with_every_mode(torch_cuda, O):
    """plain 2 + deep 5 + prev 2 + deep 1 + lean 3 + regs 2 + deep 6 == oracle 21."""
    announce("interleaved")
    cfg = fsb.FsbConfig(n_fish=300_007, seed=12, history_len=21)
    check_run(O, cfg, [(2, fsb.FSB_RUN_PLAIN), (5, DEEP), (2, fsb.FSB_RUN_FUSED_PREV), (1, DEEP),
                       (3, fsb.FSB_RUN_FUSED_LEAN), (2, fsb.FSB_RUN_FUSED_REGS), (6, DEEP)],
              "interleaved")


def test_deep_greedy_rule(torch_cuda, O):
    announce("greedy")
    cfg = fsb.FsbConfig(n_fish=(1 << 20) + 7, seed=13, swim_step=0.5,
                        swim_rule=fsb.FSB_SWIM_GREEDY, history_len=7)
    check_run(O, cfg, [(7, DEEP)], "deep greedy")


def test_deep_zero_swim(torch_cuda):
    announce("zero swim")
    sch = fsb.School(fsb.FsbConfig(n_fish=7777, seed=3, swim_step=0.0, history_len=6))
    before = sch.state()
    sch.run(6, DEEP)
    assert (sch.history(0, 6)["max_delta"] == 0).all()
    after = sch.state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    sch.close()


def test_deep_is_deterministic(torch_cuda):
    announce("determinism")
    cfg = fsb.FsbConfig(n_fish=(1 << 20) + 1, seed=9, history_len=9)
    runs = []
    for _ in range(2):
        sch = fsb.School(cfg)
        sch.run(9, DEEP)
        runs.append(sch.history(0, 9).tobytes())
        sch.close()
    assert runs[0] == runs[1]


def test_deep_cfg4_full_size_prefix(torch_cuda, O):
    """N = 2^26 (the persistent benchmark's school) through FSB_RUN_FUSED, 21
    iterations in one launch: five full supersteps of four and a short one,
    so the partials' ring (slot t mod 16) wraps."""
    n, steps = 1 << 26, 21
    announce(f"cfg4 N={n} prefix {steps}")
    check_run(O, fsb.FsbConfig(n_fish=n, seed=0, history_len=steps), [(steps, fsb.FSB_RUN_FUSED)],
              "deep cfg4 prefix")


@pytest.mark.parametrize("n,steps", [((1 << 23) + 5, 41), (10_007, 2000), ((1 << 21) + 1, 100)])
def test_deep_long_launch_ring_wraps(torch_cuda, O, n, steps):
    """One FSB_RUN_FUSED launch of many iterations, every record and the final
    columns against the oracle: above 5 x 2^20 fish four iterations per barrier
    in 768-thread blocks (41 iterations: the slot-t-mod-16 partials ring wraps
    twice), below eight per barrier (2000 iterations on 10^4 fish, as in the
    benchmark's launch length)."""
    announce(f"long launch n={n} steps={steps}")
    check_run(O, fsb.FsbConfig(n_fish=n, seed=2024 + steps, history_len=steps),
              [(steps, fsb.FSB_RUN_FUSED)], f"long launch n={n}")


def test_cfg4_full_length_sampled(torch_cuda, O):
    """The persistent benchmark run as it is timed: N = 2^26, 2000 iterations
    in one FSB_RUN_FUSED launch.  Sampled fish (the first and last groups and
    random ones) every field bit for bit against the oracle following each
    fish alone, fed with the run's recorded maxima; every maximum within the
    swim's reach, the last one the largest |prev - cur| of the final columns,
    and cur the distance of every final position."""
    import math
    n, steps = 1 << 26, 2000
    announce(f"cfg4 full length N={n} T={steps}")
    cfg = fsb.FsbConfig(n_fish=n, seed=0, history_len=steps)
    sch = fsb.School(cfg)
    start = {k: v.cpu().numpy() for k, v in sch.cols.items()}
    sch.run(steps, fsb.FSB_RUN_FUSED)
    got = sch.state()
    h = sch.history(0, steps)
    sch.close()
    assert np.array_equal(h["step_lo"], np.arange(steps))
    M = h["max_delta"]
    assert (M > 0).all() and (M <= cfg.swim_step * math.sqrt(2) + 1e-4).all()
    assert np.abs(got["prev"] - got["cur"]).max() == M[-1]
    assert np.array_equal(got["cur"], np.sqrt(got["x"] * got["x"] + got["y"] * got["y"]))
    assert (got["w"] >= cfg.w_min).all() and (got["w"] <= cfg.w_max).all()
    rng = np.random.default_rng(2026)
    sample = np.unique(np.concatenate([np.arange(8), n - 1 - np.arange(8), rng.integers(0, n, 112)]))
    assert_sampled_fish(O, oracle_config(cfg), start, got, M, sample, "cfg4 full length")


@pytest.mark.parametrize("n", [5 << 20, (5 << 20) + 3])
def test_deep_depth_boundary(torch_cuda, O, n):
    """The schools on either side of the depth boundary (eight iterations per
    barrier up to 5 x 2^20 fish, four above), over two supersteps and a
    ragged one, every record and the final columns against the oracle."""
    announce(f"depth boundary n={n}")
    check_run(O, fsb.FsbConfig(n_fish=n, seed=515, history_len=19), [(19, DEEP)],
              f"depth boundary n={n}")


def test_deep_wide_school_several_supersteps(torch_cuda, O):
    """Above 5 x 2^20 fish the library runs four iterations per barrier in
    768-thread blocks: supersteps of 4, 4 and 1, then interleaved with plain."""
    n = (1 << 23) + 5
    announce(f"wide n={n}")
    cfg = fsb.FsbConfig(n_fish=n, seed=77, history_len=13)
    check_run(O, cfg, [(9, DEEP), (1, fsb.FSB_RUN_PLAIN), (3, DEEP)], "deep wide")


CHILD_DEPTH = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import paper_2507_20173_amd as fsb
out = {}
for i, (n, steps, rule) in enumerate(CASES):
    s = fsb.School(fsb.FsbConfig(n_fish=n, seed=400 + i, swim_step=0.5 if rule else 0.1,
                                 swim_rule=rule, history_len=steps))
    s.run(steps, fsb.FSB_RUN_FUSED_DEEP)
    h = s.history(0, steps)
    out[f"max{i}"] = h["max_delta"]
    out[f"sums{i}"] = np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)
    st = s.state()
    for k in fsb.COLUMNS:
        out[f"{k}{i}"] = st[k]
    s.close()
np.savez(sys.argv[2], **out)
"""
DEPTH_CASES = [(1, 3, 0), (7, 5, 0), (4097, 9, 0), (65539, 6, 0), ((1 << 20) + 3, 11, 0),
               (300_007, 7, fsb.FSB_SWIM_GREEDY), (10_007, 2000, 0)]


@pytest.mark.parametrize("depth", ["2", "4"])
def test_forced_depth_in_a_child(torch_cuda, O, tmp_path, depth):
    """FSB_DEEP_DEPTH (read once per process) forces two or four iterations per
    barrier, the 768-thread instances, at sizes the library would run eight:
    every case still equals the oracle bit for bit.  The child launches the
    persistent kernels ordinarily (a cooperative launch from a second process
    while this one holds the GPU is refused with hipErrorIllegalState); the
    grid is the same co-resident one."""
    import os
    import subprocess
    import sys
    announce(f"FSB_DEEP_DEPTH={depth} in a child process")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = tmp_path / f"depth{depth}.npz"
    env = dict(os.environ, FSB_DEEP_DEPTH=depth, FSB_PERSISTENT_LAUNCH="regular")
    child = CHILD_DEPTH.replace("CASES", repr(DEPTH_CASES))
    subprocess.run([sys.executable, "-c", child, root, str(out)], env=env, check=True, timeout=240)
    got = np.load(out)
    for i, (n, steps, rule) in enumerate(DEPTH_CASES):
        cfg = fsb.FsbConfig(n_fish=n, seed=400 + i, swim_step=0.5 if rule else 0.1,
                            swim_rule=rule, history_len=steps)
        ocfg = oracle_config(cfg)
        school = O.init(ocfg)
        m, s, a = O.run(ocfg, school, 0, steps)
        what = f"depth {depth} n={n} steps={steps}"
        assert np.array_equal(got[f"max{i}"].view(np.uint32), m.view(np.uint32)), what
        assert_sums_close(got[f"sums{i}"], s, a, what=what)
        assert_columns_equal({k: got[f"{k}{i}"] for k in fsb.COLUMNS}, school, what)


@pytest.mark.parametrize("cfg", [dict(swim_rule=fsb.FSB_SWIM_WEIGHTED),
                                 dict(reduce_mode=fsb.FSB_REDUCE_NAIVE_F32),
                                 dict(reduce_mode=fsb.FSB_REDUCE_CRITICAL_F32)],
                         ids=["weighted", "naive", "critical"])
def test_deep_refuses_what_it_cannot_run(torch_cuda, cfg):
    sch = fsb.School(fsb.FsbConfig(n_fish=1000, seed=1, **cfg))
    with pytest.raises(fsb.FsbError) as e:
        sch.run(2, DEEP)
    assert e.value.code == fsb._lib.FSB_ERR_UNSUPPORTED
    sch.close()


CHILD_FILTER = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import paper_2507_20173_amd as fsb
out = {}
for i, (n, runs) in enumerate(CASES):
    total = sum(k for k, _ in runs)
    s = fsb.School(fsb.FsbConfig(n_fish=n, seed=900 + i, history_len=total))
    for k, mode in runs:
        s.run(k, mode)
    h = s.history(0, total)
    out[f"max{i}"] = h["max_delta"]
    out[f"sums{i}"] = np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)
    st = s.state()
    for k in fsb.COLUMNS:
        out[f"{k}{i}"] = st[k]
    s.close()
np.savez(sys.argv[2], **out)
"""
FILTER_CASES = [((1 << 20) + 3, [(13, fsb.FSB_RUN_FUSED)]),
                ((1 << 23) + 5, [(9, fsb.FSB_RUN_FUSED), (1, fsb.FSB_RUN_PLAIN),
                                 (6, fsb.FSB_RUN_FUSED)])]


@pytest.mark.parametrize("setting", ["redo", "off"])
def test_lookahead_skip_settings_in_a_child(torch_cuda, O, tmp_path, setting):
    """The deep kernel's look-ahead skips the objectives of fish whose move
    cannot reach a guess just below the current maxima, and recomputes the
    maxima exactly when a published one falls below the guess.  With
    FSB_LOOKAHEAD_FILTER=redo (read once per process) every guess is too high,
    so every superstep takes the recomputation; with "off" nothing is
    skipped.  Both equal the oracle bit for bit."""
    import os
    import subprocess
    import sys
    announce(f"FSB_LOOKAHEAD_FILTER={setting} in a child process")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = tmp_path / f"filter_{setting}.npz"
    env = dict(os.environ, FSB_LOOKAHEAD_FILTER=setting, FSB_PERSISTENT_LAUNCH="regular")
    child = CHILD_FILTER.replace("CASES", repr(FILTER_CASES))
    subprocess.run([sys.executable, "-c", child, root, str(out)], env=env, check=True, timeout=240)
    got = np.load(out)
    for i, (n, runs) in enumerate(FILTER_CASES):
        total = sum(k for k, _ in runs)
        cfg = fsb.FsbConfig(n_fish=n, seed=900 + i, history_len=total)
        ocfg = oracle_config(cfg)
        school = O.init(ocfg)
        m, s, a = O.run(ocfg, school, 0, total)
        what = f"filter {setting} n={n}"
        assert np.array_equal(got[f"max{i}"].view(np.uint32), m.view(np.uint32)), what
        assert_sums_close(got[f"sums{i}"], s, a, what=what)
        assert_columns_equal({k: got[f"{k}{i}"] for k in fsb.COLUMNS}, school, what)
