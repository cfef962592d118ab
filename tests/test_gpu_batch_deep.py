"""Deep batched kernel (fsb_tuning.variant = FSB_RUN_FUSED_DEEP): eight
iterations of every school per grid barrier.  Every school must equal the
oracle run of that school alone, bit for bit (columns, every iteration's M;
sums within the 1e-6 gate), for iteration counts that fill the last
superstep and counts that leave it short, across graph-replayed launches of
any length, under every tile schedule, and interleaved with the other
variants."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default
from paper_2507_20173_amd.workloads import log_uniform_school_sizes, packed_starts, school_seeds
from parity_util import assert_columns_equal, assert_sampled_fish, assert_sums_close, oracle_config

pytestmark = pytest.mark.gpu
DEEP = fsb.FSB_RUN_FUSED_DEEP
SIZES = [1, 2, 3, 5, 7, 64, 65, 255, 256, 257, 1000, 4099, 16385, 65537]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[batch deep] {msg}", flush=True)


def check_against_oracle(O, b, steps, common, schools=None, what=""):
    _, sums, mx = b.results()
    for i in (range(b.n) if schools is None else schools):
        cfg = fsb.FsbConfig(n_fish=int(b.sizes[i]), seed=int(b.seeds[i]),
                            pond_half=common.pond_half, swim_step=common.swim_step,
                            w_min=common.w_min, w_max=common.w_max, swim_rule=common.swim_rule)
        ocfg = oracle_config(cfg)
        school = O.init(ocfg)
        m, s, a = O.run(ocfg, school, 0, steps)
        assert mx[i].view(np.uint32) == m[-1].view(np.uint32), f"{what} school {i}"
        assert_sums_close(sums[i], s[-1], a[-1], what=f"{what} school {i}")
        assert_columns_equal(b.school_state(i), school, f"{what} school {i}")
        for step in range(max(0, steps - common.history_len), steps):
            h = b.history(step)
            assert h["step_lo"][i] == step
            assert h["max_delta"][i].view(np.uint32) == m[step].view(np.uint32), (what, i, step)


@pytest.mark.parametrize("fpl", [4, 8, 16])
@pytest.mark.parametrize("steps,per_launch", [(8, 8), (11, 11), (11, 3), (17, 8), (5, 100)])
def test_deep_batch_matches_oracle(torch_cuda, O, fpl, steps, per_launch):
    announce(f"fpl={fpl} steps={steps} per launch={per_launch}")
    common = fsb.FsbConfig(n_fish=0, history_len=steps)
    seeds = [31 * i + 7 for i in range(len(SIZES))]
    b = fsb.Batch(common, SIZES, seeds, starts=packed_starts(SIZES, 4))
    b.run(steps, fsb.tuning(256, fpl, per_launch, variant=DEEP))
    check_against_oracle(O, b, steps, common, what=f"deep fpl={fpl}")
    b.close()


SCHEDULES = [(fsb.FSB_SCHED_STATIC, 0), (fsb.FSB_SCHED_STATIC, 3), (fsb.FSB_SCHED_DYNAMIC, 1),
             (fsb.FSB_SCHED_DYNAMIC, 16), (fsb.FSB_SCHED_GUIDED, 4)]


@pytest.mark.parametrize("sched,chunk", SCHEDULES, ids=[f"s{s}c{c}" for s, c in SCHEDULES])
def test_deep_schedules_identical_to_lean(torch_cuda, sched, chunk):
    """Columns and maxima equal the lean variant's bit for bit; the sums are
    bit-identical across schedules of the deep variant (tile partials folded
    in tile order)."""
    announce(f"schedule {sched} chunk {chunk}")
    common = fsb.FsbConfig(n_fish=0, history_len=10)
    seeds = list(range(len(SIZES)))
    ref = fsb.Batch(common, SIZES, seeds)
    ref.run(10, fsb.tuning(1024, 8, 10, variant=fsb.FSB_RUN_FUSED_LEAN))
    ref_state = [ref.school_state(i) for i in range(ref.n)]
    _, _, ref_max = ref.results()
    ref.close()
    base = fsb.Batch(common, SIZES, seeds)
    base.run(10, fsb.tuning(256, 8, 10, variant=DEEP))
    _, base_sums, _ = base.results()
    base.close()
    b = fsb.Batch(common, SIZES, seeds)
    b.run(10, fsb.tuning(256, 8, 4, variant=DEEP, schedule=sched, chunk_tiles=chunk))
    _, sums, mx = b.results()
    assert np.array_equal(mx, ref_max)
    assert np.array_equal(sums.view(np.uint64), base_sums.view(np.uint64))
    for i in range(b.n):
        got = b.school_state(i)
        for k in got:
            assert np.array_equal(got[k].view(np.uint32), ref_state[i][k].view(np.uint32)), (i, k)
    b.close()


def test_deep_batch_interleaved_with_other_variants(torch_cuda, O):
    announce("interleaved")
    common = fsb.FsbConfig(n_fish=0, history_len=19)
    sizes = [3, 1000, 4099, 65537]
    seeds = [11, 12, 13, 14]
    b = fsb.Batch(common, sizes, seeds)
    b.run(3, fsb.tuning(1024, 8, 3, variant=fsb.FSB_RUN_FUSED_LEAN))
    b.run(9, fsb.tuning(256, 16, 9, variant=DEEP))
    b.run(2, fsb.tuning(256, 4, 2, variant=fsb.FSB_RUN_FUSED_PREV))
    b.run(5, fsb.tuning(256, 8, 2, variant=DEEP))
    check_against_oracle(O, b, 19, common, what="interleaved")
    b.close()


def test_deep_batch_greedy_rule(torch_cuda, O):
    announce("greedy")
    common = fsb.FsbConfig(n_fish=0, swim_step=0.5, swim_rule=fsb.FSB_SWIM_GREEDY, history_len=9)
    sizes = [5, 257, 4099, 16385]
    b = fsb.Batch(common, sizes, [1, 2, 3, 4])
    b.run(9, fsb.tuning(256, 8, 9, variant=DEEP))
    check_against_oracle(O, b, 9, common, what="greedy")
    b.close()


def test_deep_batch_gaps_untouched(torch_cuda):
    announce("gaps")
    sizes = [5, 9, 1, 130]
    starts = [0, 16, 40, 48]
    b = fsb.Batch(fsb.FsbConfig(n_fish=0), sizes, [1, 2, 3, 4], starts=starts)
    b.sync()
    mask = np.ones(b.cols["x"].numel(), bool)
    for a, n in zip(starts, sizes):
        mask[a:a + n] = False
    for v in b.cols.values():
        v[torch_cuda.from_numpy(mask).to(v.device)] = 12345.0
    b.run(10, fsb.tuning(256, 4, 10, variant=DEEP))
    b.sync()
    for k, v in b.cols.items():
        assert (v.cpu().numpy()[mask] == 12345.0).all(), k
    b.close()


def test_deep_cfg5_full_shape(torch_cuda, O):
    """The 4096-school shape for 11 iterations (a full and a short superstep):
    the smallest schools and two mid-sized ones against the oracle."""
    sizes = log_uniform_school_sizes(4096)
    seeds = school_seeds(4096)
    steps = 11
    announce(f"cfg5 deep {int(sizes.sum())} fish, {steps} iterations")
    common = fsb.FsbConfig(n_fish=0, history_len=steps)
    b = fsb.Batch(common, sizes, seeds)
    b.run(steps, fsb.tuning(256, 8, steps, variant=DEEP, schedule=fsb.FSB_SCHED_DYNAMIC,
                            chunk_tiles=16))
    _, sums, mx = b.results()
    assert (mx > 0).all() and (mx <= 0.1 * np.sqrt(2) + 1e-4).all()
    order = np.argsort(sizes)
    check_against_oracle(O, b, steps, common,
                         schools=list(order[:4]) + list(order[2048:2050]) + [order[-1]],
                         what="cfg5 deep")
    b.close()


def test_deep_cfg5_full_length_sampled(torch_cuda, O):
    """The batched benchmark run as it is timed: the 4096-school shape
    (6.07e8 fish), 500 iterations in one graph launch at the tuning the
    autotuner picks for it.  Every school's every maximum within the swim's
    reach; in the largest, the median and the smallest schools, sampled fish
    every field bit for bit against the oracle following each fish alone,
    fed with that school's recorded maxima."""
    import math
    sizes = log_uniform_school_sizes(4096)
    seeds = school_seeds(4096)
    steps = 500
    announce(f"cfg5 full length: {int(sizes.sum())} fish, {steps} iterations, one launch")
    common = fsb.FsbConfig(n_fish=0, history_len=steps)
    b = fsb.Batch(common, sizes, seeds)
    order = np.argsort(sizes)
    chosen = [int(order[-1]), int(order[-2]), int(order[2048]), int(order[0])]
    start = {s: b.school_state(s) for s in chosen}
    b.run(steps, fsb.tuning(256, 16, 1000, variant=DEEP, schedule=fsb.FSB_SCHED_DYNAMIC,
                            chunk_tiles=4))
    hist = [b.history(t) for t in range(steps)]
    M = np.stack([h["max_delta"] for h in hist])  # [steps, schools]
    assert (M > 0).all() and (M <= 0.1 * math.sqrt(2) + 1e-4).all()
    assert all(np.array_equal(h["step_lo"], np.full(b.n, t)) for t, h in enumerate(hist))
    rng = np.random.default_rng(5)
    for s in chosen:
        n = int(sizes[s])
        got = b.school_state(s)
        cfg = fsb.FsbConfig(n_fish=n, seed=int(seeds[s]))
        sample = np.unique(np.concatenate([np.arange(min(n, 5)), n - 1 - np.arange(min(n, 5)),
                                           rng.integers(0, n, 40)]))
        assert_sampled_fish(O, oracle_config(cfg), start[s], got, M[:, s], sample,
                            f"cfg5 full length school {s} ({n} fish)")
    b.close()


def test_deep_batch_long_run_rings_wrap(torch_cuda, O):
    """The batched form as the benchmark runs it (the tuning the autotuner
    picks for the 4096-school batch: 256 threads, 16 fish per lane, dynamic
    chunks of 4 tiles, launches of up to 1000 iterations), for 500 iterations
    in one graph launch on 64 schools, one of them 10^6 fish: the per-school
    max ring (slot t mod 24) and the tile-partial ring (slot t mod 16) wrap
    many times.  Every school's every record and final columns against the
    oracle's run of that school alone."""
    steps = 500
    sizes = np.concatenate([[1_000_000], log_uniform_school_sizes(63, lo=1_000, hi=10_000,
                                                                  meta_seed=5)]).astype(np.uint64)
    seeds = school_seeds(64, base=9000)
    announce(f"long run: 64 schools, {int(sizes.sum())} fish, {steps} iterations, one launch")
    common = fsb.FsbConfig(n_fish=0, history_len=steps)
    b = fsb.Batch(common, sizes, seeds)
    b.run(steps, fsb.tuning(256, 16, 1000, variant=DEEP, schedule=fsb.FSB_SCHED_DYNAMIC,
                            chunk_tiles=4))
    hist = [b.history(t) for t in range(steps)]
    for i in range(b.n):
        cfg = fsb.FsbConfig(n_fish=int(sizes[i]), seed=int(seeds[i]))
        ocfg = oracle_config(cfg)
        school = O.init(ocfg)
        m, s, a = O.run(ocfg, school, 0, steps)
        rec = np.array([h[i] for h in hist])
        what = f"long run school {i} ({int(sizes[i])} fish)"
        assert np.array_equal(rec["step_lo"], np.arange(steps)), what
        assert np.array_equal(rec["max_delta"].view(np.uint32), m.view(np.uint32)), what
        assert_sums_close(np.stack([rec["sum_w"], rec["sum_wx"], rec["sum_wy"]], 1), s, a,
                          what=what)
        assert_columns_equal(b.school_state(i), school, what)
    b.close()


def test_deep_batch_refusals(torch_cuda):
    b = fsb.Batch(fsb.FsbConfig(n_fish=0), [10, 20], [1, 2])
    with pytest.raises(fsb.FsbError) as e:
        b.run(2, fsb.tuning(1024, 8, 2, variant=DEEP))
    assert e.value.code == fsb._lib.FSB_ERR_INVALID_ARG
    b.run(2, fsb.tuning(256, 8, 2, variant=DEEP))  # the handle still works
    b.close()
    for cfg in (dict(reduce_mode=fsb.FSB_REDUCE_NAIVE_F32), dict(swim_rule=fsb.FSB_SWIM_WEIGHTED)):
        b = fsb.Batch(fsb.FsbConfig(n_fish=0, **cfg), [10, 20], [1, 2])
        with pytest.raises(fsb.FsbError) as e:
            b.run(2, fsb.tuning(256, 8, 2, variant=DEEP))
        assert e.value.code == fsb._lib.FSB_ERR_UNSUPPORTED
        b.run(2, fsb.tuning(256, 8, 2))  # the library's choice still runs
        b.close()


CHILD_FILTER = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import paper_2507_20173_amd as fsb
sizes, seeds, steps = SIZES_SEEDS_STEPS
b = fsb.Batch(fsb.FsbConfig(n_fish=0, history_len=steps), sizes, seeds)
b.run(steps, fsb.tuning(256, 16, 1000, variant=fsb.FSB_RUN_FUSED_DEEP,
                        schedule=fsb.FSB_SCHED_DYNAMIC, chunk_tiles=4))
out = {}
for t in range(steps):
    h = b.history(t)
    out[f"max{t}"] = h["max_delta"]
    out[f"sums{t}"] = np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)
for i in range(b.n):
    st = b.school_state(i)
    for k in fsb.COLUMNS:
        out[f"{k}{i}"] = st[k]
b.close()
np.savez(sys.argv[2], **out)
"""


@pytest.mark.parametrize("setting", ["redo", "off"])
def test_deep_batch_lookahead_skip_settings_in_a_child(torch_cuda, O, tmp_path, setting):
    """Schools of 2^16 fish or more skip look-ahead objectives that cannot
    reach a guess just below their current maxima; a school whose next maxima
    fall below the guess is swept once more with an exact look-ahead.  With
    FSB_LOOKAHEAD_FILTER=redo (read once per process) every guess fails, so
    every superstep takes that extra sweep for every large school; with
    "off" nothing is skipped.  Both equal the oracle, school by school."""
    import os
    import subprocess
    import sys
    sizes = [70_001, 200_003, 1_000, 5, 131_072]
    seeds = [41, 42, 43, 44, 45]
    steps = 19
    announce(f"FSB_LOOKAHEAD_FILTER={setting} batch in a child process")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = tmp_path / f"batch_filter_{setting}.npz"
    env = dict(os.environ, FSB_LOOKAHEAD_FILTER=setting, FSB_PERSISTENT_LAUNCH="regular")
    child = CHILD_FILTER.replace("SIZES_SEEDS_STEPS", repr((sizes, seeds, steps)))
    subprocess.run([sys.executable, "-c", child, root, str(out)], env=env, check=True, timeout=240)
    got = np.load(out)
    for i, (n, seed) in enumerate(zip(sizes, seeds)):
        ocfg = oracle_config(fsb.FsbConfig(n_fish=n, seed=seed))
        school = O.init(ocfg)
        m, s, a = O.run(ocfg, school, 0, steps)
        what = f"batch filter {setting} school {i} ({n} fish)"
        gm = np.array([got[f"max{t}"][i] for t in range(steps)], np.float32)
        assert np.array_equal(gm.view(np.uint32), m.view(np.uint32)), what
        gs = np.array([got[f"sums{t}"][i] for t in range(steps)])
        assert_sums_close(gs, s, a, what=what)
        assert_columns_equal({k: got[f"{k}{i}"] for k in fsb.COLUMNS}, school, what)
