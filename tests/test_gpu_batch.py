"""Batched schools: one persistent launch (replayed from a HIP graph) advances
many independent schools.  Every school must equal, bit for bit, the oracle
run of that school alone (its own size and seed), whatever the launch shape."""
import os

import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default
from paper_2507_20173_amd.workloads import log_uniform_school_sizes, packed_starts, school_seeds
from parity_util import assert_columns_equal, assert_sums_close, oracle_config

pytestmark = pytest.mark.gpu

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
    print(f"[batch] {msg}", flush=True)


def oracle_school(O, size, seed, steps, common=None):
    cfg = common or fsb.FsbConfig(n_fish=size)
    ocfg = oracle_config(fsb.FsbConfig(n_fish=size, seed=int(seed), pond_half=cfg.pond_half,
                                       swim_step=cfg.swim_step, w_init_lo=cfg.w_init_lo,
                                       w_init_hi=cfg.w_init_hi, w_min=cfg.w_min,
                                       w_max=cfg.w_max, swim_rule=cfg.swim_rule))
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, steps)
    return school, m, s, a


def check_batch_against_oracle(O, b, steps, schools=None, what=""):
    xy, sums, mx = b.results()
    for i in (range(b.n) if schools is None else schools):
        school, m, s, a = oracle_school(O, int(b.sizes[i]), b.seeds[i], steps, b.common)
        assert mx[i] == m[-1], f"{what} school {i}: M {mx[i]} != {m[-1]}"
        assert_sums_close(sums[i], s[-1], a[-1], what=f"{what} school {i}")
        assert_columns_equal(b.school_state(i), school, f"{what} school {i}")


@pytest.mark.parametrize("variant", [fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN],
                         ids=["prev", "lean"])
@pytest.mark.parametrize("align", [4, 64])
def test_batch_matches_oracle_per_school(torch_cuda, O, align, variant):
    announce(f"{len(SIZES)} schools, 6 iterations, starts aligned to {align} fish, "
             f"variant {variant}")
    common = fsb.FsbConfig(n_fish=0, history_len=6)
    seeds = [17 * i + 3 for i in range(len(SIZES))]
    b = fsb.Batch(common, SIZES, seeds, starts=packed_starts(SIZES, align))
    b.run(6, fsb.tuning(variant=variant))
    check_batch_against_oracle(O, b, 6, what="default tuning")
    for step in range(6):
        h = b.history(step)
        assert (h["step_lo"] == step).all()
    b.close()


@pytest.mark.parametrize("variant", [fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN],
                         ids=["prev", "lean"])
@pytest.mark.parametrize("block", [256, 1024])
@pytest.mark.parametrize("fpl", [4, 8, 16])
def test_every_launch_shape_gives_identical_state(torch_cuda, block, fpl, variant):
    announce(f"shape block={block} fish_per_thread={fpl} variant={variant}")
    common = fsb.FsbConfig(n_fish=0)
    seeds = list(range(len(SIZES)))
    ref = fsb.Batch(common, SIZES, seeds)
    ref.run(5, fsb.tuning(1024, 8, 5))
    ref_state = [ref.school_state(i) for i in range(ref.n)]
    _, ref_sums, ref_max = ref.results()
    for k_launch in (1, 2, 5):
        b = fsb.Batch(common, SIZES, seeds)
        b.run(5, fsb.tuning(block, fpl, k_launch, variant=variant))
        for i in range(b.n):
            got = b.school_state(i)
            for k in got:
                assert np.array_equal(got[k].view(np.uint32), ref_state[i][k].view(np.uint32)), (
                    f"school {i} column {k} differs for block={block} fpl={fpl} "
                    f"steps/launch={k_launch}")
        _, sums, mx = b.results()
        assert np.array_equal(mx, ref_max)
        assert np.allclose(sums, ref_sums, rtol=1e-12, atol=1e-9)
        b.close()
    ref.close()


SCHEDULES = [(fsb.FSB_SCHED_STATIC, 1), (fsb.FSB_SCHED_STATIC, 3),
             (fsb.FSB_SCHED_DYNAMIC, 1), (fsb.FSB_SCHED_DYNAMIC, 3), (fsb.FSB_SCHED_DYNAMIC, 64),
             (fsb.FSB_SCHED_GUIDED, 1), (fsb.FSB_SCHED_GUIDED, 8)]


@pytest.mark.parametrize("variant", [fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN],
                         ids=["prev", "lean"])
@pytest.mark.parametrize("sched,chunk", SCHEDULES, ids=[f"s{s}c{c}" for s, c in SCHEDULES])
def test_work_queue_schedules_give_identical_results(torch_cuda, sched, chunk, variant):
    """Round-robin static chunks, and dynamic and guided schedules that move
    tiles between wavefronts from sweep to sweep: with the same tiles (same
    fish per lane) the columns, maxima and even the sums (tile partials are
    combined in tile order) are identical to the contiguous static
    schedule's, bit for bit."""
    announce(f"schedule {sched} chunk {chunk} variant {variant}")
    common = fsb.FsbConfig(n_fish=0, history_len=5)
    seeds = list(range(len(SIZES)))
    ref = fsb.Batch(common, SIZES, seeds)
    ref.run(5, fsb.tuning(1024, 4, 5, variant=variant))
    ref_state = [ref.school_state(i) for i in range(ref.n)]
    _, ref_sums, ref_max = ref.results()
    ref.close()
    for block, k_launch in ((256, 1), (1024, 2), (1024, 5)):
        b = fsb.Batch(common, SIZES, seeds)
        b.run(5, fsb.tuning(block, 4, k_launch, variant=variant, schedule=sched, chunk_tiles=chunk))
        _, sums, mx = b.results()
        assert np.array_equal(mx, ref_max)
        assert np.array_equal(sums.view(np.uint64), ref_sums.view(np.uint64)), (sums, ref_sums)
        for i in range(b.n):
            got = b.school_state(i)
            for k in got:
                assert np.array_equal(got[k].view(np.uint32), ref_state[i][k].view(np.uint32)), (
                    f"school {i} column {k}, block={block} steps/launch={k_launch}")
        b.close()


def test_dynamic_schedule_matches_oracle(torch_cuda, O):
    announce("dynamic schedule vs oracle")
    common = fsb.FsbConfig(n_fish=0, history_len=6)
    seeds = [29 * i + 1 for i in range(len(SIZES))]
    b = fsb.Batch(common, SIZES, seeds)
    b.run(6, fsb.tuning(256, 8, 3, schedule=fsb.FSB_SCHED_DYNAMIC, chunk_tiles=1))
    check_batch_against_oracle(O, b, 6, what="dynamic")
    b.close()


def test_cfg5_schedules_agree(torch_cuda):
    """The full 4096-school shape for 3 iterations under the static, dynamic
    and guided schedules: identical maxima, sums and columns (columns compared
    on the device)."""
    import torch
    sizes = log_uniform_school_sizes(4096)
    seeds = school_seeds(4096)
    common = fsb.FsbConfig(n_fish=0)
    announce(f"cfg5 schedules, {int(sizes.sum())} fish")
    ref = fsb.Batch(common, sizes, seeds)
    ref.run(3, fsb.tuning(1024, 16, 3))
    _, ref_sums, ref_max = ref.results()
    ref_cols = {k: v.clone() for k, v in ref.cols.items()}
    ref.close()
    del ref
    for sched, chunk in ((fsb.FSB_SCHED_DYNAMIC, 16), (fsb.FSB_SCHED_GUIDED, 4)):
        b = fsb.Batch(common, sizes, seeds)
        b.run(3, fsb.tuning(1024, 16, 3, schedule=sched, chunk_tiles=chunk))
        _, sums, mx = b.results()
        assert np.array_equal(mx, ref_max)
        assert np.array_equal(sums.view(np.uint64), ref_sums.view(np.uint64))
        for k, v in b.cols.items():
            assert torch.equal(v.view(torch.int32), ref_cols[k].view(torch.int32)), (sched, k)
        b.close()
        del b
    del ref_cols
    torch.cuda.empty_cache()


def test_gaps_between_schools_untouched(torch_cuda):
    announce("gaps")
    sizes = [5, 9, 1, 130]
    starts = [0, 16, 40, 48]          # gaps at 5..15, 25..39, 41..47
    common = fsb.FsbConfig(n_fish=0)
    b = fsb.Batch(common, sizes, [1, 2, 3, 4], starts=starts)
    b.sync()
    mask = np.ones(b.cols["x"].numel(), bool)
    for a, n in zip(starts, sizes):
        mask[a:a + n] = False
    for v in b.cols.values():
        v[torch_cuda.from_numpy(mask).to(v.device)] = 12345.0
    b.run(4)
    b.sync()
    for k, v in b.cols.items():
        assert (v.cpu().numpy()[mask] == 12345.0).all(), k
    b.close()


def test_batch_naive_reduction(torch_cuda, O):
    announce("naive")
    common = fsb.FsbConfig(n_fish=0, reduce_mode=fsb.FSB_REDUCE_NAIVE_F32)
    sizes = [3, 1000, 70001]
    b = fsb.Batch(common, sizes, [5, 6, 7])
    b.run(3)
    xy, sums, mx = b.results()
    for i in range(3):
        school, m, s, a = oracle_school(O, sizes[i], [5, 6, 7][i], 3)
        assert mx[i] == m[-1]
        assert_sums_close(sums[i], s[-1], a[-1], tol=1e-3, what=f"naive school {i}")
        assert_columns_equal(b.school_state(i), school, f"naive school {i}")
    b.close()


def test_cfg5_full_shape(torch_cuda, O):
    """4096 schools, log-uniform sizes in [1e3, 1e6] (about 5.9e8 fish), in
    the benchmark's launch shape: the smallest schools are run in full by the
    oracle for 20 iterations and compared bit for bit; every school's record
    is checked against the invariants."""
    sizes = log_uniform_school_sizes(4096)
    seeds = school_seeds(4096)
    steps = 20
    announce(f"cfg5 {sizes.size} schools, {int(sizes.sum())} fish, {steps} iterations")
    common = fsb.FsbConfig(n_fish=0)
    b = fsb.Batch(common, sizes, seeds)
    b.run(steps)
    xy, sums, mx = b.results()
    assert (mx > 0).all() and (mx <= 0.1 * np.sqrt(2) + 1e-4).all()
    assert (sums[:, 0] >= sizes * 1.0 * (1 - 1e-9)).all() and (sums[:, 0] <= sizes * 4.0).all()
    order = np.argsort(sizes)
    picked = list(order[:6]) + list(order[2048:2050]) + [order[-1]]  # and the largest school
    check_batch_against_oracle(O, b, steps, schools=picked, what="cfg5")
    b.close()


def test_autotune_and_cache(torch_cuda, tmp_path):
    announce("autotune")
    cache = tmp_path / "tune.txt"
    os.environ["FSB_AUTOTUNE_CACHE"] = str(cache)
    try:
        common = fsb.FsbConfig(n_fish=0)
        b = fsb.Batch(common, SIZES, list(range(len(SIZES))))
        t0 = b.t
        tune = b.autotune(4)
        d = fsb.tuning_dict(tune)
        assert d["block_size"] in (256, 1024) and d["fish_per_thread"] in (4, 8, 16)
        assert d["steps_per_launch"] >= 1
        assert d["variant"] in (fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN,
                                fsb.FSB_RUN_FUSED_DEEP)
        if d["variant"] == fsb.FSB_RUN_FUSED_DEEP:
            assert d["block_size"] == 256
        assert d["schedule"] in (fsb.FSB_SCHED_STATIC, fsb.FSB_SCHED_DYNAMIC,
                                 fsb.FSB_SCHED_GUIDED)
        assert b.t > t0
        assert fsb.tuning_dict(b.tuning) == d
        assert cache.exists() and cache.read_text().strip()
        b2 = fsb.Batch(common, SIZES, list(range(len(SIZES))))
        assert fsb.tuning_dict(b2.autotune(4)) == d
        assert b2.t == 0, "cached tuning must not probe"
        b.close()
        b2.close()
    finally:
        del os.environ["FSB_AUTOTUNE_CACHE"]


def test_batch_errors(torch_cuda):
    common = fsb.FsbConfig(n_fish=0)
    b = fsb.Batch(common, [10, 20], [1, 2])
    with pytest.raises(fsb.FsbError) as e:
        b.results()
    assert e.value.code == fsb._lib.FSB_ERR_STATE
    with pytest.raises(fsb.FsbError):
        b.run(1, fsb.tuning(333, 8, 1))
    with pytest.raises(fsb.FsbError):
        b.run(1, fsb.tuning(1024, 8, 1, schedule=3, chunk_tiles=1))
    with pytest.raises(fsb.FsbError):
        b.run(1, fsb.tuning(1024, 8, 1, schedule=fsb.FSB_SCHED_DYNAMIC, chunk_tiles=0))
    b.run(1, fsb.tuning(1024, 8, 1, schedule=fsb.FSB_SCHED_STATIC, chunk_tiles=0))
    b.close()
