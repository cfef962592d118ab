"""Greedy and weighted swim rules on the GPU: every path (plain passes, both
persistent variants, batches) must equal the oracle under each rule, bit for
bit in the columns and maxima, sums within the 1e-6 gate."""
import numpy as np
import pytest

import oracle_pins
import paper_2507_20173_amd as fsb
from oracle.oracle import default
from paper_2507_20173_amd.workloads import packed_starts
from parity_util import (assert_columns_equal, assert_sums_close, columns_of, oracle_config,
                         school_of)

pytestmark = pytest.mark.gpu
GREEDY, WEIGHTED = fsb.FSB_SWIM_GREEDY, fsb.FSB_SWIM_WEIGHTED
RULES = [GREEDY, WEIGHTED, GREEDY | WEIGHTED]
RULE_IDS = ["greedy", "weighted", "both"]
MODES = [fsb.FSB_RUN_PLAIN, fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN]
MODE_IDS = ["plain", "prev", "lean"]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[swim rules] {msg}", flush=True)


def history_sums(h):
    return np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)


@pytest.mark.parametrize("name", ["worked_example_greedy.json", "worked_example_weighted.json"])
def test_rule_worked_examples(torch_cuda, name):
    announce(name)
    fx = oracle_pins.load_golden(name)
    c = fx["config"]
    cfg = fsb.FsbConfig(n_fish=len(fx["before"]), pond_half=c["pondHalf"],
                        swim_step=c["swimStep"], w_min=c["weightMin"], w_max=c["weightMax"],
                        swim_rule=c["swimRule"])
    sch = fsb.School(cfg, state=columns_of(oracle_pins.golden_school(fx, "before")))
    d = np.array(fx["displacement"], np.float32)
    sch.step_displaced(torch_cuda.tensor(d[:, 0].copy(), device="cuda"),
                       torch_cuda.tensor(d[:, 1].copy(), device="cuda"))
    assert sch.max_delta() == np.float32(fx["maxDiff"])
    xy, sums = sch.barycentre()
    assert list(sums) == fx["sums"] and list(xy) == fx["barycentre"]
    assert_columns_equal(sch.state(), oracle_pins.golden_school(fx, "after"), name)
    sch.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("rule", RULES, ids=RULE_IDS)
@pytest.mark.parametrize("n,steps", [(5, 4), (1001, 5), (65539, 4), ((1 << 20) + 3, 3)])
def test_rule_matches_oracle(torch_cuda, O, n, steps, rule, mode):
    announce(f"n={n} steps={steps} rule={rule} mode={mode}")
    cfg = fsb.FsbConfig(n_fish=n, seed=900 + n, swim_step=0.5, swim_rule=rule,
                        history_len=steps)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, steps)
    sch = fsb.School(cfg)
    sch.run(steps, mode)
    h = sch.history(0, steps)
    assert np.array_equal(h["max_delta"], m), f"maxima {h['max_delta']} vs {m}"
    assert_sums_close(history_sums(h), s, a, what=f"rule {rule} mode {mode} n={n}")
    assert_columns_equal(sch.state(), school, f"rule {rule} mode {mode} n={n}")
    sch.close()


@pytest.mark.parametrize("rule", RULES, ids=RULE_IDS)
def test_rule_interleaved_forms(torch_cuda, O, rule):
    """plain 2 + prev 3 + lean 2 + plain 1 under a rule == oracle 8."""
    announce(f"interleaved rule={rule}")
    n = 40_009
    cfg = fsb.FsbConfig(n_fish=n, seed=77, swim_step=1.0, swim_rule=rule, history_len=8)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, 8)
    sch = fsb.School(cfg)
    for k, mode in ((2, fsb.FSB_RUN_PLAIN), (3, fsb.FSB_RUN_FUSED_PREV),
                    (2, fsb.FSB_RUN_FUSED_LEAN), (1, fsb.FSB_RUN_PLAIN)):
        sch.run(k, mode)
    h = sch.history(0, 8)
    assert np.array_equal(h["max_delta"], m)
    assert_sums_close(history_sums(h), s, a, what="interleaved")
    assert_columns_equal(sch.state(), school, "interleaved")
    sch.close()


@pytest.mark.parametrize("rule", RULES, ids=RULE_IDS)
@pytest.mark.parametrize("variant", [fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN],
                         ids=["prev", "lean"])
def test_rule_batch_matches_oracle(torch_cuda, O, rule, variant):
    sizes = [1, 3, 64, 257, 1000, 4099, 16385]
    seeds = [5 * i + 2 for i in range(len(sizes))]
    steps = 5
    announce(f"batch rule={rule} variant={variant}")
    common = fsb.FsbConfig(n_fish=0, swim_step=0.5, swim_rule=rule, history_len=steps)
    b = fsb.Batch(common, sizes, seeds, starts=packed_starts(sizes, 4))
    b.run(steps, fsb.tuning(256, 8, 2, variant=variant, schedule=fsb.FSB_SCHED_DYNAMIC,
                            chunk_tiles=1))
    _, sums, mx = b.results()
    for i, (size, seed) in enumerate(zip(sizes, seeds)):
        ocfg = oracle_config(fsb.FsbConfig(n_fish=size, seed=seed, swim_step=0.5, swim_rule=rule))
        school = O.init(ocfg)
        m, s, a = O.run(ocfg, school, 0, steps)
        assert mx[i] == m[-1], f"school {i}"
        assert_sums_close(sums[i], s[-1], a[-1], what=f"batch school {i}")
        assert_columns_equal(b.school_state(i), school, f"batch school {i}")
    b.close()


def test_greedy_long_run_sampled(torch_cuda, O):
    """N = 2^24 under the greedy rule for 300 plain iterations: greedy swimming
    does not depend on weights, so sampled fish followed alone by the oracle
    must match bit for bit; every recorded max is that of a non-negative diff
    (greedy never moves a fish away from the centre)."""
    n, steps = 1 << 24, 300
    announce(f"greedy n={n} {steps} iterations, sampled")
    cfg = fsb.FsbConfig(n_fish=n, seed=0, swim_rule=GREEDY, history_len=steps)
    ocfg = oracle_config(cfg)
    start = fsb.School(cfg)
    idx = np.unique(np.concatenate([np.arange(8), n - 1 - np.arange(8),
                                    np.random.default_rng(4).integers(0, n, 48)]))
    init = start.state()
    start.run(steps)
    got = start.state()
    h = start.history(0, steps)
    assert (h["max_delta"] > 0).all()
    diff = got["prev"] - got["cur"]
    assert (diff >= 0).all()
    school0 = school_of({k: v[idx] for k, v in init.items()})
    for j, i in enumerate(idx):
        f = O.follow_fish(ocfg, int(i), 0, steps, school0[j])
        for k, field in (("x", "x"), ("y", "y"), ("prev", "prevObjective"),
                         ("cur", "currentObjective")):
            assert got[k][i].view(np.uint32) == np.float32(f[field]).view(np.uint32), (i, k)
    start.close()
