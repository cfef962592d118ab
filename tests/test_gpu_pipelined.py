"""FSB_RUN_PLAIN's pipelined launches (the feed of iteration t - 1 and the
swim of t in one pass) against the oracle, and against fsb_step's two
passes (FSB_RUN_PLAIN_SPLIT).

Every run checks every iteration's record (the max bit for bit, the sums
within 1e-6 of the oracle's binary64 reference) and the final columns bit
for bit, cur included (the pipelined passes leave cur to the run's closing
feed pass)."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default
from parity_util import assert_columns_equal, assert_sums_close, oracle_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[pipelined] {msg}", flush=True)


def history_sums(h):
    return np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)


def check_run(O, sch, ocfg, school, t0, steps, tol=1e-6, what=""):
    """Run `steps` pipelined iterations on the school and the oracle; compare."""
    m, s, a = O.run(ocfg, school, t0, steps)
    sch.run(steps)
    h = sch.history(t0, steps)
    assert np.array_equal(h["step_lo"], np.arange(t0, t0 + steps)), what
    assert np.array_equal(h["max_delta"], m), f"{what}: maxima differ"
    assert_sums_close(history_sums(h), s, a, tol=tol, what=what)
    assert_columns_equal(sch.state(), school, what)


# Ragged tails (n % 4 = 1, 2, 3), one group, several blocks, several rounds
# of the pipelined grid (512 blocks x 256 threads x 4 fish = 2^19 per round).
SIZES = [1, 2, 3, 4, 5, 7, 65, 1001, 4099, 65538, (1 << 20) + 3, (1 << 21) + 1]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("steps", [2, 3, 11])
def test_pipelined_matches_oracle(torch_cuda, O, n, steps):
    if n > 70_000 and steps > 3:
        pytest.skip("large schools: the shorter runs cover the shape")
    announce(f"n={n} steps={steps}")
    cfg = fsb.FsbConfig(n_fish=n, seed=0xF00D + n, history_len=steps)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    sch = fsb.School(cfg)
    check_run(O, sch, ocfg, school, 0, steps, what=f"n={n} steps={steps}")
    sch.close()


def test_one_launch_per_iteration(torch_cuda):
    """n iterations: one swim pass, n - 1 pipelined passes, one feed pass."""
    announce("launch counts")
    sch = fsb.School(fsb.FsbConfig(n_fish=100_000, seed=4))
    fsb.fsb_profile_enable(sch.h, 1)
    fsb.fsb_kernel_times(sch.h)
    sch.run(9)
    counts, _ = fsb.fsb_kernel_times(sch.h)
    assert counts[fsb.FSB_KERNEL_SWIM_EVAL] == 1
    assert counts[fsb.FSB_KERNEL_FEED_SWIM] == 8
    assert counts[fsb.FSB_KERNEL_FEED_BARY] == 1
    sch.run(1)  # a single iteration is fsb_step's two passes
    counts, _ = fsb.fsb_kernel_times(sch.h)
    assert (counts[fsb.FSB_KERNEL_SWIM_EVAL], counts[fsb.FSB_KERNEL_FEED_SWIM],
            counts[fsb.FSB_KERNEL_FEED_BARY]) == (1, 0, 1)
    sch.close()


def test_interleaved_with_every_mode(torch_cuda, O):
    """Pipelined runs between single steps, split runs and persistent runs:
    every record of the 32 iterations and the final columns."""
    announce("interleaved")
    n = 300_007
    cfg = fsb.FsbConfig(n_fish=n, seed=77, history_len=64)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, 32)
    sch = fsb.School(cfg)
    sch.run(4)
    sch.step()
    sch.run(2)
    sch.run(3, fsb.FSB_RUN_PLAIN_SPLIT)
    sch.run(5)
    sch.run(4, fsb.FSB_RUN_FUSED)
    sch.run(6)
    sch.run(3, fsb.FSB_RUN_FUSED_PREV)
    sch.run(1)
    sch.run(3)
    assert sch.t == 32
    h = sch.history(0, 32)
    assert np.array_equal(h["step_lo"], np.arange(32))
    assert np.array_equal(h["max_delta"], m)
    assert_sums_close(history_sums(h), s, a, what="interleaved")
    assert_columns_equal(sch.state(), school, "interleaved")
    sch.close()


def test_pipelined_equals_split(torch_cuda):
    """The pipelined and the two-pass launches leave the same columns and
    records, bit for bit: both feed every iteration on the same grid."""
    announce("pipelined vs split")
    n = (1 << 22) + 3
    out = {}
    for mode in (fsb.FSB_RUN_PLAIN, fsb.FSB_RUN_PLAIN_SPLIT):
        sch = fsb.School(fsb.FsbConfig(n_fish=n, seed=21, history_len=12))
        sch.run(12, mode)
        out[mode] = (sch.state(), sch.history(0, 12))
        sch.close()
    (ca, ha), (cb, hb) = out[fsb.FSB_RUN_PLAIN], out[fsb.FSB_RUN_PLAIN_SPLIT]
    for k in ca:
        assert np.array_equal(ca[k].view(np.uint32), cb[k].view(np.uint32)), k
    assert ha.tobytes() == hb.tobytes()


def test_pipelined_naive_sums(torch_cuda, O):
    announce("naive sums")
    n = 100_003
    cfg = fsb.FsbConfig(n_fish=n, seed=6, reduce_mode=fsb.FSB_REDUCE_NAIVE_F32, history_len=6)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    sch = fsb.School(cfg)
    check_run(O, sch, ocfg, school, 0, 6, tol=1e-3, what="naive")
    sch.close()


@pytest.mark.parametrize("rule", [fsb.FSB_SWIM_GREEDY, fsb.FSB_SWIM_WEIGHTED,
                                  fsb.FSB_SWIM_GREEDY | fsb.FSB_SWIM_WEIGHTED],
                         ids=["greedy", "weighted", "both"])
def test_pipelined_swim_rules(torch_cuda, O, rule):
    """The weighted rule swims with the weight the same pass has just fed."""
    announce(f"rule={rule}")
    n = 50_001
    cfg = fsb.FsbConfig(n_fish=n, seed=31 + rule, swim_rule=rule, w_min=0.5,
                        w_init_lo=1.0, w_init_hi=3.0, w_max=4.0, history_len=9)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    sch = fsb.School(cfg)
    check_run(O, sch, ocfg, school, 0, 9, what=f"rule {rule}")
    sch.close()


def test_pipelined_zero_swim(torch_cuda):
    """S = 0: every maximum is 0, so no fish is fed and nothing moves."""
    announce("zero swim")
    sch = fsb.School(fsb.FsbConfig(n_fish=9_999, seed=3, swim_step=0.0, history_len=5))
    before = sch.state()
    sch.run(5)
    assert (sch.history(0, 5)["max_delta"] == 0).all()
    after = sch.state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    sch.close()


def test_pipelined_resumes_at_an_index(torch_cuda, O):
    """Attached at t = 2^32 - 6, run to the last iteration the counter allows."""
    announce("attach near the index limit")
    n = 10_001
    cfg = fsb.FsbConfig(n_fish=n, seed=12, history_len=8)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    O.run(ocfg, school, 0, 2)
    t0 = (1 << 32) - 6
    state = {k: np.ascontiguousarray(school[f]) for k, f in
             (("x", "x"), ("y", "y"), ("w", "weight"), ("prev", "prevObjective"),
              ("cur", "currentObjective"))}
    sch = fsb.School(cfg, state=state, t=t0)
    check_run(O, sch, ocfg, school, t0, 6, what="near 2^32")
    with pytest.raises(fsb.FsbError):
        sch.run(2)
    sch.close()


def test_cfg2_pipelined_prefix(torch_cuda, O):
    """The benchmarked school (N = 2^24) in the benchmark's launch shape."""
    n, steps = 1 << 24, 4
    announce(f"cfg2 N={n} prefix {steps}")
    cfg = fsb.FsbConfig(n_fish=n, seed=0, history_len=steps)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    sch = fsb.School(cfg)
    check_run(O, sch, ocfg, school, 0, steps, what="cfg2 pipelined")
    sch.close()


def test_pipelined_record_ring_wraps(torch_cuda, O):
    """A ring of 3 records over 17 pipelined iterations: each record lands in
    slot t mod 3 one launch late, and the last three are the oracle's."""
    announce("record ring of 3")
    n = 20_003
    cfg = fsb.FsbConfig(n_fish=n, seed=41, history_len=3)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, 17)
    sch = fsb.School(cfg)
    sch.run(17)
    h = sch.history(14, 3)
    assert np.array_equal(h["step_lo"], np.arange(14, 17))
    assert np.array_equal(h["max_delta"], m[14:])
    assert_sums_close(history_sums(h), s[14:], a[14:], what="ring")
    with pytest.raises(fsb.FsbError):
        sch.history(13, 1)
    assert_columns_equal(sch.state(), school, "ring")
    sch.close()
