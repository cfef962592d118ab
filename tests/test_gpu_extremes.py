"""Parameter extremes that the library accepts, on every path: each must
still equal the oracle bit for bit (columns and maxima; sums within the
1e-6 gate).

- a pond of half-width 2^-63: every x*x + y*y lies below 2^-96, many in the
  subnormal range, so every objective takes the kernels' slow square-root
  branch and the products round in gradual underflow;
- a pond of half-width 2^63, the largest accepted: x*x + y*y reaches 2^127;
- the smallest nonzero swim step, 2^-103, in the default pond: every move
  rounds away, so every difference is zero, M = 0 and feeding is skipped;
- negative weights (limits [-4, -1]) and weights spanning [-2^24, 2^24], the
  widest accepted: the sum of weights can be near zero, which the
  condition-normalised gate still measures."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default
from paper_2507_20173_amd.workloads import packed_starts
from parity_util import assert_columns_equal, assert_sums_close, oracle_config

EXTREMES = {
    "tiny_pond": dict(pond_half=2.0 ** -63, swim_step=2.0 ** -64),
    "huge_pond": dict(pond_half=2.0 ** 63, swim_step=2.0 ** 62),
    "min_step": dict(swim_step=2.0 ** -103),
    "negative_weights": dict(w_init_lo=-2.0, w_init_hi=-1.0, w_min=-4.0, w_max=-1.0),
    "widest_weights": dict(w_init_lo=-(2.0 ** 24), w_init_hi=2.0 ** 24, w_min=-(2.0 ** 24),
                           w_max=2.0 ** 24),
}
MODES = {"plain": fsb.FSB_RUN_PLAIN, "prev": fsb.FSB_RUN_FUSED_PREV,
         "lean": fsb.FSB_RUN_FUSED_LEAN}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[extremes] {msg}", flush=True)


def history_sums(h):
    return np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", list(MODES), ids=list(MODES))
@pytest.mark.parametrize("case", list(EXTREMES), ids=list(EXTREMES))
def test_extreme_school_matches_oracle(torch_cuda, O, case, mode):
    n, steps = 65_539, 4
    announce(f"{case} n={n} steps={steps} mode={mode}")
    cfg = fsb.FsbConfig(n_fish=n, seed=31, history_len=steps, **EXTREMES[case])
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, steps)
    sch = fsb.School(cfg)
    sch.run(steps, MODES[mode])
    h = sch.history(0, steps)
    assert np.array_equal(h["max_delta"].view(np.uint32), m.view(np.uint32)), (h["max_delta"], m)
    assert_sums_close(history_sums(h), s, a, what=f"{case} {mode}")
    assert_columns_equal(sch.state(), school, f"{case} {mode}")
    sch.close()


def test_tiny_pond_exercises_the_slow_square_root(O):
    """The premise of the tiny-pond case, on the oracle's own school: every
    squared distance is below 2^-96 and some are subnormal."""
    cfg = fsb.FsbConfig(n_fish=65_539, seed=31, **EXTREMES["tiny_pond"])
    school = O.init(oracle_config(cfg))
    x, y = school["x"], school["y"]
    s = x * x + y * y
    assert s.dtype == np.float32
    assert (s < np.float32(2.0 ** -96)).all()
    assert ((s > 0) & (s < np.finfo(np.float32).tiny)).any()


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN],
                         ids=["prev", "lean"])
@pytest.mark.parametrize("case", ["tiny_pond", "huge_pond", "widest_weights"])
def test_extreme_batch_matches_oracle(torch_cuda, O, case, variant):
    sizes = [3, 1000, 4099, 20_001]
    seeds = [7, 8, 9, 10]
    steps = 4
    announce(f"batch {case} variant={variant}")
    common = fsb.FsbConfig(n_fish=0, history_len=steps, **EXTREMES[case])
    b = fsb.Batch(common, sizes, seeds, starts=packed_starts(sizes, 4))
    b.run(steps, fsb.tuning(256, 4, 2, variant=variant))
    _, sums, mx = b.results()
    for i, (size, seed) in enumerate(zip(sizes, seeds)):
        ocfg = oracle_config(fsb.FsbConfig(n_fish=size, seed=seed, **EXTREMES[case]))
        school = O.init(ocfg)
        m, s, a = O.run(ocfg, school, 0, steps)
        assert mx[i].view(np.uint32) == m[-1].view(np.uint32), f"school {i}"
        assert_sums_close(sums[i], s[-1], a[-1], what=f"batch {case} school {i}")
        assert_columns_equal(b.school_state(i), school, f"batch {case} school {i}")
    b.close()
