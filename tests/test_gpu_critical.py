"""Critical reduction mode (the GPU counterpart of the critical-section
construct of Sec. 2.3.2, Experiment 3): every fish updates the shared max word
and the three float32 sums with its own atomic.  The max is order-independent,
so it and every column must still equal the oracle's bit for bit; the sums
are float32 recursive sums in an arbitrary order, held to the a-priori bound
of such a sum (Higham, Accuracy and Stability of Numerical Algorithms, 2nd
ed., eq. 4.4): |S_hat - S| <= gamma_(n-1) sum|terms|, plus one rounding of
each product w*x against the oracle's exact products."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
import oracle_pins
from oracle.oracle import default
from parity_util import assert_columns_equal, assert_sums_close, columns_of, oracle_config

pytestmark = pytest.mark.gpu
CRIT = fsb.FSB_REDUCE_CRITICAL_F32
U = 2.0 ** -24


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[critical] {msg}", flush=True)


def float_sum_bound(n: int) -> float:
    """Relative (to sum|terms|) error bound of an n-term float32 sum of
    rounded float32 products, any order."""
    k = max(n - 1, 0) * U
    assert k < 0.5, "the bound is only meaningful for n * 2^-24 well below 1"
    gamma = k / (1.0 - k)
    return gamma + U * (1.0 + gamma)


def history_sums(h):
    return np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)


@pytest.mark.parametrize("n,steps", [(1, 3), (5, 4), (1001, 6), (65539, 4), ((1 << 20) + 3, 3)])
def test_critical_matches_oracle(torch_cuda, O, n, steps):
    """Every iteration's M (so the shared max word is cleared between
    iterations), the columns bit-exact, the sums within the bound."""
    announce(f"n={n} steps={steps}")
    cfg = fsb.FsbConfig(n_fish=n, seed=777 + n, reduce_mode=CRIT, history_len=steps)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, s, a = O.run(ocfg, school, 0, steps)
    sch = fsb.School(cfg)
    sch.run(steps, fsb.FSB_RUN_PLAIN)
    h = sch.history(0, steps)
    assert np.array_equal(h["step_lo"], np.arange(steps))
    assert np.array_equal(h["max_delta"], m), f"maxima {h['max_delta']} vs {m}"
    assert_sums_close(history_sums(h), s, a, tol=float_sum_bound(n), what=f"critical n={n}")
    assert_columns_equal(sch.state(), school, f"critical n={n}")
    sch.close()


def test_critical_equals_tree_columns(torch_cuda):
    """Same school under the tree and the critical reduction: identical
    columns and maxima at every iteration."""
    announce("critical vs compensated tree")
    n, steps = 300_007, 5
    out = []
    for mode in (fsb.FSB_REDUCE_COMPENSATED, CRIT):
        sch = fsb.School(fsb.FsbConfig(n_fish=n, seed=42, reduce_mode=mode, history_len=steps))
        sch.run(steps)
        out.append((sch.state(), sch.history(0, steps)["max_delta"]))
        sch.close()
    for k in fsb.COLUMNS:
        assert np.array_equal(out[0][0][k].view(np.uint32), out[1][0][k].view(np.uint32)), k
    assert np.array_equal(out[0][1], out[1][1])


def test_critical_worked_example_exact(torch_cuda):
    """The 4-fish worked example: every term and partial sum is exact in
    binary32, so the atomic sums are exact in any order."""
    announce("worked example")
    fx = oracle_pins.load_golden("worked_example_4fish.json")
    c = fx["config"]
    cfg = fsb.FsbConfig(n_fish=len(fx["before"]), pond_half=c["pondHalf"],
                        swim_step=c["swimStep"], w_min=c["weightMin"], w_max=c["weightMax"],
                        reduce_mode=CRIT)
    sch = fsb.School(cfg, state=columns_of(oracle_pins.golden_school(fx, "before")))
    d = np.array(fx["displacement"], np.float32)
    sch.step_displaced(torch_cuda.tensor(d[:, 0].copy(), device="cuda"),
                       torch_cuda.tensor(d[:, 1].copy(), device="cuda"))
    assert sch.max_delta() == np.float32(fx["maxDiff"])
    xy, sums = sch.barycentre()
    assert list(sums) == fx["sums"] and list(xy) == fx["barycentre"]
    assert_columns_equal(sch.state(), oracle_pins.golden_school(fx, "after"), "worked example")
    sch.close()


def test_critical_zero_swim(torch_cuda):
    announce("zero swim")
    cfg = fsb.FsbConfig(n_fish=4099, seed=8, swim_step=0.0, reduce_mode=CRIT, history_len=3)
    sch = fsb.School(cfg)
    before = sch.state()
    sch.run(3)
    assert (sch.history(0, 3)["max_delta"] == 0).all()
    after = sch.state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    sch.close()


def test_critical_full_size_iteration(torch_cuda, O):
    """N = 2^24 (the plain benchmark's school) for one iteration: columns and
    M bit-exact against the oracle.  At this size the float32 sums stagnate
    (n * 2^-24 = 1 leaves no useful a-priori bound); only their sign-free
    part is checked: sum w stays within [N w_min, N w_max]."""
    n = 1 << 24
    announce(f"n={n} one iteration")
    cfg = fsb.FsbConfig(n_fish=n, seed=0, reduce_mode=CRIT, history_len=1)
    ocfg = oracle_config(cfg)
    school = O.init(ocfg)
    m, _, _ = O.run(ocfg, school, 0, 1)
    sch = fsb.School(cfg)
    sch.step()
    assert sch.max_delta() == m[-1]
    _, sums = sch.barycentre()
    assert n * cfg.w_min * 0.9 <= sums[0] <= n * cfg.w_max * 1.1
    assert_columns_equal(sch.state(), school, "critical n=2^24")
    sch.close()


def test_critical_is_refused_by_persistent_and_batched_forms(torch_cuda):
    announce("unsupported forms")
    sch = fsb.School(fsb.FsbConfig(n_fish=1000, seed=1, reduce_mode=CRIT))
    for mode in (fsb.FSB_RUN_FUSED, fsb.FSB_RUN_FUSED_PREV, fsb.FSB_RUN_FUSED_LEAN):
        with pytest.raises(fsb.FsbError) as e:
            sch.run(2, mode)
        assert e.value.code == fsb._lib.FSB_ERR_UNSUPPORTED
    sch.run(2, fsb.FSB_RUN_PLAIN)  # the handle still works
    assert sch.max_delta() > 0
    sch.close()
    with pytest.raises(fsb.FsbError) as e:
        fsb.Batch(fsb.FsbConfig(n_fish=0, reduce_mode=CRIT), [10, 20], [1, 2])
    assert e.value.code == fsb._lib.FSB_ERR_UNSUPPORTED
