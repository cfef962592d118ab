"""Register-resident persistent mode (FSB_RUN_FUSED_REGS): every fish of the
school stays in registers for the whole launch.  Columns and maxima must
equal the oracle's bit for bit, sums within the 1e-6 gate, at sizes that
take one, two and four groups of four fish per thread, and across launches
interleaved with the other modes."""
import numpy as np
import pytest

import paper_2507_20173_amd as fsb
from oracle.oracle import default
from parity_util import assert_columns_equal, assert_sums_close, oracle_config

pytestmark = pytest.mark.gpu
REGS = fsb.FSB_RUN_FUSED_REGS


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


@pytest.fixture(scope="module")
def O():
    return default()


def announce(msg):
    print(f"[regs] {msg}", flush=True)


def history_sums(h):
    return np.stack([h["sum_w"], h["sum_wx"], h["sum_wy"]], 1)


def check_run(O, cfg, runs, what):
    """Run (k, mode) pairs on one school; compare with the oracle's run of
    the same total length."""
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
    tol = 1e-3 if cfg.reduce_mode == fsb.FSB_REDUCE_NAIVE_F32 else 1e-6
    assert_sums_close(history_sums(h), s, a, tol=tol, what=what)
    assert_columns_equal(sch.state(), school, what)
    sch.close()


# On MI355X the kernel runs 256 blocks of 512 threads: one group per thread up
# to 2^19 fish, two up to 2^20, four up to 2^21 (plus up to 3 tail fish).
@pytest.mark.parametrize("n,steps", [(1, 4), (3, 2), (5, 5), (64, 3), (1001, 6), (4097, 4),
                                     (65539, 4), (1 << 19, 3), ((1 << 19) + 5, 3),
                                     ((1 << 20) + 3, 3), ((1 << 20) + 6, 3), ((1 << 21) + 3, 2)])
def test_regs_matches_oracle(torch_cuda, O, n, steps):
    announce(f"n={n} steps={steps}")
    check_run(O, fsb.FsbConfig(n_fish=n, seed=808 + n, history_len=steps), [(steps, REGS)],
              f"regs n={n}")


def test_regs_interleaved_with_every_mode(torch_cuda, O):
    """plain 2 + regs 3 + prev 2 + regs 1 + lean 2 + regs 2 == oracle 12."""
    announce("interleaved")
    cfg = fsb.FsbConfig(n_fish=300_007, seed=12, history_len=12)
    check_run(O, cfg, [(2, fsb.FSB_RUN_PLAIN), (3, REGS), (2, fsb.FSB_RUN_FUSED_PREV), (1, REGS),
                       (2, fsb.FSB_RUN_FUSED_LEAN), (2, REGS)], "interleaved")


@pytest.mark.parametrize("rule", [fsb.FSB_SWIM_GREEDY, fsb.FSB_SWIM_WEIGHTED,
                                  fsb.FSB_SWIM_GREEDY | fsb.FSB_SWIM_WEIGHTED],
                         ids=["greedy", "weighted", "both"])
def test_regs_swim_rules(torch_cuda, O, rule):
    announce(f"rule={rule}")
    cfg = fsb.FsbConfig(n_fish=(1 << 20) + 7, seed=13, swim_step=0.5, swim_rule=rule,
                        history_len=5)
    check_run(O, cfg, [(5, REGS)], f"regs rule {rule}")


def test_regs_naive_reduction(torch_cuda, O):
    announce("naive")
    cfg = fsb.FsbConfig(n_fish=100_003, seed=14, reduce_mode=fsb.FSB_REDUCE_NAIVE_F32,
                        history_len=4)
    check_run(O, cfg, [(4, REGS)], "regs naive")


def test_regs_zero_swim(torch_cuda):
    announce("zero swim")
    sch = fsb.School(fsb.FsbConfig(n_fish=7777, seed=3, swim_step=0.0, history_len=5))
    before = sch.state()
    sch.run(5, REGS)
    assert (sch.history(0, 5)["max_delta"] == 0).all()
    after = sch.state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    sch.close()


def test_regs_is_deterministic(torch_cuda):
    announce("determinism")
    cfg = fsb.FsbConfig(n_fish=(1 << 20) + 1, seed=9, history_len=6)
    runs = []
    for _ in range(2):
        sch = fsb.School(cfg)
        sch.run(6, REGS)
        runs.append(sch.history(0, 6).tobytes())
        sch.close()
    assert runs[0] == runs[1]


def test_regs_refuses_a_school_too_large(torch_cuda):
    """2^22 fish would need eight groups per thread on MI355X's 256 blocks;
    the refusal leaves the handle usable."""
    announce("too large")
    sch = fsb.School(fsb.FsbConfig(n_fish=1 << 22, seed=1))
    with pytest.raises(fsb.FsbError) as e:
        sch.run(2, REGS)
    assert e.value.code == fsb._lib.FSB_ERR_UNSUPPORTED
    sch.run(1, fsb.FSB_RUN_FUSED)
    assert sch.max_delta() > 0
    sch.close()


def test_regs_refuses_the_critical_reduction(torch_cuda):
    sch = fsb.School(fsb.FsbConfig(n_fish=1000, seed=1,
                                   reduce_mode=fsb.FSB_REDUCE_CRITICAL_F32))
    with pytest.raises(fsb.FsbError) as e:
        sch.run(2, REGS)
    assert e.value.code == fsb._lib.FSB_ERR_UNSUPPORTED
    sch.close()
