"""The allocation-free entry point (fsb_run_static) against the handle-based
one (fsb_attach + fsb_run) on the same school: bit-identical columns and
records, for two calls in a row on the one scratch, the second on a smaller
school, in the per-iteration mode and in the persistent mode."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2507_20173_amd as fsb  # noqa: E402

pytestmark = pytest.mark.gpu

RECORD = fsb.RECORD


def _twin(cfg):
    """A school from the init kernel, and a copy of its columns."""
    a = fsb.School(cfg)
    a.sync()
    b = {k: v.clone() for k, v in a.cols.items()}
    torch.cuda.synchronize()
    return a, b


def _check(cfg, t0, n_steps, mode, a, b):
    """Advance twin a with the handle API and twin b with fsb_run_static from
    iteration t0; compare everything."""
    records = torch.zeros(cfg.history_len * RECORD.itemsize, dtype=torch.uint8, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    fsb.fsb_set_step_index(a.h, t0)
    a.run(n_steps, mode)
    fsb.fsb_run_static(cfg, b, t0, n_steps, mode, records, status)
    torch.cuda.synchronize()
    want = a.history(t0 + n_steps - min(n_steps, cfg.history_len), min(n_steps, cfg.history_len))
    got_ring = records.cpu().numpy().view(RECORD)
    slots = [(t0 + n_steps - len(want) + i) % cfg.history_len for i in range(len(want))]
    got = got_ring[slots]
    assert int(status.item()) == 0
    assert np.array_equal(got["step_lo"], want["step_lo"])
    assert np.array_equal(got["max_delta"].view(np.uint32), want["max_delta"].view(np.uint32))
    for k in ("sum_w", "sum_wx", "sum_wy"):
        assert np.array_equal(got[k].view(np.uint64), want[k].view(np.uint64)), k
    st = a.state()
    for k in fsb.COLUMNS:
        assert np.array_equal(b[k].cpu().numpy().view(np.uint32), st[k].view(np.uint32)), k


@pytest.mark.parametrize("mode", [fsb.FSB_RUN_PLAIN, fsb.FSB_RUN_PLAIN_SPLIT, fsb.FSB_RUN_FUSED],
                         ids=["plain", "split", "persistent"])
def test_static_matches_handle_two_calls(mode):
    print(f"\nfsb_run_static mode={mode}: call 1 n=1048579, call 2 n=4099", flush=True)
    # call 1: a larger school, several grid strides and a ragged tail
    cfg1 = fsb.FsbConfig(n_fish=(1 << 20) + 3, seed=31, history_len=16)
    a1, b1 = _twin(cfg1)
    _check(cfg1, 0, 11, mode, a1, b1)
    a1.close()
    # call 2 right after, on the same scratch: a smaller school from iteration 7
    cfg2 = fsb.FsbConfig(n_fish=4099, seed=32, history_len=4)
    a2, b2 = _twin(cfg2)
    _check(cfg2, 7, 9, mode, a2, b2)
    a2.close()
