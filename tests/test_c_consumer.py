"""The library driven from plain C (tests/c_consumer.c): only include/fsb.h
and the HIP runtime's C API, no Python on the library's side.  On the CPU the
program runs its host-side checks; on a GPU its columns must equal the
oracle's bit for bit and its M and sums must pass the usual gates."""
import os
import subprocess

import numpy as np
import pytest

from oracle.oracle import Config, default
from parity_util import FIELD_OF, assert_sums_close

TESTS = os.path.dirname(os.path.abspath(__file__))
BINARY = os.path.join(TESTS, "c_consumer")
RUN_PLAIN, RUN_FUSED, RUN_FUSED_LEAN = 0, 1, 3


def binary():
    assert os.path.exists(BINARY), "tests/c_consumer is missing: run __graft_entry__.build() first"
    return BINARY


def test_c_consumer_host_checks():
    r = subprocess.run([binary(), "host"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("host ok")


def test_c_consumer_usage_error():
    r = subprocess.run([binary()], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "usage" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("n,steps,mode", [(4099, 7, RUN_PLAIN), (65_539, 5, RUN_FUSED),
                                          (100_003, 4, RUN_FUSED_LEAN),
                                          ((1 << 23) + 7, 6, RUN_FUSED)])
def test_c_consumer_matches_oracle(tmp_path, n, steps, mode):
    print(f"[c consumer] n={n} steps={steps} mode={mode}", flush=True)
    out = tmp_path / "columns.bin"
    # a cooperative launch from a second process is refused while the test
    # process holds the GPU, so the persistent kernels launch ordinarily here
    env = dict(os.environ, FSB_PERSISTENT_LAUNCH="regular")
    r = subprocess.run([binary(), "run", str(n), str(steps), str(mode), "21", str(out)],
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr
    fields = dict(line.split(" ", 1) for line in r.stdout.strip().splitlines())
    assert int(fields["t"]) == steps
    got_m = np.float32(float.fromhex(fields["M"]))
    got_sums = [float.fromhex(v) for v in fields["sums"].split()]

    O = default()
    cfg = Config(numFish=n, seed=21)
    school = O.init(cfg)
    m, s, a = O.run(cfg, school, 0, steps)
    assert got_m.view(np.uint32) == m[-1].view(np.uint32), (got_m, m[-1])
    assert_sums_close(got_sums, s[-1], a[-1], what="C consumer")
    cols = np.fromfile(out, np.float32).reshape(5, n)
    for k, name in enumerate(("x", "y", "w", "prev", "cur")):
        want = np.ascontiguousarray(school[FIELD_OF[name]])
        bad = np.nonzero(cols[k].view(np.uint32) != want.view(np.uint32))[0]
        assert bad.size == 0, f"column {name}: {bad.size} fish differ, first at {bad[0]}"
