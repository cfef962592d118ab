"""Helpers shared by the GPU parity tests: moving schools between the
oracle's record layout and the library's columns, and the comparison
gates."""
from __future__ import annotations

import numpy as np

from oracle.oracle import FISH, Config

# oracle field -> library column
FIELD_OF = {"x": "x", "y": "y", "w": "weight", "prev": "prevObjective",
            "cur": "currentObjective"}

# Reduction gates: sum w relative to itself; the signed sums relative to
# the sum of |terms| (the school is centred at the origin, so sum w*x can be
# ~0 and a plain relative error would be meaningless).
REL_TOL = 1e-6


def oracle_config(cfg) -> Config:
    return Config(numFish=cfg.n_fish, seed=cfg.seed, pondHalf=cfg.pond_half,
                  swimStep=cfg.swim_step, initWeightLo=cfg.w_init_lo,
                  initWeightHi=cfg.w_init_hi, weightMin=cfg.w_min, weightMax=cfg.w_max,
                  swimRule=cfg.swim_rule)


def columns_of(school: np.ndarray) -> dict:
    return {k: np.ascontiguousarray(school[f]) for k, f in FIELD_OF.items()}


def school_of(cols: dict) -> np.ndarray:
    s = np.zeros(len(cols["x"]), FISH)
    for k, f in FIELD_OF.items():
        s[f] = cols[k]
    return s


def assert_columns_equal(got: dict, school: np.ndarray, what: str = "") -> None:
    """Bit-exact comparison of every column with the oracle's school."""
    for k, f in FIELD_OF.items():
        g = np.asarray(got[k]).view(np.uint32)
        e = np.ascontiguousarray(school[f]).view(np.uint32)
        bad = np.nonzero(g != e)[0]
        assert bad.size == 0, (
            f"{what} column {k}: {bad.size} fish differ, first at {bad[0]}: "
            f"got {np.asarray(got[k])[bad[0]]!r} want {school[f][bad[0]]!r}")


def sum_errors(got_sums, ref_sums, ref_abs) -> np.ndarray:
    """(rel error of sum w, |err| / sum|w x|, |err| / sum|w y|)."""
    got = np.asarray(got_sums, np.float64)
    ref = np.asarray(ref_sums, np.float64)
    den = np.asarray(ref_abs, np.float64)
    return np.abs(got - ref) / den


def assert_sums_close(got_sums, ref_sums, ref_abs, tol: float = REL_TOL, what: str = ""):
    err = sum_errors(got_sums, ref_sums, ref_abs)
    assert (err <= tol).all(), f"{what} sums {got_sums} vs {ref_sums}: errors {err}"
    return err


def assert_sampled_fish(O, ocfg: Config, start: dict, got: dict, max_delta, sample,
                        what: str = "") -> None:
    """Every field of the sampled fish bit for bit against the oracle
    following each fish alone from its starting record (start: columns at the
    run's first iteration), fed with the run's recorded maxima (max_delta,
    one per iteration): at sizes where the whole-school oracle would take
    minutes, the fish's own arithmetic is still checked exactly."""
    steps = len(max_delta)
    for i in sample:
        rec = np.zeros(1, FISH)
        for k, f in FIELD_OF.items():
            rec[f] = start[k][i]
        f = O.follow_fish_fed(ocfg, int(i), 0, steps, rec[0], max_delta)
        for k, fld in FIELD_OF.items():
            g, e = np.float32(got[k][i]), np.float32(f[fld])
            assert g.view(np.uint32) == e.view(np.uint32), f"{what} fish {i} {k}: {g!r} vs {e!r}"
