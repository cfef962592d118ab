"""Pins of the CPU oracle against facts fixed outside it.

Each pin takes a loaded ``Oracle`` and raises ``AssertionError`` when the
oracle disagrees with:
  * ATen's open-source Philox4_32 engine, an independent third implementation
    of Philox4x32-10 (words and counter layout);
  * the exact value of the u32 -> float maps, over every 24-bit input;
  * hand-computed worked examples (tests/golden/);
  * special cases with closed forms: zero swim, uniform weights (barycentre =
    arithmetic mean, numpy's mean), point-symmetric dyadic schools (sums
    exactly 0);
  * invariants of the method (pond bound, weight limits, triangle inequality
    on the objective change, sign of the weight change);
  * ``math.fsum`` (correctly rounded exact sum) for the reference sums;
  * step-index composition.
``run_all`` collects the failures; ``test_oracle_mutants.py`` shows that a
plausible mistake planted in the oracle source trips at least one pin.
"""
from __future__ import annotations

import functools
import json
import math
import os
import subprocess
import tempfile

import numpy as np

from oracle.oracle import (DOMAIN_INIT, DOMAIN_SWIM, FISH, FISH_F64, SWIM_GREEDY, SWIM_WEIGHTED,
                           Config)

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
FIELDS = ("x", "y", "weight", "prevObjective", "currentObjective")

f32 = np.float32


# --------------------------------------------------------------------------
# ATen's Philox4_32 (torch/include/ATen/core/PhiloxRNGEngine.h)
# --------------------------------------------------------------------------

class AtenUnavailable(RuntimeError):
    pass


@functools.lru_cache(maxsize=1)
def aten_helper() -> str:
    """Build tests/aten_philox_words.cpp against torch's headers (once)."""
    try:
        import torch
    except ImportError as e:  # pragma: no cover
        raise AtenUnavailable(str(e))
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        raise AtenUnavailable("ATen PhiloxRNGEngine.h not found")
    out = os.path.join(tempfile.mkdtemp(prefix="aten_philox_"), "aten_philox")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc,
                    os.path.join(HERE, "aten_philox_words.cpp"), "-o", out],
                   check=True)
    return out


def aten_words(seeds, subsequences, offsets) -> np.ndarray:
    """(n, 4) words of at::Philox4_32(seed, subsequence, offset)."""
    lines = "".join(f"{int(s)} {int(q)} {int(o)}\n"
                    for s, q, o in zip(seeds, subsequences, offsets))
    res = subprocess.run([aten_helper()], input=lines, capture_output=True,
                         text=True, check=True)
    return np.array([[int(w) for w in ln.split()] for ln in res.stdout.splitlines()],
                    dtype=np.uint32).reshape(-1, 4)


def _u64(rng, n):
    hi = rng.integers(0, 2**32, n, dtype=np.uint64)
    lo = rng.integers(0, 2**32, n, dtype=np.uint64)
    return [int(h) << 32 | int(l) for h, l in zip(hi, lo)]


# --------------------------------------------------------------------------
# Random-number pins
# --------------------------------------------------------------------------

def pin_philox_matches_aten(O):
    """Philox4x32-10 words equal ATen's for random and edge (key, counter)."""
    rng = np.random.default_rng(20250727)
    edge = [0, 1, 2**32 - 1, 2**32, 2**63, 2**64 - 1]
    seeds = edge + _u64(rng, 300)
    subs = edge[::-1] + _u64(rng, 300)
    offs = edge + _u64(rng, 300)
    want = aten_words(seeds, subs, offs)
    counters = [(o & 0xFFFFFFFF, o >> 32, q & 0xFFFFFFFF, q >> 32)
                for q, o in zip(subs, offs)]
    keys = [(s & 0xFFFFFFFF, s >> 32) for s in seeds]
    got = O.philox(counters, keys)
    assert np.array_equal(got, want), "Philox words differ from ATen's engine"


def pin_fish_word_layout(O):
    """Fish i draws words 2(i&1), 2(i&1)+1 of the call with counter
    (pair lo, pair hi, sub-stream, domain), key = seed, pair = i >> 1."""
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, DOMAIN_SWIM), (5, 1, 3, DOMAIN_SWIM), (5, 2**33 + 3, 1, DOMAIN_INIT),
             (2**64 - 1, 2**40 + 1, 2**32 - 1, DOMAIN_SWIM)]
    for _ in range(60):
        cases.append((_u64(rng, 1)[0], int(rng.integers(0, 2**62)),
                      int(rng.integers(0, 2**32)), int(rng.integers(0, 2))))
    want = aten_words([c[0] for c in cases], [c[2] | (c[3] << 32) for c in cases],
                      [c[1] >> 1 for c in cases])
    for (seed, fish, sub, dom), w in zip(cases, want):
        j = 2 * (fish & 1)
        assert O.fish_words(seed, fish, sub, dom) == (int(w[j]), int(w[j + 1])), (
            f"fish words differ for seed={seed} fish={fish} sub={sub} domain={dom}")


def pin_unit_map_exhaustive(O):
    """u = (r>>8)*2^-24 and v = 2u-1 exactly, for all 2^24 top-24-bit values."""
    k = np.arange(1 << 24, dtype=np.uint64)
    low = (k * np.uint64(2654435761)) & np.uint64(0xFF)
    r = ((k << np.uint64(8)) | low).astype(np.uint32)
    u, v = O.units(r)
    kf = k.astype(np.float64)
    assert np.array_equal(u.astype(np.float64), kf * 2.0**-24), "u map not exact"
    assert np.array_equal(v.astype(np.float64), kf * 2.0**-23 - 1.0), "v map not exact"
    assert u.min() == 0.0 and u.max() < 1.0 and v.min() == -1.0 and v.max() < 1.0
    assert not np.signbit(v[v == 0]).any(), "v produced -0"


def pin_philox_statistics(O):
    """Gross-defect check on the swim stream: byte histogram, mean, and
    independence of the two words a fish draws."""
    n = 1 << 18
    pair = np.arange(n, dtype=np.uint64)
    counters = np.stack([pair & np.uint64(0xFFFFFFFF), pair >> np.uint64(32),
                         np.full(n, 7, np.uint64), np.zeros(n, np.uint64)], 1)
    keys = np.tile(np.array([[0x1234, 0x5678]], np.uint64), (n, 1))
    w = O.philox(counters, keys)
    top = (w >> 24).ravel()
    hist = np.bincount(top, minlength=256)
    exp = top.size / 256
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert 255 - 8 * math.sqrt(510) < chi2 < 255 + 8 * math.sqrt(510), f"chi2={chi2}"
    u = (w >> 8).astype(np.float64) * 2.0**-24
    assert abs(u.mean() - 0.5) < 8 / math.sqrt(12 * u.size)
    c = np.corrcoef(u[:, 0], u[:, 1])[0, 1]
    assert abs(c) < 8 / math.sqrt(n), f"word correlation {c}"


# --------------------------------------------------------------------------
# Worked examples and special cases
# --------------------------------------------------------------------------

def load_golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def golden_school(fx: dict, key: str) -> np.ndarray:
    return np.array([tuple(f[k] for k in FIELDS) for f in fx[key]], FISH)


def golden_config(fx: dict) -> Config:
    c = fx["config"]
    return Config(numFish=len(fx["before"]), pondHalf=c["pondHalf"],
                  swimStep=c["swimStep"], weightMin=c["weightMin"],
                  weightMax=c["weightMax"], swimRule=c.get("swimRule", 0))


WORKED_EXAMPLES = ("worked_example_4fish.json", "worked_example_division.json",
                   "worked_example_greedy.json", "worked_example_weighted.json")


def pin_worked_examples(O):
    for name in WORKED_EXAMPLES:
        fx = load_golden(name)
        cfg = golden_config(fx)
        school = golden_school(fx, "before")
        d = np.array(fx["displacement"], np.float32)
        m, s, _ = O.step_displaced(cfg, school, d[:, 0], d[:, 1])
        want = golden_school(fx, "after")
        for k in FIELDS:
            assert np.array_equal(school[k], want[k]), f"{name}: {k} {school[k]} != {want[k]}"
        assert m == f32(fx["maxDiff"]), f"{name}: maxDiff {m}"
        assert list(s) == fx["sums"], f"{name}: sums {s}"
        assert [s[1] / s[0], s[2] / s[0]] == fx["barycentre"], f"{name}: barycentre"
    # The binary64 variant on the exact example gives the same exact values.
    fx = load_golden("worked_example_4fish.json")
    cfg = golden_config(fx)
    school = golden_school(fx, "before").astype(FISH_F64)
    d = np.array(fx["displacement"], np.float64)
    m, s = O.step_displaced_f64(cfg, school, d[:, 0], d[:, 1])
    want = golden_school(fx, "after")
    for k in FIELDS:
        assert np.array_equal(school[k], want[k].astype(np.float64)), f"f64 {k}"
    assert m == fx["maxDiff"] and list(s) == fx["sums"]


def pin_zero_swim(O):
    """S = 0: nobody moves, every diff is 0, maxDiff = 0, weights stay."""
    cfg = Config(numFish=1001, seed=3, swimStep=0.0)
    school = O.init(cfg)
    before = school.copy()
    for t in range(4):
        m, s, a = O.step(cfg, school, t)
        assert m == 0.0, f"maxDiff {m} with zero swim"
        for k in FIELDS:
            assert np.array_equal(school[k], before[k]), f"zero swim changed {k}"
        assert np.isfinite(s).all()
    f64 = O.init_f64(cfg)
    w0 = f64["weight"].copy()
    m, s = O.step_f64(cfg, f64, 0)
    assert m == 0.0 and np.array_equal(f64["weight"], w0)


def pin_uniform_weights_mean(O):
    """All weights pinned to one value: the barycentre is the plain mean of
    the positions (numpy's pairwise mean as the reference)."""
    c = 1.5
    cfg = Config(numFish=4097, seed=11, initWeightLo=c, initWeightHi=c,
                 weightMin=c, weightMax=c)
    school = O.init(cfg)
    for t in range(3):
        m, s, a = O.step(cfg, school, t)
        assert (school["weight"] == f32(c)).all()
        assert s[0] == c * cfg.numFish
        x = school["x"].astype(np.float64)
        y = school["y"].astype(np.float64)
        assert abs(s[1] / s[0] - x.mean()) <= 1e-13 * np.abs(x).mean()
        assert abs(s[2] / s[0] - y.mean()) <= 1e-13 * np.abs(y).mean()


def symmetric_dyadic_school(n_pairs: int, seed: int) -> np.ndarray:
    """Fish in mirror pairs (p, -p) with equal weights, on a dyadic grid so
    every product and every partial sum is exact: sum w*x = sum w*y = 0."""
    rng = np.random.default_rng(seed)
    x = rng.integers(-200, 201, n_pairs) / 2.0
    y = rng.integers(-200, 201, n_pairs) / 2.0
    w = rng.integers(4, 16, n_pairs) / 4.0
    xs = np.concatenate([x, -x])
    ys = np.concatenate([y, -y])
    ws = np.concatenate([w, w])
    perm = rng.permutation(2 * n_pairs)
    school = np.zeros(2 * n_pairs, FISH)
    school["x"], school["y"], school["weight"] = xs[perm], ys[perm], ws[perm]
    cur = np.sqrt(school["x"] * school["x"] + school["y"] * school["y"])
    school["currentObjective"] = cur
    school["prevObjective"] = cur
    return school


def pin_symmetric_school_exact(O):
    school = symmetric_dyadic_school(2048, 5)
    cfg = Config(numFish=school.size, swimStep=0.0)
    exact_w = math.fsum(school["weight"].astype(np.float64))
    m, s, a = O.step(cfg, school, 0)
    assert m == 0.0
    assert s[1] == 0.0 and s[2] == 0.0, f"symmetric sums {s}"
    assert s[0] == exact_w


# --------------------------------------------------------------------------
# Draw streams (init and swim) against ATen's words
# --------------------------------------------------------------------------

def _v_from_word(w):
    return (np.asarray(w, np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0**-23 - 1.0


def pin_init_stream(O):
    """Initial positions come from the init domain's sub-stream 0, weights
    from sub-stream 1; the objective is the distance from the centre."""
    cfg = Config(numFish=513, seed=987654321987)
    school = O.init(cfg)
    i = np.arange(cfg.numFish)
    j = 2 * (i & 1)
    wp = aten_words([cfg.seed] * cfg.numFish, [0 | (DOMAIN_INIT << 32)] * cfg.numFish, i >> 1)
    ww = aten_words([cfg.seed] * cfg.numFish, [1 | (DOMAIN_INIT << 32)] * cfg.numFish, i >> 1)
    H = f32(cfg.pondHalf)
    assert np.array_equal(school["x"], H * _v_from_word(wp[i, j]).astype(np.float32))
    assert np.array_equal(school["y"], H * _v_from_word(wp[i, j + 1]).astype(np.float32))
    u = ((ww[i, j] >> 8).astype(np.float64) * 2.0**-24).astype(np.float32)
    lo, hi = f32(cfg.initWeightLo), f32(cfg.initWeightHi)
    assert np.array_equal(school["weight"], lo + (hi - lo) * u)
    cur = np.sqrt(school["x"] * school["x"] + school["y"] * school["y"])
    assert np.array_equal(school["currentObjective"], cur)
    assert np.array_equal(school["prevObjective"], cur)
    assert (np.abs(school["x"]) <= H).all() and (school["weight"] >= lo).all()
    assert (school["weight"] <= hi).all()


def pin_swim_stream(O):
    """The displacement of fish i at iteration t is S*v of the words of
    counter (i>>1, t, swim domain)."""
    cfg = Config(numFish=257, seed=12345)
    school = O.init(cfg)
    O.run(cfg, school, 0, 3, with_sums=False)
    before = school.copy()
    t = 3
    O.step(cfg, school, t)
    i = np.arange(cfg.numFish)
    j = 2 * (i & 1)
    w = aten_words([cfg.seed] * cfg.numFish, [t | (DOMAIN_SWIM << 32)] * cfg.numFish, i >> 1)
    S = f32(cfg.swimStep)
    dx = S * _v_from_word(w[i, j]).astype(np.float32)
    dy = S * _v_from_word(w[i, j + 1]).astype(np.float32)
    inside = (np.abs(before["x"]) < 99) & (np.abs(before["y"]) < 99)
    assert inside.sum() > 200
    assert np.array_equal(school["x"][inside], (before["x"] + dx)[inside])
    assert np.array_equal(school["y"][inside], (before["y"] + dy)[inside])


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------

def check_step_invariants(cfg: Config, before: np.ndarray, after: np.ndarray,
                          m, s, a) -> None:
    H = f32(cfg.pondHalf)
    for k in FIELDS:
        v = after[k]
        assert np.isfinite(v).all(), f"non-finite {k}"
        assert not np.signbit(v[v == 0]).any(), f"-0 in {k}"
    assert (np.abs(after["x"]) <= H).all() and (np.abs(after["y"]) <= H).all()
    w = after["weight"]
    assert (w >= f32(cfg.weightMin)).all() and (w <= f32(cfg.weightMax)).all()
    cur = np.sqrt(after["x"] * after["x"] + after["y"] * after["y"])
    assert np.array_equal(after["currentObjective"], cur), "objective not distance"
    assert np.array_equal(after["prevObjective"], before["currentObjective"])
    diff = after["prevObjective"] - after["currentObjective"]
    assert m == np.abs(diff).max(), "maxDiff is not the max |diff| of the state"
    # triangle inequality: |diff| <= |displacement| <= S*sqrt(2), plus the
    # rounding of the two objectives (each within half an ulp of <= H*sqrt 2)
    ulp = float(np.spacing(f32(cfg.pondHalf * 1.5)))
    assert m <= cfg.swimStep * math.sqrt(2) * (1 + 1e-6) + 2 * ulp
    dw = after["weight"].astype(np.float64) - before["weight"].astype(np.float64)
    if m == 0:
        assert (dw == 0).all()
    else:
        wmin, wmax = f32(cfg.weightMin), f32(cfg.weightMax)
        at_bound = (w == wmin) | (w == wmax)
        assert (np.abs(dw) <= 1 + 4 * 2.0**-22).all(), "weight moved by more than 1"
        pos = diff > 0
        neg = diff < 0
        assert ((dw[pos] > 0) | at_bound[pos]).all(), "weight fell on positive diff"
        assert ((dw[neg] < 0) | at_bound[neg]).all(), "weight rose on negative diff"
        assert (dw[diff == 0] == 0).all()
    assert s[0] >= cfg.numFish * cfg.weightMin * (1 - 1e-12)
    assert a[0] == s[0] and abs(s[1]) <= a[1] and abs(s[2]) <= a[2]
    xs = after["x"].astype(np.float64)
    ys = after["y"].astype(np.float64)
    ws = after["weight"].astype(np.float64)
    for got, terms in ((s[0], ws), (s[1], ws * xs), (s[2], ws * ys)):
        ref = math.fsum(terms)
        assert abs(got - ref) <= 2.0**-51 * abs(ref) + 1e-25 * np.abs(terms).sum()


def pin_invariants(O):
    for cfg in (Config(numFish=1000, seed=1),
                Config(numFish=333, seed=2**64 - 5, swimStep=3.0),
                Config(numFish=64, seed=9, pondHalf=1.0, swimStep=0.5,
                       weightMin=0.5, weightMax=2.5),
                Config(numFish=1, seed=4)):
        school = O.init(cfg)
        for t in range(6):
            before = school.copy()
            m, s, a = O.step(cfg, school, t)
            check_step_invariants(cfg, before, school, m, s, a)


def pin_exact_sums(O):
    """Reference sums agree with math.fsum (the exact sum, correctly
    rounded) on ill-conditioned data with heavy cancellation."""
    rng = np.random.default_rng(3)
    n = 20000
    school = np.zeros(n, FISH)
    mag = 10.0 ** rng.uniform(-30, 2, n)
    school["x"] = (mag * rng.choice([-1, 1], n)).astype(np.float32)
    school["y"] = np.concatenate([np.full(n // 2, 1e2), np.full(n - n // 2, -1e2)])
    school["y"][:5] = [1e-7, 3e-9, -2e-8, 5e-30, 7e-12]
    school["weight"] = (10.0 ** rng.uniform(-3, 3, n)).astype(np.float32)
    s, a = O.barycentre_sums(school)
    w = school["weight"].astype(np.float64)
    for got, terms in ((s[0], w), (s[1], w * school["x"]), (s[2], w * school["y"])):
        ref = math.fsum(terms)
        assert abs(got - ref) <= 2.0**-51 * abs(ref) + 1e-25 * np.abs(terms).sum(), (
            f"{got} vs fsum {ref}")
    assert a[1] == math.fsum(np.abs(w * school["x"]))


def pin_composition(O):
    """Iterations are indexed globally: 3 then 4 iterations equal 7; one
    fish followed alone equals the school's fish."""
    cfg = Config(numFish=777, seed=5)
    a = O.init(cfg)
    b = a.copy()
    m1, s1, _ = O.run(cfg, a, 0, 3)
    m2, s2, _ = O.run(cfg, a, 3, 4)
    m, s, _ = O.run(cfg, b, 0, 7)
    assert np.array_equal(np.concatenate([m1, m2]), m)
    assert np.array_equal(np.concatenate([s1, s2]), s)
    assert a.tobytes() == b.tobytes()
    start = O.init(cfg)
    for i in (0, 1, 2, 391, 776):
        f = O.follow_fish(cfg, i, 0, 7, start[i])
        for k in ("x", "y", "prevObjective", "currentObjective"):
            assert f[k] == a[i][k], f"follow_fish {i} {k}"


def pin_swim_rules(O):
    """The greedy and weighted swim rules on random schools: the step
    invariants hold under every rule; greedy diffs are never negative and a
    fish moves exactly when its objective drops; greedy swimming still does
    not depend on weights (one fish followed alone equals the school's); and
    with every weight pinned at weightMin the weighted rule's mobility is
    exactly 1, so the school evolves bit for bit as under the plain rule."""
    for rule in (SWIM_GREEDY, SWIM_WEIGHTED, SWIM_GREEDY | SWIM_WEIGHTED):
        cfg = Config(numFish=2000, seed=17, swimStep=2.0, swimRule=rule)
        school = O.init(cfg)
        start = school.copy()
        for t in range(6):
            before = school.copy()
            m, s, a = O.step(cfg, school, t)
            check_step_invariants(cfg, before, school, m, s, a)
            if rule & SWIM_GREEDY:
                diff = school["prevObjective"] - school["currentObjective"]
                assert (diff >= 0).all(), "greedy diff < 0"
                moved = (school["x"] != before["x"]) | (school["y"] != before["y"])
                assert np.array_equal(moved, diff > 0), "greedy moved without improving"
        if rule == SWIM_GREEDY:
            for i in (0, 1, 1000, 1999):
                f = O.follow_fish(cfg, i, 0, 6, start[i])
                for k in ("x", "y", "prevObjective", "currentObjective"):
                    assert f[k] == school[i][k], f"greedy follow_fish {i} {k}"
        else:
            try:
                O.follow_fish(cfg, 0, 0, 1, start[0])
            except ValueError:
                pass
            else:
                raise AssertionError("follow_fish accepted the weighted rule")
    fixed = dict(numFish=999, seed=23, initWeightLo=1.0, initWeightHi=1.0, weightMin=1.0,
                 weightMax=1.0, swimStep=0.7)
    a = O.init(Config(**fixed))
    b = a.copy()
    O.run(Config(**fixed), a, 0, 5)
    O.run(Config(**fixed, swimRule=SWIM_WEIGHTED), b, 0, 5)
    assert a.tobytes() == b.tobytes(), "weighted rule with mobility 1 differs from the plain swim"


# --------------------------------------------------------------------------
# binary64 drift variant
# --------------------------------------------------------------------------

def pin_init_f64(O):
    """The binary64 initial state rounds to the binary32 one, bit for bit.

    x = H * v(a): v(a) = (k - 2^23) 2^-23 has at most 24 significant bits and
    so has H, so the product is exact in binary64 and binary32 rounds it
    once: float32(x_f64) is the binary32 product.  The weight lo + (hi - lo)
    u(a) is exact in binary64; in binary32 only its last addition rounds when
    hi - lo and (hi - lo) u are exact there (hi - lo a power of two), so the
    two agree after rounding.  The objective is the Euclidean distance
    (Sec. 2.1.1): within four binary64 ulps of math.hypot (the binary64
    square root of a sum of rounded squares is within two, hypot within one).  The binary32 init
    is itself pinned to ATen's words, so a wrong sub-stream, word or sign in
    the binary64 init fails here."""
    for cfg in (Config(numFish=1001, seed=987654321987),
                Config(numFish=64, seed=3, pondHalf=1.0, initWeightLo=0.5, initWeightHi=4.5)):
        s32 = O.init(cfg)
        s64 = O.init_f64(cfg)
        for k in ("x", "y", "weight"):
            assert np.array_equal(s64[k].astype(np.float32), s32[k]), f"init_f64 {k}"
        hyp = np.array([math.hypot(x, y) for x, y in zip(s64["x"], s64["y"])])
        assert (np.abs(s64["currentObjective"] - hyp) <= 4 * np.spacing(hyp)).all(), (
            "init_f64 objective is not the distance from the centre")
        assert np.array_equal(s64["prevObjective"], s64["currentObjective"])


def pin_step_f64_drawn(O):
    """Drawn binary64 iterations take the documented words and stay within the
    binary32 trajectory's rounding bound.

    One iteration from the binary64 initial state moves each fish away from
    the walls by S * v of ATen's words for counter (i >> 1, t, swim domain),
    added in binary64 (S * v is exact there: two 24-bit factors).  Over k
    iterations, every binary32 position differs from the binary64 one by at
    most k (ulp32(H) / 2 + ulp32(S) / 2): each binary32 iteration rounds the
    displacement and the addition once, clamping is 1-Lipschitz and the
    binary64 roundings are far smaller (the initial positions already differ
    by up to ulp32(H) / 2).  A wrong word, sign or iteration
    index in the binary64 draw moves a fish by O(S) and fails both checks."""
    cfg = Config(numFish=257, seed=12345)
    s64 = O.init_f64(cfg)
    s32 = O.init(cfg)
    t = 0
    before = s64.copy()
    m, _ = O.step_f64(cfg, s64, t)
    O.step(cfg, s32, t)
    i = np.arange(cfg.numFish)
    j = 2 * (i & 1)
    w = aten_words([cfg.seed] * cfg.numFish, [t | (DOMAIN_SWIM << 32)] * cfg.numFish, i >> 1)
    S = float(f32(cfg.swimStep))
    dx = S * _v_from_word(w[i, j])
    dy = S * _v_from_word(w[i, j + 1])
    inside = (np.abs(before["x"]) < 99) & (np.abs(before["y"]) < 99)
    assert inside.sum() > 200
    assert np.array_equal(s64["x"][inside], (before["x"] + dx)[inside])
    assert np.array_equal(s64["y"][inside], (before["y"] + dy)[inside])
    assert 0 < m <= S * math.sqrt(2) * (1 + 1e-15)
    diff = s64["prevObjective"] - s64["currentObjective"]
    assert m == np.abs(diff).max()
    k_max = 12
    per = float(np.spacing(f32(cfg.pondHalf))) / 2 + float(np.spacing(f32(S))) / 2
    for k in range(1, k_max):
        O.step_f64(cfg, s64, k)
        O.step(cfg, s32, k)
        bound = ((k + 1) * per + float(np.spacing(f32(cfg.pondHalf))) / 2) * (1 + 1e-6)
        for f in ("x", "y"):
            d = np.abs(s32[f].astype(np.float64) - s64[f]).max()
            assert d <= bound, f"binary64 {f} drifted {d:.3e} > {bound:.3e} after {k + 1} iterations"


def pin_f64_invariants(O):
    """The binary64 iteration keeps the method's invariants: positions in the
    pond, weights within the limits, the objective is the distance (math.hypot
    within four ulps), maxDiff is the attained max |diff|, the weight change
    follows the sign of diff unless a limit stops it, and the sums equal
    math.fsum of the binary64 terms."""
    cfg = Config(numFish=999, seed=77, swimStep=1.5)
    s = O.init_f64(cfg)
    for t in range(5):
        before = s.copy()
        m, sums = O.step_f64(cfg, s, t)
        H = cfg.pondHalf
        assert (np.abs(s["x"]) <= H).all() and (np.abs(s["y"]) <= H).all()
        w = s["weight"]
        assert (w >= cfg.weightMin).all() and (w <= cfg.weightMax).all()
        hyp = np.array([math.hypot(x, y) for x, y in zip(s["x"], s["y"])])
        assert (np.abs(s["currentObjective"] - hyp) <= 4 * np.spacing(hyp)).all()
        assert np.array_equal(s["prevObjective"], before["currentObjective"])
        diff = s["prevObjective"] - s["currentObjective"]
        assert m == np.abs(diff).max() and m > 0
        dw = w - before["weight"]
        at_bound = (w == cfg.weightMin) | (w == cfg.weightMax)
        assert ((dw > 0) | at_bound)[diff > 0].all() and ((dw < 0) | at_bound)[diff < 0].all()
        assert (np.abs(dw) <= 1 + 1e-12).all()
        for got, terms in ((sums[0], w), (sums[1], w * s["x"]), (sums[2], w * s["y"])):
            ref = math.fsum(terms)
            assert abs(got - ref) <= 1e-14 * np.abs(terms).sum(), f"f64 sums {got} vs {ref}"


def pin_follow_fish_fed(O):
    """One fish followed alone with the school's recorded maxima (eat(),
    Sec. 2.3.2: a weight depends on the rest of the school only through the
    maximum) ends with the record the whole school's run gives it, every
    field, for every fish of a school, with the weight limits reached and
    the zero-swim iteration (M = 0, weights kept) among them."""
    for cfg, steps in ((Config(numFish=257, seed=31, weightMin=1.0, weightMax=1.3), 40),
                       (Config(numFish=64, seed=5, swimStep=0.0), 3),
                       (Config(numFish=129, seed=8, swimRule=1), 25)):
        school = O.init(cfg)
        start = school.copy()
        m, _, _ = O.run(cfg, school, 0, steps)
        for i in range(cfg.numFish):
            f = O.follow_fish_fed(cfg, i, 0, steps, start[i], m)
            for k in school.dtype.names:
                assert np.float32(f[k]).view(np.uint32) == np.float32(school[i][k]).view(np.uint32), \
                    f"fish {i} {k} of {cfg}"


ALL_PINS = (pin_philox_matches_aten, pin_fish_word_layout, pin_unit_map_exhaustive,
            pin_philox_statistics, pin_worked_examples, pin_zero_swim,
            pin_uniform_weights_mean, pin_symmetric_school_exact, pin_init_stream,
            pin_swim_stream, pin_invariants, pin_exact_sums, pin_composition, pin_swim_rules,
            pin_init_f64, pin_step_f64_drawn, pin_f64_invariants, pin_follow_fish_fed)


def run_all(O) -> list[str]:
    """Names (and messages) of the pins the given oracle fails."""
    failed = []
    for pin in ALL_PINS:
        try:
            pin(O)
        except AtenUnavailable:
            raise
        except Exception as e:  # any error counts as a failed pin
            failed.append(f"{pin.__name__}: {type(e).__name__}: {e}")
    return failed
