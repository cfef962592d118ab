"""Plant plausible mistakes in a copy of the oracle source (on the CPU) and
check that the pins in oracle_pins.py catch every one of them.  A pin suite
that a dropped term, a wrong sign or a wrong index slips through would not
be a pin."""
import os
import shutil
import tempfile

import pytest

import oracle_pins
from oracle import oracle as orc

# (name, text in fsb_oracle.c, replacement)
MUTANTS = [
    ("philox_multiplier", "#define PHILOX_MULT_0 0xD2511F53u", "#define PHILOX_MULT_0 0xD2511F55u"),
    ("philox_no_key_schedule", "        k0 += PHILOX_WEYL_0;\n", ""),
    ("philox_word_swap", "        uint32_t n1 = (uint32_t)p1;", "        uint32_t n1 = (uint32_t)p0;"),
    ("counter_uses_fish_not_pair", "uint64_t pair = fish >> 1;", "uint64_t pair = fish;"),
    ("word_pick_stride", "unsigned first = 2u * (unsigned)(fish & 1u);",
     "unsigned first = (unsigned)(fish & 1u);"),
    ("unit_drops_bit", "return (float)(r >> 8) * 0x1p-24f;", "return (float)(r >> 9) * 0x1p-23f;"),
    ("signed_unit_halved", "return 2.0f * u - 1.0f;", "return u - 0.5f;"),
    ("swim_step_off_by_one", "(uint32_t)t, ORACLE_DOMAIN_SWIM, &a, &b);\n    float dx",
     "(uint32_t)(t + 1), ORACLE_DOMAIN_SWIM, &a, &b);\n    float dx"),
    ("swim_in_init_domain", "(uint32_t)t, ORACLE_DOMAIN_SWIM, &a, &b);\n    float dx",
     "(uint32_t)t, ORACLE_DOMAIN_INIT, &a, &b);\n    float dx"),
    ("no_pond_clamp", "float x = clampf(f->x + dx, -H, H);", "float x = f->x + dx;"),
    ("objective_wrong_term", "return sqrtf(x * x + y * y);", "return sqrtf(x * x + y * x);"),
    ("prev_not_kept", "    float c = objective(x, y);\n    f->prevObjective = f->currentObjective;\n",
     "    float c = objective(x, y);\n"),
    ("greedy_accepts_ties", "    float c = objective(x, y);\n    f->prevObjective = f->currentObjective;\n"
     "    if (!(cfg->swimRule & ORACLE_SWIM_GREEDY) || c < f->currentObjective) {",
     "    float c = objective(x, y);\n    f->prevObjective = f->currentObjective;\n"
     "    if (!(cfg->swimRule & ORACLE_SWIM_GREEDY) || c <= f->currentObjective) {"),
    ("greedy_ignored", "    float c = objective(x, y);\n    f->prevObjective = f->currentObjective;\n"
     "    if (!(cfg->swimRule & ORACLE_SWIM_GREEDY) || c < f->currentObjective) {",
     "    float c = objective(x, y);\n    f->prevObjective = f->currentObjective;\n"
     "    if (1) {"),
    ("greedy_prev_only_on_accept", "    float c = objective(x, y);\n    f->prevObjective = f->currentObjective;\n"
     "    if (!(cfg->swimRule & ORACLE_SWIM_GREEDY) || c < f->currentObjective) {\n",
     "    float c = objective(x, y);\n"
     "    if (!(cfg->swimRule & ORACLE_SWIM_GREEDY) || c < f->currentObjective) {\n"
     "        f->prevObjective = f->currentObjective;\n"),
    ("weighted_inverted", "float mobility = cfg->weightMin / f->weight;",
     "float mobility = f->weight / cfg->weightMin;"),
    ("weighted_ignored", "        dx = dx * mobility;\n        dy = dy * mobility;\n    }\n    float x",
     "    }\n    float x"),
    ("weighted_one_axis", "        dy = dy * mobility;\n    }\n    float x", "    }\n    float x"),
    ("signed_max", "float mag = fabsf(diff);", "float mag = diff;"),
    ("no_zero_guard", "if (maxDiff > 0.0f) {", "{"),
    ("feed_sign_flip", "float diff = f->prevObjective - f->currentObjective;\n    f->weight = clampf(",
     "float diff = f->currentObjective - f->prevObjective;\n    f->weight = clampf("),
    ("feed_not_normalised", "f->weight + diff / maxDiff", "f->weight + diff"),
    ("no_weight_clamp", "f->weight = clampf(f->weight + diff / maxDiff, cfg->weightMin, cfg->weightMax);",
     "f->weight = f->weight + diff / maxDiff;"),
    ("sums_before_feeding", "    float m = eat(cfg, school);\n    if (maxDiff)\n        *maxDiff = m;\n    if (sums || absSums)\n        oracle_barycentre_sums(school, cfg->numFish, sums, absSums);",
     "    if (sums || absSums)\n        oracle_barycentre_sums(school, cfg->numFish, sums, absSums);\n    float m = eat(cfg, school);\n    if (maxDiff)\n        *maxDiff = m;"),
    ("sum_drops_compensation", "sums[1] = sx.sum + sx.comp;\n        sums[2] = sy.sum + sy.comp;\n    }\n    if (absSums)",
     "sums[1] = sx.sum;\n        sums[2] = sy.sum + sy.comp;\n    }\n    if (absSums)"),
    ("sum_wy_uses_x", "double wy = w * (double)school[i].y;", "double wy = w * (double)school[i].x;"),
    ("init_weight_range", "f->weight = lo + (hi - lo) * oracle_unit(a);", "f->weight = lo + hi * oracle_unit(a);"),
    ("init_weight_same_words", "oracle_fish_words(cfg->seed, i, 1u, ORACLE_DOMAIN_INIT, &a, &b);\n        f->weight = lo + (hi - lo) * oracle_unit(a);",
     "oracle_fish_words(cfg->seed, i, 0u, ORACLE_DOMAIN_INIT, &a, &b);\n        f->weight = lo + (hi - lo) * oracle_unit(a);"),
    ("init_prev_zero", "        f->prevObjective = f->currentObjective;\n    }\n}\n\n/* Move",
     "        f->prevObjective = 0.0f;\n    }\n}\n\n/* Move"),
    # one fish followed with the school's maxima
    ("fed_follow_wrong_max", "feed_fish(cfg, f, maxDiff[t - t0]);", "feed_fish(cfg, f, maxDiff[t1 - 1 - t]);"),
    ("fed_follow_feeds_before_swim", "        swim_drawn(cfg, f, fish, t);\n        if (maxDiff[t - t0] > 0.0f)\n            feed_fish(cfg, f, maxDiff[t - t0]);",
     "        if (maxDiff[t - t0] > 0.0f)\n            feed_fish(cfg, f, maxDiff[t - t0]);\n        swim_drawn(cfg, f, fish, t);"),
    # the binary64 drift variant
    ("init_f64_sign", "f->x = H * (2.0 * unit_f64(a) - 1.0);", "f->x = H * (1.0 - 2.0 * unit_f64(a));"),
    ("init_f64_same_word", "f->y = H * (2.0 * unit_f64(b) - 1.0);", "f->y = H * (2.0 * unit_f64(a) - 1.0);"),
    ("init_f64_weight_word", "f->weight = lo + (hi - lo) * unit_f64(a);",
     "f->weight = lo + (hi - lo) * unit_f64(b);"),
    ("init_f64_weight_substream",
     "oracle_fish_words(cfg->seed, i, 1u, ORACLE_DOMAIN_INIT, &a, &b);\n        f->weight = lo + (hi - lo) * unit_f64(a);",
     "oracle_fish_words(cfg->seed, i, 0u, ORACLE_DOMAIN_INIT, &a, &b);\n        f->weight = lo + (hi - lo) * unit_f64(a);"),
    ("init_f64_objective_term", "f->currentObjective = sqrt(f->x * f->x + f->y * f->y);",
     "f->currentObjective = sqrt(f->x * f->x + f->y * f->x);"),
    ("step_f64_off_by_one", "(uint32_t)t, ORACLE_DOMAIN_SWIM, &a, &b);\n        swim_fish_f64",
     "(uint32_t)(t + 1), ORACLE_DOMAIN_SWIM, &a, &b);\n        swim_fish_f64"),
    ("step_f64_words_swapped", "S * (2.0 * unit_f64(a) - 1.0),\n                      S * (2.0 * unit_f64(b) - 1.0));",
     "S * (2.0 * unit_f64(b) - 1.0),\n                      S * (2.0 * unit_f64(a) - 1.0));"),
    ("step_f64_sign", "S * (2.0 * unit_f64(a) - 1.0),\n", "S * (1.0 - 2.0 * unit_f64(a)),\n"),
    ("step_f64_no_clamp", "double x = clampd(f->x + dx, -H, H);", "double x = f->x + dx;"),
    ("f64_signed_max", "double mag = fabs(school[i].prevObjective - school[i].currentObjective);",
     "double mag = school[i].prevObjective - school[i].currentObjective;"),
    ("f64_feed_sign", "double diff = f->prevObjective - f->currentObjective;\n            f->weight = clampd",
     "double diff = f->currentObjective - f->prevObjective;\n            f->weight = clampd"),
    ("f64_sums_drop_weight", "neumaier_add(&sx, school[i].weight * school[i].x);",
     "neumaier_add(&sx, school[i].x);"),
]


@pytest.fixture(scope="module")
def source():
    with open(orc.SOURCE) as fh:
        return fh.read()


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mutants_")
    shutil.copy(os.path.join(orc.HERE, "fsb_oracle.h"), d)
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(source, workdir, name, old, new):
    assert source.count(old) == 1, f"mutation site for {name} not unique/found"
    src = os.path.join(workdir, f"{name}.c")
    with open(src, "w") as fh:
        fh.write(source.replace(old, new))
    lib = orc.build(src, os.path.join(workdir, f"lib{name}.so"))
    try:
        failed = oracle_pins.run_all(orc.Oracle(lib))
    except oracle_pins.AtenUnavailable as e:
        pytest.skip(f"ATen Philox header unavailable: {e}")
    assert failed, f"planted mistake '{name}' passed every pin"
