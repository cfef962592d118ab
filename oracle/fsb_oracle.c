/*
 * fsb_oracle.c -- plain CPU oracle of the Fish School Behaviour step.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the tests, the smoke check and
 * the benchmark's CPU-baseline leg use it.  Readings of the paper and the
 * floating-point contract are listed in fsb_oracle.h.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -fPIC -shared -lm.
 * Plain loops, one fish at a time; the only parallelism is OpenMP
 * "parallel for" over fish, with the max taken by reduction(max:) as in the
 * paper's Reduction Construct (Sec. 2.3.2, Experiment 3).
 */
#include "fsb_oracle.h"

#include <math.h>
#include <omp.h>

/* Philox4x32-10 constants from the SC'11 paper: the two round multipliers
 * and the two Weyl increments of the key schedule. */
#define PHILOX_MULT_0 0xD2511F53u
#define PHILOX_MULT_1 0xCD9E8D57u
#define PHILOX_WEYL_0 0x9E3779B9u
#define PHILOX_WEYL_1 0xBB67AE85u
#define PHILOX_ROUNDS 10

/* ------------------------------------------------------------------------ */
/* Random numbers                                                            */
/* ------------------------------------------------------------------------ */

/* Philox4x32: each round multiplies counter words 0 and 2 by the two
 * constants (full 64-bit products), then
 *   new0 = hi(M1*c2) ^ c1 ^ k0,  new1 = lo(M1*c2),
 *   new2 = hi(M0*c0) ^ c3 ^ k1,  new3 = lo(M0*c0),
 * and the key advances by the Weyl increments between rounds. */
void oracle_philox4x32_10(const uint32_t counter[4], const uint32_t key[2],
                          uint32_t out[4])
{
    uint32_t c0 = counter[0], c1 = counter[1], c2 = counter[2], c3 = counter[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < PHILOX_ROUNDS; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_MULT_0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_MULT_1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += PHILOX_WEYL_0;
        k1 += PHILOX_WEYL_1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void oracle_philox_many(uint64_t n, const uint32_t *counters,
                        const uint32_t *keys, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        oracle_philox4x32_10(counters + 4 * i, keys + 2 * i, out + 4 * i);
}

/* The top 24 bits of the word, as a multiple of 2^-24: exact in binary32. */
float oracle_unit(uint32_t r)
{
    return (float)(r >> 8) * 0x1p-24f;
}

/* 2u - 1: doubling is exact and so is the subtraction (both operands are
 * multiples of 2^-23 below 2 in magnitude). */
float oracle_signed_unit(uint32_t r)
{
    float u = oracle_unit(r);
    return 2.0f * u - 1.0f;
}

void oracle_unit_many(uint64_t n, const uint32_t *r, float *u, float *v)
{
    for (uint64_t i = 0; i < n; ++i) {
        u[i] = oracle_unit(r[i]);
        v[i] = oracle_signed_unit(r[i]);
    }
}

void oracle_fish_words(uint64_t seed, uint64_t fish, uint32_t sub,
                       uint32_t domain, uint32_t *a, uint32_t *b)
{
    uint64_t pair = fish >> 1;
    uint32_t counter[4] = {(uint32_t)pair, (uint32_t)(pair >> 32), sub, domain};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t words[4];
    oracle_philox4x32_10(counter, key, words);
    unsigned first = 2u * (unsigned)(fish & 1u);
    *a = words[first];
    *b = words[first + 1];
}

/* ------------------------------------------------------------------------ */
/* binary32 school                                                           */
/* ------------------------------------------------------------------------ */

static float clampf(float v, float lo, float hi)
{
    return fminf(fmaxf(v, lo), hi);
}

/* Euclidean distance from the pond centre (Sec. 2.1.1). */
static float objective(float x, float y)
{
    return sqrtf(x * x + y * y);
}

void oracle_init(const Config *cfg, Fish *school)
{
    const float H = cfg->pondHalf;
    const float lo = cfg->initWeightLo, hi = cfg->initWeightHi;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < cfg->numFish; ++i) {
        uint32_t a, b;
        Fish *f = &school[i];
        oracle_fish_words(cfg->seed, i, 0u, ORACLE_DOMAIN_INIT, &a, &b);
        f->x = H * oracle_signed_unit(a);
        f->y = H * oracle_signed_unit(b);
        oracle_fish_words(cfg->seed, i, 1u, ORACLE_DOMAIN_INIT, &a, &b);
        f->weight = lo + (hi - lo) * oracle_unit(a);
        f->currentObjective = objective(f->x, f->y);
        f->prevObjective = f->currentObjective;
    }
}

/* Move one fish by (dx, dy) inside the pond and re-evaluate its objective.
 * Weighted rule: the fish's weight affects its mobility (Sec. 2.1.1), read
 * as a step scaled by weightMin / weight.  Greedy rule: the movement is
 * influenced by the objective (Sec. 2.1.2), read as keeping a move only if
 * the new position is strictly closer to the pond centre. */
static void swim_fish(const Config *cfg, Fish *f, float dx, float dy)
{
    const float H = cfg->pondHalf;
    if (cfg->swimRule & ORACLE_SWIM_WEIGHTED) {
        float mobility = cfg->weightMin / f->weight;
        dx = dx * mobility;
        dy = dy * mobility;
    }
    float x = clampf(f->x + dx, -H, H);
    float y = clampf(f->y + dy, -H, H);
    float c = objective(x, y);
    f->prevObjective = f->currentObjective;
    if (!(cfg->swimRule & ORACLE_SWIM_GREEDY) || c < f->currentObjective) {
        f->x = x;
        f->y = y;
        f->currentObjective = c;
    }
}

static void swim_drawn(const Config *cfg, Fish *f, uint64_t fish, uint64_t t)
{
    uint32_t a, b;
    oracle_fish_words(cfg->seed, fish, (uint32_t)t, ORACLE_DOMAIN_SWIM, &a, &b);
    float dx = cfg->swimStep * oracle_signed_unit(a);
    float dy = cfg->swimStep * oracle_signed_unit(b);
    swim_fish(cfg, f, dx, dy);
}

/* One fish's weight update of eat(): its objective change over the school's
 * maximum, kept within the weight limits (maxDiff > 0). */
static void feed_fish(const Config *cfg, Fish *f, float maxDiff)
{
    float diff = f->prevObjective - f->currentObjective;
    f->weight = clampf(f->weight + diff / maxDiff, cfg->weightMin, cfg->weightMax);
}

/* eat(): the school-wide max of |prevObjective - currentObjective|, then the
 * weight update normalised by it. */
static float eat(const Config *cfg, Fish *school)
{
    const uint64_t n = cfg->numFish;
    float maxDiff = 0.0f;
#pragma omp parallel for schedule(static) reduction(max : maxDiff)
    for (uint64_t i = 0; i < n; ++i) {
        float diff = school[i].prevObjective - school[i].currentObjective;
        float mag = fabsf(diff);
        if (mag > maxDiff)
            maxDiff = mag;
    }
    if (maxDiff > 0.0f) {
#pragma omp parallel for schedule(static)
        for (uint64_t i = 0; i < n; ++i)
            feed_fish(cfg, &school[i], maxDiff);
    }
    return maxDiff;
}

/* Neumaier's compensated sum, one binary64 term at a time. */
typedef struct {
    double sum;
    double comp;
} Neumaier;

static void neumaier_add(Neumaier *acc, double v)
{
    double t = acc->sum + v;
    if (fabs(acc->sum) >= fabs(v))
        acc->comp += (acc->sum - t) + v;
    else
        acc->comp += (v - t) + acc->sum;
    acc->sum = t;
}

void oracle_barycentre_sums(const Fish *school, uint64_t n, double sums[3],
                            double absSums[3])
{
    Neumaier sw = {0, 0}, sx = {0, 0}, sy = {0, 0};
    Neumaier aw = {0, 0}, ax = {0, 0}, ay = {0, 0};
    for (uint64_t i = 0; i < n; ++i) {
        double w = (double)school[i].weight;
        double wx = w * (double)school[i].x; /* exact: 24 + 24 bits */
        double wy = w * (double)school[i].y;
        neumaier_add(&sw, w);
        neumaier_add(&sx, wx);
        neumaier_add(&sy, wy);
        neumaier_add(&aw, fabs(w));
        neumaier_add(&ax, fabs(wx));
        neumaier_add(&ay, fabs(wy));
    }
    if (sums) {
        sums[0] = sw.sum + sw.comp;
        sums[1] = sx.sum + sx.comp;
        sums[2] = sy.sum + sy.comp;
    }
    if (absSums) {
        absSums[0] = aw.sum + aw.comp;
        absSums[1] = ax.sum + ax.comp;
        absSums[2] = ay.sum + ay.comp;
    }
}

static void finish_step(const Config *cfg, Fish *school, float *maxDiff,
                        double sums[3], double absSums[3])
{
    float m = eat(cfg, school);
    if (maxDiff)
        *maxDiff = m;
    if (sums || absSums)
        oracle_barycentre_sums(school, cfg->numFish, sums, absSums);
}

void oracle_step(const Config *cfg, Fish *school, uint64_t t, float *maxDiff,
                 double sums[3], double absSums[3])
{
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < cfg->numFish; ++i)
        swim_drawn(cfg, &school[i], i, t);
    finish_step(cfg, school, maxDiff, sums, absSums);
}

void oracle_step_displaced(const Config *cfg, Fish *school, const float *dx,
                           const float *dy, float *maxDiff, double sums[3],
                           double absSums[3])
{
    for (uint64_t i = 0; i < cfg->numFish; ++i)
        swim_fish(cfg, &school[i], dx[i], dy[i]);
    finish_step(cfg, school, maxDiff, sums, absSums);
}

void oracle_run(const Config *cfg, Fish *school, uint64_t t0, uint64_t nSteps,
                float *maxDiff, double *sums, double *absSums)
{
    for (uint64_t k = 0; k < nSteps; ++k)
        oracle_step(cfg, school, t0 + k, maxDiff ? maxDiff + k : 0,
                    sums ? sums + 3 * k : 0, absSums ? absSums + 3 * k : 0);
}

int oracle_follow_fish(const Config *cfg, uint64_t fish, uint64_t t0,
                       uint64_t t1, Fish *f)
{
    if (cfg->swimRule & ORACLE_SWIM_WEIGHTED)
        return -1;
    for (uint64_t t = t0; t < t1; ++t)
        swim_drawn(cfg, f, fish, t);
    return 0;
}

int oracle_follow_fish_fed(const Config *cfg, uint64_t fish, uint64_t t0,
                           uint64_t t1, const float *maxDiff, Fish *f)
{
    if (cfg->swimRule & ORACLE_SWIM_WEIGHTED)
        return -1;
    for (uint64_t t = t0; t < t1; ++t) {
        swim_drawn(cfg, f, fish, t);
        if (maxDiff[t - t0] > 0.0f)
            feed_fish(cfg, f, maxDiff[t - t0]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* binary64 drift variant: the same integer draws and the same rules, with  */
/* every quantity held in binary64.  Information only.                       */
/* ------------------------------------------------------------------------ */

static double unit_f64(uint32_t r)
{
    return (double)(r >> 8) * 0x1p-24;
}

static double clampd(double v, double lo, double hi)
{
    return fmin(fmax(v, lo), hi);
}

void oracle_init_f64(const Config *cfg, FishD *school)
{
    const double H = cfg->pondHalf;
    const double lo = cfg->initWeightLo, hi = cfg->initWeightHi;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < cfg->numFish; ++i) {
        uint32_t a, b;
        FishD *f = &school[i];
        oracle_fish_words(cfg->seed, i, 0u, ORACLE_DOMAIN_INIT, &a, &b);
        f->x = H * (2.0 * unit_f64(a) - 1.0);
        f->y = H * (2.0 * unit_f64(b) - 1.0);
        oracle_fish_words(cfg->seed, i, 1u, ORACLE_DOMAIN_INIT, &a, &b);
        f->weight = lo + (hi - lo) * unit_f64(a);
        f->currentObjective = sqrt(f->x * f->x + f->y * f->y);
        f->prevObjective = f->currentObjective;
    }
}

static void swim_fish_f64(const Config *cfg, FishD *f, double dx, double dy)
{
    const double H = cfg->pondHalf;
    if (cfg->swimRule & ORACLE_SWIM_WEIGHTED) {
        double mobility = (double)cfg->weightMin / f->weight;
        dx = dx * mobility;
        dy = dy * mobility;
    }
    double x = clampd(f->x + dx, -H, H);
    double y = clampd(f->y + dy, -H, H);
    double c = sqrt(x * x + y * y);
    f->prevObjective = f->currentObjective;
    if (!(cfg->swimRule & ORACLE_SWIM_GREEDY) || c < f->currentObjective) {
        f->x = x;
        f->y = y;
        f->currentObjective = c;
    }
}

static void finish_step_f64(const Config *cfg, FishD *school, double *maxDiff,
                            double sums[3])
{
    const uint64_t n = cfg->numFish;
    double m = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        double mag = fabs(school[i].prevObjective - school[i].currentObjective);
        if (mag > m)
            m = mag;
    }
    if (m > 0.0) {
        for (uint64_t i = 0; i < n; ++i) {
            FishD *f = &school[i];
            double diff = f->prevObjective - f->currentObjective;
            f->weight = clampd(f->weight + diff / m, cfg->weightMin, cfg->weightMax);
        }
    }
    if (maxDiff)
        *maxDiff = m;
    if (sums) {
        Neumaier sw = {0, 0}, sx = {0, 0}, sy = {0, 0};
        for (uint64_t i = 0; i < n; ++i) {
            neumaier_add(&sw, school[i].weight);
            neumaier_add(&sx, school[i].weight * school[i].x);
            neumaier_add(&sy, school[i].weight * school[i].y);
        }
        sums[0] = sw.sum + sw.comp;
        sums[1] = sx.sum + sx.comp;
        sums[2] = sy.sum + sy.comp;
    }
}

void oracle_step_f64(const Config *cfg, FishD *school, uint64_t t,
                     double *maxDiff, double sums[3])
{
    const double S = cfg->swimStep;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < cfg->numFish; ++i) {
        uint32_t a, b;
        oracle_fish_words(cfg->seed, i, (uint32_t)t, ORACLE_DOMAIN_SWIM, &a, &b);
        swim_fish_f64(cfg, &school[i], S * (2.0 * unit_f64(a) - 1.0),
                      S * (2.0 * unit_f64(b) - 1.0));
    }
    finish_step_f64(cfg, school, maxDiff, sums);
}

void oracle_step_displaced_f64(const Config *cfg, FishD *school,
                               const double *dx, const double *dy,
                               double *maxDiff, double sums[3])
{
    for (uint64_t i = 0; i < cfg->numFish; ++i)
        swim_fish_f64(cfg, &school[i], dx[i], dy[i]);
    finish_step_f64(cfg, school, maxDiff, sums);
}

/* ------------------------------------------------------------------------ */

void oracle_set_threads(int n)
{
    if (n > 0)
        omp_set_num_threads(n);
}

int oracle_max_threads(void)
{
    return omp_get_max_threads();
}
