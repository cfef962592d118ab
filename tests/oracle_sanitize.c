/* oracle_sanitize.c -- drives every entry point of the CPU oracle
 * (oracle/fsb_oracle.c) on small schools, for a build with the address and
 * undefined-behaviour sanitizers: any out-of-bounds access, use of freed
 * memory, signed overflow or invalid shift in the oracle stops the program.
 * Checks a few results that hold whatever the draws (pond bound, weight
 * limits, composition) and prints "oracle checks ok". */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fsb_oracle.h"

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static Config config(uint64_t n, uint64_t seed, uint32_t rule)
{
    Config c;
    memset(&c, 0, sizeof(c));
    c.numFish = n;
    c.seed = seed;
    c.pondHalf = 100.0f;
    c.swimStep = 0.1f;
    c.initWeightLo = 1.0f;
    c.initWeightHi = 2.0f;
    c.weightMin = 1.0f;
    c.weightMax = 4.0f;
    c.swimRule = rule;
    return c;
}

static void school_case(uint64_t n, uint32_t rule)
{
    const uint64_t steps = 5;
    Config c = config(n, 0x9E3779B97F4A7C15ull + n, rule);
    Fish *a = malloc(n * sizeof(Fish)), *b = malloc(n * sizeof(Fish));
    FishD *d = malloc(n * sizeof(FishD));
    float *dx = malloc(n * sizeof(float)), *dy = malloc(n * sizeof(float));
    double *ddx = malloc(n * sizeof(double)), *ddy = malloc(n * sizeof(double));
    float m[5];
    double s[15], ab[15];
    oracle_init(&c, a);
    memcpy(b, a, n * sizeof(Fish));
    oracle_run(&c, a, 0, steps, m, s, ab);
    oracle_run(&c, b, 0, 2, NULL, NULL, NULL);
    oracle_run(&c, b, 2, steps - 2, NULL, NULL, NULL);
    CHECK(memcmp(a, b, n * sizeof(Fish)) == 0);
    for (uint64_t i = 0; i < n; ++i) {
        CHECK(fabsf(a[i].x) <= c.pondHalf && fabsf(a[i].y) <= c.pondHalf);
        CHECK(a[i].weight >= c.weightMin && a[i].weight <= c.weightMax);
        dx[i] = (float)(i % 7) * 0.25f - 0.75f;
        dy[i] = 0.5f - (float)(i % 5) * 0.25f;
        ddx[i] = dx[i];
        ddy[i] = dy[i];
    }
    float mm;
    double ss[3], aa[3];
    oracle_step_displaced(&c, a, dx, dy, &mm, ss, aa);
    CHECK(ss[0] >= (double)n * c.weightMin * (1 - 1e-12));
    oracle_barycentre_sums(a, n, ss, aa);
    CHECK(aa[0] == ss[0]);
    Fish f = b[n - 1];
    int rc = oracle_follow_fish(&c, n - 1, steps, steps + 3, &f);
    CHECK(rc == ((rule & ORACLE_SWIM_WEIGHTED) ? -1 : 0));
    /* the last fish followed alone from its start, fed with the run's maxima */
    Fish g;
    oracle_init(&c, b);
    g = b[n - 1];
    rc = oracle_follow_fish_fed(&c, n - 1, 0, steps, m, &g);
    CHECK(rc == ((rule & ORACLE_SWIM_WEIGHTED) ? -1 : 0));
    oracle_init_f64(&c, d);
    double md, sd[3];
    for (uint64_t t = 0; t < 3; ++t) oracle_step_f64(&c, d, t, &md, sd);
    oracle_step_displaced_f64(&c, d, ddx, ddy, &md, sd);
    for (uint64_t i = 0; i < n; ++i) CHECK(fabs(d[i].x) <= c.pondHalf);
    free(a);
    free(b);
    free(d);
    free(dx);
    free(dy);
    free(ddx);
    free(ddy);
}

int main(void)
{
    uint32_t counters[8] = {0, 0, 0, 0, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 1};
    uint32_t keys[4] = {0, 0, 0xFFFFFFFFu, 0xFFFFFFFFu}, out[8], w[4];
    oracle_philox_many(2, counters, keys, out);
    oracle_philox4x32_10(counters + 4, keys + 2, w);
    CHECK(memcmp(w, out + 4, sizeof(w)) == 0);
    uint32_t r[3] = {0, 0xFFu, 0xFFFFFFFFu};
    float u[3], v[3];
    oracle_unit_many(3, r, u, v);
    CHECK(u[0] == 0.0f && v[0] == -1.0f && u[2] < 1.0f && v[2] < 1.0f);
    uint32_t a, b;
    oracle_fish_words(~0ull, ~0ull, 0xFFFFFFFFu, ORACLE_DOMAIN_INIT, &a, &b);
    oracle_set_threads(2);
    CHECK(oracle_max_threads() >= 1);
    const uint64_t sizes[4] = {1, 2, 1001, 4099};
    const uint32_t rules[4] = {0, ORACLE_SWIM_GREEDY, ORACLE_SWIM_WEIGHTED,
                               ORACLE_SWIM_GREEDY | ORACLE_SWIM_WEIGHTED};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) school_case(sizes[i], rules[j]);
    if (failures) {
        fprintf(stderr, "%d oracle checks failed\n", failures);
        return 1;
    }
    printf("oracle checks ok\n");
    return 0;
}
