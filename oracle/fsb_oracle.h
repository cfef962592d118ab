/*
 * fsb_oracle.h -- plain CPU oracle of the Fish School Behaviour (FSB) step.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.  It
 * shares no code, header, table or constant with the GPU library: the two are
 * written separately from the same definitions, so that agreement between
 * them means something.
 *
 * What it computes, per the paper (arXiv 2507.20173):
 *   - the fish record {x, y, weight, prevObjective, currentObjective}
 *     (Sec. 2.1.1), held here as an array of structs like the paper's
 *     school[i];
 *   - the 200x200 pond (Sec. 2.1.2), centred at the origin: |x|,|y| <= H;
 *   - random initial position and weight, initial currentObjective equal to
 *     the Euclidean distance from the pond centre (Sec. 2.1.1);
 *   - a randomised swim (Sec. 2.1.2), then eat(): diff = prevObjective -
 *     currentObjective and its school-wide maximum (the Reduction Construct
 *     of Sec. 2.3.2, Experiment 3), which normalises the weight update;
 *   - the weighted barycentre sums of the school.
 * The paper leaves the swim rule, the feeding formula, the weight limits and
 * the random generator unstated; the readings taken here are:
 *   swim      d = S * v, v uniform on [-1,1) per axis, position clamped to
 *             [-H, H]; two optional rules read the paper's remarks that a
 *             fish's weight affects its mobility (Sec. 2.1.1) and that its
 *             movement is influenced by its weight and objective
 *             (Sec. 2.1.2):
 *               weighted: d is scaled by weightMin / weight, so heavier fish
 *                         take shorter steps;
 *               greedy:   the move is kept only if it brings the fish
 *                         strictly closer to the pond centre; otherwise the
 *                         fish stays where it was (its diff is then 0);
 *   normaliser maxDiff = max_i |diff_i| (a magnitude, so that feeding keeps
 *             its sign even when every fish moved away from the centre);
 *   feeding   if maxDiff > 0: weight = clamp(weight + diff / maxDiff,
 *             weightMin, weightMax); if maxDiff == 0 weights stay as they are;
 *   sums      over the same step's post-swim positions and post-feed weights;
 *   random    Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random
 *             Numbers: As Easy as 1, 2, 3", SC'11), key = 64-bit seed,
 *             counter = (pair lo, pair hi, step or init sub-stream, domain),
 *             pair = fish >> 1, fish i takes output words 2*(i&1) and
 *             2*(i&1)+1.
 * Floating point: IEEE binary32, round to nearest even, every operation
 * rounded on its own (built with -ffp-contract=off), correctly rounded sqrtf
 * and division, no flush to zero.
 */
#ifndef FSB_ORACLE_H
#define FSB_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One fish, as the paper's Fish structure (Sec. 2.1.1). */
typedef struct Fish {
    float x;
    float y;
    float weight;
    float prevObjective;
    float currentObjective;
} Fish;

/* The same record in binary64, for the drift variant. */
typedef struct FishD {
    double x;
    double y;
    double weight;
    double prevObjective;
    double currentObjective;
} FishD;

/* Simulation part of the paper's Config structure (Sec. 2.1.3). */
typedef struct Config {
    uint64_t numFish;
    uint64_t seed;
    float pondHalf;     /* H: the pond is [-H, H] x [-H, H] */
    float swimStep;     /* S: per-axis swim displacement lies in [-S, S) */
    float initWeightLo; /* initial weight drawn in [lo, hi] */
    float initWeightHi;
    float weightMin;    /* weight limits applied by feeding */
    float weightMax;
    uint32_t swimRule;  /* ORACLE_SWIM_* flags */
} Config;

/* Swim rules (flags; 0 = the plain random swim). */
#define ORACLE_SWIM_GREEDY 1u
#define ORACLE_SWIM_WEIGHTED 2u

/* Random-stream domains (the fourth counter word). */
#define ORACLE_DOMAIN_SWIM 0u
#define ORACLE_DOMAIN_INIT 1u

/* ---- random numbers ---------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t counter[4], const uint32_t key[2],
                          uint32_t out[4]);
/* n independent calls: counters[4*n], keys[2*n], out[4*n]. */
void oracle_philox_many(uint64_t n, const uint32_t *counters,
                        const uint32_t *keys, uint32_t *out);
/* u = (r >> 8) * 2^-24 in [0, 1), and v = 2u - 1 in [-1, 1). */
float oracle_unit(uint32_t r);
float oracle_signed_unit(uint32_t r);
void oracle_unit_many(uint64_t n, const uint32_t *r, float *u, float *v);
/* The two words fish `fish` draws from sub-stream `sub` of `domain`. */
void oracle_fish_words(uint64_t seed, uint64_t fish, uint32_t sub,
                       uint32_t domain, uint32_t *a, uint32_t *b);

/* ---- binary32 school (the parity authority) ---------------------------- */
void oracle_init(const Config *cfg, Fish *school);
/* One iteration t: swim, eat (max |diff| and feeding), barycentre sums.
 * maxDiff, sums[3] = {sum w, sum w*x, sum w*y} and absSums[3] = {sum |w|,
 * sum |w*x|, sum |w*y|} are written when non-null. */
void oracle_step(const Config *cfg, Fish *school, uint64_t t, float *maxDiff,
                 double sums[3], double absSums[3]);
/* The same iteration with the displacements given instead of drawn. */
void oracle_step_displaced(const Config *cfg, Fish *school, const float *dx,
                           const float *dy, float *maxDiff, double sums[3],
                           double absSums[3]);
/* Iterations t0 .. t0+nSteps-1.  Per-step maxDiff[nSteps], sums[3*nSteps]
 * and absSums[3*nSteps] are written when non-null. */
void oracle_run(const Config *cfg, Fish *school, uint64_t t0, uint64_t nSteps,
                float *maxDiff, double *sums, double *absSums);
/* Position and objectives of a single fish over iterations t0 .. t1-1.
 * Unless the weighted rule is on, swimming depends neither on weights nor on
 * other fish, so one fish can be followed on its own (under the weighted rule
 * this does nothing and returns -1; otherwise 0).  f holds the fish's state
 * at the start of t0. */
int oracle_follow_fish(const Config *cfg, uint64_t fish, uint64_t t0,
                       uint64_t t1, Fish *f);
/* The same fish with its weight fed as eat() feeds it (Sec. 2.3.2), given the
 * school's maximum of every iteration, maxDiff[t1 - t0] (from a run of the
 * whole school): a fish's weight depends on the rest of the school only
 * through those maxima.  Returns -1 under the weighted rule, else 0. */
int oracle_follow_fish_fed(const Config *cfg, uint64_t fish, uint64_t t0,
                           uint64_t t1, const float *maxDiff, Fish *f);
/* Exact-as-possible reference sums: each product of two binary32 values is
 * exact in binary64, summed with Neumaier's compensated summation. */
void oracle_barycentre_sums(const Fish *school, uint64_t n, double sums[3],
                            double absSums[3]);

/* ---- binary64 drift variant (same integer draws, information only) ----- */
void oracle_init_f64(const Config *cfg, FishD *school);
void oracle_step_f64(const Config *cfg, FishD *school, uint64_t t,
                     double *maxDiff, double sums[3]);
void oracle_step_displaced_f64(const Config *cfg, FishD *school,
                               const double *dx, const double *dy,
                               double *maxDiff, double sums[3]);

/* ---- threads ----------------------------------------------------------- */
void oracle_set_threads(int n);
int oracle_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
