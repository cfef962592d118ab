/*
 * fsb.h -- C ABI of libfsb, the MI355X (gfx950) Fish School Behaviour step.
 *
 * The method (arXiv 2507.20173, "High-Performance Parallel Optimization of
 * the Fish School Behaviour on the Setonix Platform Using OpenMP"):
 *   - each fish carries {x, y, weight, prevObjective, currentObjective}
 *     (Sec. 2.1.1); here they are five float32 structure-of-arrays columns
 *     x[], y[], w[], prev[], cur[];
 *   - the pond is 200x200 (Sec. 2.1.2), read as [-H, H]^2 centred at the
 *     origin, H = 100;
 *   - positions and weights start random; the objective is the Euclidean
 *     distance from the pond centre (Sec. 2.1.1);
 *   - every iteration each fish swims a random step and is re-evaluated
 *     (Sec. 2.1.2), then eat() takes diff = prevObjective - currentObjective
 *     and its school-wide maximum (the Reduction Construct, Sec. 2.3.2,
 *     Experiment 3), which normalises the weight update;
 *   - the school's weighted barycentre (sum w*x / sum w, sum w*y / sum w).
 * Readings where the paper is silent (swim rule, feeding formula, weight
 * limits, random generator):
 *   iteration t, fish i:
 *     (a, b)  = two words of Philox4x32-10 (Salmon et al., SC'11) with key =
 *               seed and counter = (pair lo, pair hi, t, 0), pair = i >> 1;
 *               fish i takes words 2(i&1) and 2(i&1)+1
 *     v(r)    = (r >> 8) * 2^-23 - 1, exact, in [-1, 1)
 *     x       = min(max(x + S*v(a), -H), H);  y likewise with v(b)
 *     prev    = cur;  cur = sqrtf(x*x + y*y)
 *     diff    = prev - cur;   M = max over the school of |diff|
 *     w       = min(max(w + diff / M, w_min), w_max)   if M > 0, else w kept
 *     sums    = (sum w, sum w*x, sum w*y) over the post-feed state
 *   every float operation is binary32 round-to-nearest-even, rounded on its
 *   own (no fused multiply-add), with correctly rounded sqrtf and division
 *   and no flush to zero: per-fish state is bit-exact and reproducible.
 *   Initial state: counter (pair, 0, 1) gives x = H*v(a), y = H*v(b);
 *   counter (pair, 1, 1) gives w = lo + (hi - lo) * u(a), u(r) = (r >> 8) *
 *   2^-24; cur = prev = sqrtf(x*x + y*y).
 *
 * Conventions for every entry point:
 *   - Device pointers are caller-owned (allocated by the caller, e.g. with
 *     PyTorch); the library never allocates, frees or retains device memory
 *     beyond the handle's lifetime.  Arrays are 16-byte aligned, hold at
 *     least n_fish floats and do not overlap.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All work is enqueued on it; calls are asynchronous unless documented
 *     as synchronising.
 *   - Every call returns FSB_OK (0) or a negative FSB_ERR_* code; arguments
 *     are checked on the host before anything is enqueued, so an invalid
 *     call has no effect.  fsb_last_error() returns a message for the last
 *     failure on the calling thread.  No C++ exception crosses the ABI.
 *   - A handle is used by one host thread at a time.
 */
#ifndef FSB_H
#define FSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSB_ABI_VERSION 2

/* Return codes. */
#define FSB_OK 0
#define FSB_ERR_INVALID_ARG (-1) /* bad pointer, size, alignment or value */
#define FSB_ERR_HIP (-2)         /* the HIP runtime reported an error      */
#define FSB_ERR_UNSUPPORTED (-3) /* e.g. persistent grid cannot be resident */
#define FSB_ERR_STATE (-4)       /* call not valid in the handle's state   */
#define FSB_ERR_DEVICE (-5)      /* a kernel reported a failure (barrier timeout) */

/* fsb_config.reduce_mode: how the school max and the barycentre sums are
 * reduced.  The max is exact in every mode (it does not depend on order). */
#define FSB_REDUCE_COMPENSATED 0u /* per-lane compensated (TwoSum) float32 over pairwise sums
                                     of four fish, binary64 cross-block combine, fixed order */
#define FSB_REDUCE_NAIVE_F32 1u   /* float32 block trees + float32 atomicAdd (accuracy baseline) */
#define FSB_REDUCE_CRITICAL_F32 2u /* no tree: every fish updates one shared max word and three
                                      shared float32 sums with its own device-scope atomic, the GPU
                                      counterpart of the critical-section construct of Sec. 2.3.2
                                      (Experiment 3).  An ablation baseline: plain iterations only
                                      (fsb_step, fsb_step_displaced, FSB_RUN_PLAIN); the persistent
                                      modes and batches return FSB_ERR_UNSUPPORTED.  The sums are
                                      not deterministic (atomic order). */

/* fsb_config.swim_rule: flags; 0 is the plain random swim.  Readings of the
 * paper's remarks that a fish's weight affects its mobility (Sec. 2.1.1) and
 * that its movement is influenced by its weight and objective (Sec. 2.1.2). */
#define FSB_SWIM_GREEDY 1u   /* a move is kept only if the objective strictly decreases;
                                otherwise the fish stays and its diff is 0 */
#define FSB_SWIM_WEIGHTED 2u /* the displacement is scaled by w_min / w, w being the weight
                                the fish has when it swims; needs w_min > 0 and
                                w_init_lo > 0 */

/* fsb_run modes. */
#define FSB_RUN_PLAIN 0u      /* one launch per iteration: for n_steps >= 2 the swim
                                 pass of the first iteration, then one pipelined pass per
                                 further iteration t that feeds t - 1 and swims t (x, y,
                                 w, prev read and written once: 32 B per fish-iteration,
                                 cur left unwritten), then the feed pass of the last
                                 iteration, which also writes cur.  n_steps = 1 and
                                 FSB_REDUCE_CRITICAL_F32 take FSB_RUN_PLAIN_SPLIT */
#define FSB_RUN_FUSED 1u      /* one persistent launch; the library picks a variant below:
                                 deep whenever it can run, else registers for a school
                                 they hold, else store-prev or lean by footprint */
#define FSB_RUN_FUSED_PREV 2u /* persistent, x, y, w, prev live: 32 B/fish per iteration */
#define FSB_RUN_FUSED_LEAN 3u /* persistent, x, y, w live and each swim computed twice:
                                 24 B/fish per iteration, more arithmetic */
#define FSB_RUN_FUSED_REGS 4u /* persistent, all five values of every fish held in
                                 registers for the whole launch: the columns are read
                                 once and written once, no bytes per iteration.  Schools
                                 of at most 4 x 512 x (co-resident blocks) groups of four
                                 fish (2^21 + 3 fish on MI355X); FSB_ERR_UNSUPPORTED above */
#define FSB_RUN_FUSED_DEEP 5u /* persistent, x, y, w live, several iterations per grid
                                 barrier: positions do not depend on weights, so the
                                 differences of the next iterations are formed before
                                 their maxima are known; each swim is computed twice,
                                 32 B per fish per barrier (x, y, w and cur read and
                                 written).  8 iterations per barrier (4 B per
                                 fish-iteration) for schools of up to 5 x 2^20 fish, 4
                                 above (8 B per fish-iteration, in blocks that
                                 keep three waves per SIMD: faster there on MI355X);
                                 the environment variable FSB_DEEP_DEPTH, read once,
                                 may force 2, 4 or 8.
                                 FSB_ERR_UNSUPPORTED under the weighted swim rule or a
                                 reduce_mode other than FSB_REDUCE_COMPENSATED */
#define FSB_RUN_PLAIN_SPLIT 6u /* fsb_step n_steps times: two kernels per iteration
                                  (swim pass 24 B per fish, feed pass 20 B) */

typedef struct fsb_config {
    uint64_t n_fish;      /* fish in the school, >= 1 */
    uint64_t seed;        /* Philox key */
    float pond_half;      /* H in (0, 2^63]: the pond is [-H, H]^2 (Sec. 2.1.2: 200x200 ->
                             100); the bound keeps x*x + y*y finite */
    float swim_step;      /* S: per-axis displacement in [-S, S); 0 (zero swim) or
                             >= 2^-103 (so that S * 2^-23 is exact) */
    float w_init_lo;      /* initial weights in [lo, hi], lo <= hi */
    float w_init_hi;
    float w_min;          /* weight limits applied by feeding, w_min <= w_max */
    float w_max;          /* all four weight bounds within [-2^24, 2^24], so that no
                             float32 partial sum of w*x can overflow (2^40 fish x 2^24
                             x 2^63 = 2^127) */
    uint32_t reduce_mode; /* FSB_REDUCE_* */
    uint32_t history_len; /* per-iteration records kept, >= 1 (a ring) */
    uint32_t swim_rule;   /* FSB_SWIM_* flags, 0 = plain random swim */
} fsb_config;

/* The school's state: five float32 columns of n_fish (caller-owned device
 * memory).  For a batch of schools the columns are packed school after
 * school (see fsb_batch_init). */
typedef struct fsb_state {
    float *x;
    float *y;
    float *w;
    float *prev;
    float *cur;
} fsb_state;

/* What one iteration reduced, as kept in the workspace ring. */
typedef struct fsb_record {
    double sum_w;     /* sum of post-feed weights */
    double sum_wx;    /* sum of w*x */
    double sum_wy;    /* sum of w*y */
    float max_delta;  /* M = max |prev - cur| (exact) */
    uint32_t step_lo; /* low 32 bits of the iteration index it belongs to */
} fsb_record;

typedef struct fsb_school fsb_school; /* opaque host-side handle */
typedef struct fsb_batch fsb_batch;   /* opaque host-side handle */

/* fsb_tuning.schedule: how the tiles of a sweep are shared among the
 * wavefronts of the persistent batched kernel (the GPU counterpart of the
 * loop schedules of Sec. 2.3.2, Experiment 2).  Results do not depend on it. */
#define FSB_SCHED_STATIC 0u  /* chunks of chunk_tiles consecutive tiles dealt to the W
                                wavefronts round robin, the same in every sweep; chunk_tiles
                                0 = one chunk of ceil(n_tiles / W) tiles per wavefront */
#define FSB_SCHED_DYNAMIC 1u /* chunks of chunk_tiles consecutive tiles, handed out in order
                                by one device-scope atomic counter per sweep (one atomic per
                                chunk) */
#define FSB_SCHED_GUIDED 2u  /* as dynamic, the chunk starting at tile p spanning
                                max(chunk_tiles, ceil((n_tiles - p) / W)) tiles */

/* Launch shape of the persistent batched kernel. */
typedef struct fsb_tuning {
    uint32_t block_size;       /* threads per block: 256 or 1024 */
    uint32_t fish_per_thread;  /* fish per lane per tile: 4, 8 or 16 (a tile is one
                                  wavefront's share of one school: 64 x this many fish) */
    uint32_t steps_per_launch; /* iterations per persistent launch, >= 1 */
    uint32_t blocks_per_cu;    /* resident blocks per compute unit to use (0 = all that fit) */
    uint32_t variant;          /* 0 = chosen by the library (deep with 256-thread blocks where
                                  it can run, else by footprint), FSB_RUN_FUSED_PREV (x, y, w,
                                  prev live: 32 B/fish per iteration), FSB_RUN_FUSED_LEAN (x, y,
                                  w live, each swim done twice: 24 B/fish) or FSB_RUN_FUSED_DEEP
                                  (8 iterations per grid barrier, 3 B/fish-iteration; needs
                                  block_size 256, compensated sums, no weighted rule) */
    uint32_t schedule;         /* FSB_SCHED_* */
    uint32_t chunk_tiles;      /* static: tiles per chunk (0 = n_tiles / W); dynamic: tiles
                                  per chunk, >= 1; guided: smallest chunk, >= 1 */
} fsb_tuning;

/* ---- errors ------------------------------------------------------------ */

/* Static text for a return code. */
const char *fsb_strerror(int code);
/* Message of the last failing call on this thread ("" if none). */
const char *fsb_last_error(void);
int fsb_abi_version(void);

/* ---- one school -------------------------------------------------------- */

/* Bytes of device workspace a school with this config needs (256-byte
 * aligned start).  Pure host arithmetic.  Returns FSB_ERR_INVALID_ARG for a
 * bad config. */
int fsb_workspace_bytes(const fsb_config *cfg, size_t *out_bytes);

/* Initialisation (Sec. 2.1.1: random position and weight; objective = the
 * distance from the pond centre): writes all five columns from the init
 * draws, clears the workspace's control words, and returns a handle at
 * iteration t = 0.  `workspace` is caller-owned device memory of at least
 * fsb_workspace_bytes, 256-byte aligned, used by this handle only.  The
 * handle copies `cfg` and the pointers; the memory must outlive it.
 * Asynchronous. */
int fsb_init(const fsb_config *cfg, fsb_state state, void *workspace,
             size_t workspace_bytes, void *stream, fsb_school **out);

/* Wrap existing state (resume from a checkpoint, or a hand-made school) at
 * iteration `t`, without writing the columns.  The state must be one an
 * iteration could leave: cur == sqrtf(x*x + y*y) in binary32 (each operation
 * rounded on its own), since the kernels recompute a fish's objective from
 * its position rather than read cur; prev is the objective before the last
 * swim.  Clears the control words.  Asynchronous. */
int fsb_attach(const fsb_config *cfg, fsb_state state, void *workspace,
               size_t workspace_bytes, void *stream, uint64_t t,
               fsb_school **out);

/* One iteration t (swim, objective, diff, school max, feeding, barycentre
 * sums; Sec. 2.1.2 and eat() of Sec. 2.3.2) as two kernels on the stream;
 * the record goes to slot t mod history_len; t advances.  Asynchronous.
 * FSB_ERR_INVALID_ARG once t reaches 2^32 (the counter word is 32 bits). */
int fsb_step(fsb_school *h);

/* n_steps iterations of the simulation loop (Sec. 2.1.3: the total
 * iteration count is a Config parameter; each iteration swims every fish,
 * Sec. 2.1.2, then runs eat(), Sec. 2.3.2).  FSB_RUN_PLAIN_SPLIT issues
 * fsb_step n_steps times; FSB_RUN_PLAIN launches one kernel per iteration,
 * the feed of each iteration fused into the swim of the next (the columns are
 * complete once the run's last kernel has finished, as for every mode);
 * the FSB_RUN_FUSED* modes run them in one persistent launch with a grid
 * barrier per iteration (per 4 or 8 iterations for FSB_RUN_FUSED_DEEP).  All give
 * bit-identical columns and maxima (the sums agree to rounding and, for
 * FSB_RUN_PLAIN and FSB_RUN_PLAIN_SPLIT, are bit-identical too; each mode is
 * deterministic).  Asynchronous; FSB_ERR_UNSUPPORTED if the fused grid cannot
 * be co-resident, for FSB_RUN_FUSED_REGS on a school too large for it, or for
 * a fused mode under FSB_REDUCE_CRITICAL_F32.  If the runtime refuses a launch
 * part-way (FSB_ERR_HIP), the launches already enqueued still run, and the
 * columns may hold a state between two iterations that the handle's t does
 * not describe: attach a saved state (fsb_attach) or initialise again before
 * going on. */
int fsb_run(fsb_school *h, uint64_t n_steps, uint32_t mode);

/* Test hook: one iteration with the displacements dx[n_fish], dy[n_fish]
 * (device float32) used in place of the Philox draws.  t advances.
 * Asynchronous. */
int fsb_step_displaced(fsb_school *h, const float *dx, const float *dy);

/* Barycentre of the last completed iteration: out_xy = (sum w*x / sum w,
 * sum w*y / sum w) in binary64; out_sums3 (nullable) = the three sums.
 * The paper defines no barycentre: this weight-weighted centre of the
 * school's post-feed positions is a reading added to the method, with the
 * fish record of Sec. 2.1.1 as its terms (all weights equal: the plain mean
 * position).
 * Synchronises the stream.  FSB_ERR_STATE before the first iteration;
 * FSB_ERR_DEVICE if a kernel reported a failure. */
int fsb_barycentre(fsb_school *h, double out_xy[2], double *out_sums3);

/* M = max |diff| of the last completed iteration: the school-wide maximum
 * that eat() takes with the Reduction Construct (Sec. 2.3.2, Experiment 3),
 * of diff = prevObjective - currentObjective, read as a magnitude (a signed
 * maximum can be 0 or negative and would invert feeding).  Synchronises. */
int fsb_max_delta(fsb_school *h, float *out_max);

/* Records of iterations [first, first + count): each must still be in the
 * ring (t - history_len <= first, first + count <= t).  Synchronises. */
int fsb_history(fsb_school *h, uint64_t first, uint64_t count,
                fsb_record *out);

/* Wait for the handle's work; reports asynchronous HIP or kernel errors. */
int fsb_sync(fsb_school *h);

/* Current iteration index (the next iteration fsb_step will run). */
int fsb_step_index(const fsb_school *h, uint64_t *out_t);

/* Move the iteration index (resume); clears the pending maximum slot.
 * Asynchronous. */
int fsb_set_step_index(fsb_school *h, uint64_t t);

/* Free the handle (host memory only; the caller frees device memory after
 * the stream's work is done). */
int fsb_destroy(fsb_school *h);

/* ---- batch of independent schools ------------------------------------- */

/* Many independent schools advanced together (the same iteration on every
 * school): school s holds fish [starts[s], starts[s] + sizes[s]) of packed
 * float32 columns of length packed_len (caller-owned device memory, the
 * same five columns as one school).  starts[s] is a multiple of 4 (each
 * school 16-byte aligned; multiples of 64, i.e. 256 bytes, stream about
 * 15% faster because no wavefront row then straddles an extra cache line),
 * starts are increasing and schools do not overlap; gaps are allowed and
 * never touched.  School s draws from its own
 * Philox key seeds[s] with the same counter layout as a single school, so
 * school s evolves exactly as a single school of sizes[s] fish with seed
 * seeds[s] would.  All host arrays are read during the call only. */

/* Workspace bytes for such a batch (pure host arithmetic).  common supplies
 * H, S, the weight ranges, reduce_mode and history_len; its n_fish and seed
 * are ignored. */
int fsb_batch_workspace_bytes(const fsb_config *common, uint32_t n_schools,
                              const uint64_t *starts, const uint64_t *sizes,
                              size_t *out_bytes);

/* Initialise every school (Sec. 2.1.1 draws, per-school key) and return a
 * handle at iteration 0 with the default tuning (8 fish per lane, 100
 * iterations per launch, variant chosen by the library; 256 threads, which
 * lets it choose the deep variant, with compensated sums and no weighted
 * rule, else 1024 threads).  Uploads
 * the school tables (synchronous copies), then enqueues the init kernel on
 * `stream`.  FSB_ERR_UNSUPPORTED for reduce_mode FSB_REDUCE_CRITICAL_F32. */
int fsb_batch_init(const fsb_config *common, uint32_t n_schools,
                   const uint64_t *starts, const uint64_t *sizes,
                   const uint64_t *seeds, fsb_state packed, uint64_t packed_len,
                   void *workspace, size_t workspace_bytes, void *stream,
                   fsb_batch **out);

/* n_steps iterations of every school (the loop of Sec. 2.1.3 and eat() of
 * Sec. 2.3.2 run on each school independently; batching many schools is an
 * addition of this library, not part of the paper): persistent launches of
 * steps_per_launch iterations (one grid barrier per iteration), each launch
 * a replay of a captured HIP graph.  tuning NULL keeps the handle's tuning;
 * otherwise it becomes the handle's tuning.  Per-fish state and maxima do
 * not depend on the tuning (sums agree to rounding).  Asynchronous. */
int fsb_batch_run(fsb_batch *b, uint64_t n_steps, const fsb_tuning *tuning);

/* Results of the last completed iteration, per school: out_xy[2*n_schools]
 * barycentres (nullable), out_sums[3*n_schools] (sum w, sum w*x, sum w*y;
 * nullable), out_max[n_schools] (M, the maximum eat() takes, Sec. 2.3.2;
 * nullable).  The barycentre is not in the paper (see fsb_barycentre).
 * Host arrays, caller-owned.  Synchronises.  FSB_ERR_STATE before the first
 * iteration. */
int fsb_batch_results(fsb_batch *b, double *out_xy, double *out_sums,
                      float *out_max);

/* Barycentre of every school after the last completed iteration (the
 * single-school fsb_barycentre, per school): out_xy[2*n_schools] = (sum w*x
 * / sum w, sum w*y / sum w) of school s at 2s, 2s+1 (required);
 * out_sums[3*n_schools] the three sums (nullable).  Host arrays,
 * caller-owned.  The paper defines no barycentre: a reading added to the
 * method.  Synchronises.  FSB_ERR_INVALID_ARG for a NULL handle or out_xy,
 * FSB_ERR_STATE before the first iteration. */
int fsb_batch_barycentre(fsb_batch *b, double *out_xy, double *out_sums);

/* Records of iteration `step` for every school (out[n_schools]); the
 * iteration must still be in the history ring.  Synchronises. */
int fsb_batch_history(fsb_batch *b, uint64_t step, fsb_record *out);

/* Time candidate tunings, each on probe_steps real iterations (the schools
 * advance): 256 or 1024 threads x 4, 8 or 16 fish per lane with the variant
 * the library would pick; then the other variant; then the dynamic (4, 8, 16
 * and 64 tiles per chunk) and guided (at least 4) schedules against static;
 * then iterations per launch.  Keeps the fastest as the handle's tuning and
 * copies it to *out.  If the environment variable FSB_AUTOTUNE_CACHE names a
 * file, a tuning recorded there for this device and batch shape is reused
 * without probing, and new results are appended.  Synchronises. */
int fsb_autotune(fsb_batch *b, uint64_t probe_steps, fsb_tuning *out);

int fsb_batch_get_tuning(const fsb_batch *b, fsb_tuning *out);
int fsb_batch_step_index(const fsb_batch *b, uint64_t *out_t);
/* Wait for the handle's work; reports asynchronous HIP or kernel errors. */
int fsb_batch_sync(fsb_batch *b);
int fsb_batch_destroy(fsb_batch *b);

/* ---- allocation-free entry point --------------------------------------- */

/* For callers that cannot allocate device memory, not even a workspace ahead
 * of time: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Runs iterations t .. t + n_steps - 1 of the school held
 * in `state` exactly as fsb_attach(cfg, state, workspace, t) followed by
 * fsb_run(h, n_steps, mode) would (the same kernels and launch shapes, so the
 * same bits in the columns and the records), with a scratch array inside
 * the library in place of the workspace.  The scratch is 1 MiB of device
 * memory per GPU, held from the first call on that GPU until the process
 * ends; its use does not grow with n_fish, n_steps or history_len (the
 * record ring is the caller's), so no accepted size exceeds it.
 *   cfg      as for fsb_attach (history_len = the length of `records`).
 *   state    the five columns at iteration t (device, caller-owned; cur must
 *            equal sqrtf(x*x + y*y) as after any iteration), updated in place.
 *   records  device array of cfg->history_len records (caller-owned, 8-byte
 *            aligned): the record of iteration s goes to records[s mod
 *            history_len].
 *   status   device word (nullable, caller-owned): receives the kernels'
 *            failure flags of this call, 0 if none (bit 0: a persistent
 *            kernel's grid barrier timed out; the records are then
 *            incomplete).
 *   stream   a stream of the current device; everything is enqueued on it and
 *            the call returns without waiting.
 * Calls no hipMalloc, hipFree or other allocating routine.  Every call on a
 * GPU uses that GPU's one scratch: calls that overlap on one GPU (concurrent
 * streams, or host threads) race and give wrong results; serialise them.
 * Each call clears the scratch's control words itself.  Errors: as
 * fsb_attach and fsb_run (FSB_ERR_INVALID_ARG for NULL records, a misaligned
 * records or status, an unknown mode or t + n_steps > 2^32; all checked
 * before any HIP call). */
int fsb_run_static(const fsb_config *cfg, fsb_state state, uint64_t t,
                   uint64_t n_steps, uint32_t mode, fsb_record *records,
                   uint32_t *status, void *stream);

/* ---- instrumentation --------------------------------------------------- */

/* Kernel timing: with every = n > 0, every n-th launch of each kernel kind
 * (the 1st, the (n+1)-th, ...) is timed by HIP events on the handle's
 * stream: the plain passes' launches record a start and a stop event
 * themselves (the kernel's own execution), the other launches are bracketed
 * by them (n = 1 times every launch; sampling keeps the events' own cost out
 * of the other launches); every = 0 turns timing off.
 * fsb_kernel_times synchronises and returns, per kernel kind
 * (FSB_KERNEL_*), the number of timed launches and their summed duration in
 * milliseconds since the previous read (reading resets the counts). */
#define FSB_KERNEL_SWIM_EVAL 0 /* plain pass 1: swim, objective, max |diff| */
#define FSB_KERNEL_FEED_BARY 1 /* plain pass 2: feeding, barycentre sums */
#define FSB_KERNEL_FUSED 2     /* persistent multi-iteration kernel */
#define FSB_KERNEL_INIT 3
#define FSB_KERNEL_FEED_SWIM 4 /* FSB_RUN_PLAIN's pipelined pass: feed of t - 1, swim of t */
#define FSB_KERNEL_KINDS 5
int fsb_profile_enable(fsb_school *h, int every);
int fsb_kernel_times(fsb_school *h, uint64_t counts[FSB_KERNEL_KINDS],
                     double ms[FSB_KERNEL_KINDS]);
/* The same for a batch: launches of the persistent batched kernel. */
int fsb_batch_profile_enable(fsb_batch *b, int every);
int fsb_batch_kernel_times(fsb_batch *b, uint64_t *count, double *ms);

/* Synchronisation cost of the persistent form: one persistent launch of
 * `grid` blocks of 1024 threads (0 = the grid of the streaming persistent
 * variants for this school) that does n_barriers >= 1 of its grid barriers and nothing
 * else.  Each barrier carries the school-wide max, the dependency of eat()
 * (Sec. 2.3.2): barrier k folds max(block index + k) over the grid.  Writes
 * the average microseconds per barrier (HIP events around the launch, so a
 * launch's own overhead is spread over n_barriers) and, if out_max is
 * non-NULL, the max of the last barrier (grid - 1 + n_barriers - 1).  Uses
 * the handle's workspace and stream, touches no fish; finishes a pending
 * record first; synchronises.  FSB_ERR_INVALID_ARG if grid exceeds the
 * co-resident maximum. */
int fsb_barrier_probe(fsb_school *h, uint32_t grid, uint32_t n_barriers, double *out_us,
                      uint32_t *out_max);

/* out[i] = the square root every kernel uses for the objective (Sec. 2.1.1:
 * Euclidean distance), i < n: a correctly rounded binary32 sqrt built from
 * the hardware estimate and one residual correction, with the general
 * expansion below 2^-96.  in and out are device arrays of n floats, 4-byte
 * aligned (caller-owned); enqueued on `stream`, asynchronous.  For testing
 * it against IEEE sqrt. */
int fsb_eval_sqrt(const float *in, float *out, uint64_t n, void *stream);

/* Plain-VALU ceiling probe (instrumentation; measures the second roofline
 * the persistent kernels are held against): `blocks` blocks of 256 threads,
 * every lane running `iters` rounds of independent chains of one kind of
 * vector instruction (FSB_PROBE_FMA: 8 v_fma_f32 per round; FSB_PROBE_PHILOX:
 * one Philox4x32-10 call, as the kernels draw them, on each of 2 counters,
 * 2 v_mad_u64_u32 and 2 v_bitop3_b32 per Philox round, 80 per round of the
 * probe; FSB_PROBE_MIXED: one Philox call and 40 v_fma_f32, the integer and
 * float mix of the kernels' swims, 80 per round).  out: device memory of at least
 * blocks x 256 x 4 bytes, overwritten with one word per lane (keeps the
 * chains live).  Synchronises the stream; *out_ms gets the launch's duration
 * by HIP events and *out_lane_instructions the lane instructions it issued
 * (blocks x 256 x iters x per round).  FSB_ERR_INVALID_ARG for an unknown
 * kind, zero blocks or iters, NULL or misaligned pointers, or out too small. */
#define FSB_PROBE_FMA 0u
#define FSB_PROBE_PHILOX 1u
#define FSB_PROBE_MIXED 2u
#define FSB_PROBE_KINDS 3u
int fsb_valu_probe(uint32_t kind, uint32_t blocks, uint32_t iters, void *out, size_t out_bytes,
                   void *stream, double *out_ms, uint64_t *out_lane_instructions);

/* Streaming probe (instrumentation; the copy rate of the plain kernels' own
 * access pattern, against which their bandwidth is judged): the four device
 * columns cols[0..3] of n floats each (n a positive multiple of 4, each
 * 16-byte aligned) are read and written in place once, as float4 groups, one
 * group per thread per round on `grid` blocks of 256 threads (0: 512, the
 * plain passes' grid), every float gaining 1.0f: 32 B per group of four
 * elements, the pipelined pass's traffic.  streamed != 0 makes every access
 * non-temporal.  Synchronises the stream; *out_ms gets the launch's duration
 * by HIP events.  FSB_ERR_INVALID_ARG for NULL or misaligned pointers or a
 * bad n. */
int fsb_sweep_probe(float *cols[4], uint64_t n, uint32_t grid, uint32_t streamed, void *stream,
                    double *out_ms);

#ifdef __cplusplus
}
#endif
#endif
