// fsb_internal.hpp -- layout of the device workspace and the launchers the
// C ABI layer (fsb_api.cpp) calls in the kernel translation unit.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "fsb.h"

namespace fsb {

// Largest grid of any single-school kernel; sizes the per-block arrays.
constexpr uint32_t kMaxGrid = 8192;
constexpr size_t kAlign = 256;

// Control words at the start of the workspace (zeroed by init/attach).
struct Ctrl {
    uint32_t last_max;        // bits of M of the last iteration whose record is pending
    uint32_t error;           // kernel-reported failure flags (kErr*)
    uint32_t step;            // batches: next iteration (advanced by each launch)
    uint32_t probe_max;       // M of the last barrier of a barrier probe
    float naive_acc[2][4];    // float32 atomic sums of the naive and critical modes, slot t & 1
    uint32_t crit_max[2];     // critical mode: max |diff| bits by per-fish atomics, slot t & 1
    uint32_t redo[2];         // deep batches: some school's look-ahead guess failed in the sweep
                              // of this parity, its maxima are recomputed
    uint32_t pad[48];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl is one aligned block");

constexpr uint32_t kErrBarrierTimeout = 1u;

// Polls of a persistent kernel's barrier wait before it gives up (with
// 2-cycle-group sleeps, well over a second).  The environment variable
// FSB_BARRIER_SPIN_LIMIT (read once) overrides it, so that tests can force
// the time-out path from the host; every wait still ends.
constexpr uint32_t kBarrierSpinLimit = 1u << 22;
uint32_t barrier_spin_limit();

// Synchronisation words of the persistent kernels' grid barrier (cleared
// before every persistent launch).  A barrier reduces KD maxima at once
// (KD = 1, or the look-ahead depth of the deep kernel, at most kMaxDepth):
//   kSyncPub    KD 64-bit words {max (low half), barrier number (high half)}
//               that block 0 publishes when every block has arrived;
//   kSyncSlots  KD 64-bit words per block, {its max, the barrier number it
//               has reached}.
constexpr uint32_t kLineWords = 64;
constexpr uint32_t kMaxDepth = 8;
constexpr uint32_t kSyncPub = 0;
constexpr uint32_t kSyncSlots = kLineWords;
constexpr uint32_t kMaxBarrierBlocks = 1024;  // largest persistent grid
constexpr uint32_t kSyncWords = kSyncSlots + 2 * kMaxDepth * kMaxBarrierBlocks;
static_assert(2 * kMaxDepth <= kLineWords, "the publish words fit one line");

// Workspace of one school:
//   [Ctrl][history ring][block maxima u32 x kMaxGrid x 2 (slot t & 1)]
//   [block partials f64 x 3 x kMaxGrid x 2 (slot t & 1)][barrier sync area]
//   [deep kernel's block partials f64 x 3 x kMaxBarrierBlocks x 2 kMaxDepth
//    (slot t mod 2 kMaxDepth)]
struct Layout {
    size_t ctrl, hist, blockmax, partials, sync, deep, total;
};
constexpr uint32_t kDeepSlots = 2 * kMaxDepth;

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr Layout school_layout(uint32_t history_len) {
    Layout L{};
    L.ctrl = 0;
    L.hist = align_up(L.ctrl + sizeof(Ctrl), kAlign);
    L.blockmax = align_up(L.hist + (size_t)history_len * sizeof(fsb_record), kAlign);
    L.partials = align_up(L.blockmax + 2 * (size_t)kMaxGrid * sizeof(uint32_t), kAlign);
    L.sync = align_up(L.partials + 2 * 3 * (size_t)kMaxGrid * sizeof(double), kAlign);
    L.deep = align_up(L.sync + kSyncWords * sizeof(uint32_t), kAlign);
    L.total = align_up(L.deep + (size_t)kDeepSlots * 3 * kMaxBarrierBlocks * sizeof(double),
                       kAlign);
    return L;
}

// Device scratch of the allocation-free entry point (fsb_run_static): every
// area of one school's workspace except the record ring, which that call's
// caller passes.  None of them grows with the school, the iteration count or
// the ring, so one fixed array serves any call.  A file-scope array in the
// kernel translation unit; each GPU holds its own copy until the process
// ends.
constexpr size_t kStaticScratchBytes = 1u << 20;
constexpr Layout kStaticLayout = school_layout(0);
static_assert(kStaticLayout.total <= kStaticScratchBytes, "the static scratch holds a school");
// Device address of the current device's copy (looked up once per device).
hipError_t static_scratch(void** out);
// Copies the control block's error flags to *out (a device word), on the stream.
struct SchoolArgs;
hipError_t launch_copy_error(const SchoolArgs& a, uint32_t* out, hipStream_t stream);

// Everything a single-school kernel needs, passed by value.
struct SchoolArgs {
    float *x, *y, *w, *prev, *cur;
    uint64_t n;           // fish
    uint32_t k0, k1;      // Philox key (seed lo, hi)
    float H, S, wmin, wmax;
    uint32_t rule;        // swim rule flags (FSB_SWIM_*)
    Ctrl *ctrl;
    fsb_record *hist;
    uint32_t hist_len;
    uint32_t *blockmax;   // [2][kMaxGrid] per-block max |diff| bits of the swim of iteration t,
                          // slot t & 1
    double *partials;     // [2][3][kMaxGrid] per-block binary64 sums
    uint32_t *sync;       // [kSyncWords] persistent-kernel barrier words
    double *deep;         // [kDeepSlots][3][kMaxBarrierBlocks] the deep kernel's partials
};

// Step-specific arguments of the plain passes.
struct StepArgs {
    uint32_t t;           // iteration index (low 32 bits; host keeps t < 2^32)
    uint32_t swim_grid;   // blocks of the launch that swam the iteration being fed (the feed
                          // reads that many maxima); the swim pass's own grid when it launches
    uint32_t combine;     // swim pass block 0 first writes the pending record
    uint32_t prev_t;      // iteration whose record is pending
    uint32_t prev_grid;   // blocks that produced its partials
    uint32_t naive;       // sums in float32 accumulators (naive or critical mode)
    uint32_t critical;    // FSB_REDUCE_CRITICAL_F32: one atomic per fish for M and the sums
    const float *dx;      // test hook: displacements instead of draws (or null)
    const float *dy;
};

// Arguments of the persistent multi-iteration kernel.
struct FusedArgs {
    uint32_t t0;          // first iteration of the launch
    uint32_t steps;       // iterations in the launch, >= 1
    uint32_t naive;
    uint32_t streaming;   // non-temporal loads/stores (state larger than the last-level cache)
    uint32_t spin_limit;  // barrier polls before giving up
    uint32_t lean;        // keep (x, y, w) live and redo each swim (24 B/fish) instead of
                          // keeping (x, y, w, prev) (32 B/fish)
    uint32_t regs;        // > 0: the register-resident kernel holding `regs` groups of four
                          // fish per thread (1, 2 or 4); streaming and lean are then unused
    uint32_t deep;        // > 0: the deep kernel, `deep` iterations per grid barrier (lean is
                          // then unused)
    float look_theta;     // deep kernel, plain swim: > 0 lets the look-ahead skip the objective
                          // of a fish that cannot reach theta times the smallest maximum of
                          // the current superstep (0 = every objective is formed)
};

// Schools from this size on run the deep kernel's look-ahead with the skip
// test (smaller schools' maxima vary more from one iteration to the next, so
// the recomputation a wrong guess costs would come more often).
constexpr uint64_t kLookFilterFish = 1ull << 20;
// Fraction of the current maxima below which a look-ahead objective is skipped.
constexpr float kLookTheta = 1.0f - 0x1p-7f;
// theta for a school of n fish: kLookTheta from kLookFilterFish fish on, else
// 0; the environment variable FSB_LOOKAHEAD_FILTER (read once) may say "off"
// (never skip) or "redo" (theta 2: every guess fails and every superstep's
// maxima are recomputed, for tests of that path).
float look_theta(uint64_t n);

// Launchers (fsb_kernels.hip).  All enqueue on `stream` and return the HIP
// status of the launch.
uint32_t plain_grid(uint64_t n);  // swim pass (and init)
uint32_t feed_grid(uint64_t n);   // feed pass
uint32_t pipe_grid(uint64_t n);   // pipelined pass (feed of t - 1 and swim of t)
hipError_t launch_reset(const SchoolArgs& a, hipStream_t stream);
hipError_t launch_init(const SchoolArgs& a, float wlo, float whi, hipStream_t stream);
// The plain passes; with a start and a stop event the launch records them
// itself, around the kernel's own execution.
hipError_t launch_swim_eval(const SchoolArgs& a, const StepArgs& s, hipStream_t stream,
                            hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// The feed pass; write_cur also stores each fish's objective in cur (the
// closing pass of a pipelined run, whose passes leave cur unwritten).
hipError_t launch_feed_bary(const SchoolArgs& a, const StepArgs& s, uint32_t grid,
                            hipStream_t stream, hipEvent_t start = nullptr,
                            hipEvent_t stop = nullptr, bool write_cur = false);
// The pipelined pass: feeds iteration s.t - 1 and swims iteration s.t.
hipError_t launch_feed_swim(const SchoolArgs& a, const StepArgs& s, uint32_t grid,
                            hipStream_t stream, hipEvent_t start = nullptr,
                            hipEvent_t stop = nullptr);
hipError_t launch_combine(const SchoolArgs& a, uint32_t t, uint32_t grid, uint32_t naive,
                          hipStream_t stream);
// Largest co-resident grid of the persistent kernel (0 if it cannot run).
hipError_t fused_resident_grid(uint32_t naive, uint32_t* out_grid);
// Grid the persistent kernel uses for n fish given the resident maximum.
uint32_t fused_grid(uint64_t n, uint32_t resident);
// Iterations per grid barrier of the deep kernel for a school of n fish:
// eight up to kDeepWideFish fish, four above, unless the environment variable
// FSB_DEEP_DEPTH (read once) says 2, 4 or 8.  Eight unrolled iterations need
// ~230 registers per lane, so that instance runs 512-thread blocks (two waves
// per SIMD); four need ~150, so those instances run 768-thread blocks, three
// waves per SIMD, which hide more latency but barrier twice as often: the
// faster choice above ~5 x 2^20 fish, measured on MI355X.
constexpr uint64_t kDeepWideFish = 5ull << 20;
uint32_t deep_depth(uint64_t n);
// Threads per block of the deep kernel of a depth.
inline uint32_t deep_block(uint32_t depth) { return depth == 8 ? 512u : 768u; }
// Largest co-resident grid of the deep kernels of a depth, and the grid for n fish.
hipError_t deep_resident_grid(uint32_t depth, uint32_t* out_grid);
uint32_t deep_grid(uint64_t n, uint32_t depth, uint32_t resident);
// Largest co-resident grid of the register-resident kernels (0 if they cannot run).
hipError_t regs_resident_grid(uint32_t naive, uint32_t* out_grid);
// Launch plan of the register-resident kernel for n fish: its grid, and in
// *groups the groups of four fish per thread (1, 2 or 4); 0 if n does not fit.
uint32_t regs_plan(uint64_t n, uint32_t resident, uint32_t* groups);
hipError_t launch_fused(const SchoolArgs& a, const FusedArgs& f, uint32_t grid,
                        hipStream_t stream);
// out[i] = the kernels' square root of in[i] (instrumentation).
hipError_t launch_eval_sqrt(const float* in, float* out, uint64_t n, hipStream_t stream);
// f.steps grid barriers of the persistent kind and nothing else (instrumentation).
hipError_t launch_barrier_probe(const SchoolArgs& a, const FusedArgs& f, uint32_t grid,
                                hipStream_t stream);

// ---------------------------------------------------------------------------
// Batches of independent schools.
// ---------------------------------------------------------------------------

// A tile is one wavefront's share of one school for a sweep: the fish
// [4*group0, 4*group0 + n_fish) of school `school`, whose packed float4 index
// starts at `col4`.  It carries what the sweep needs (key, extent) so one
// 32-byte load describes it.  Tiles never straddle schools and are listed
// school after school.
struct Tile {
    uint64_t col4;     // float4 index of the tile's first group in the packed columns
    uint32_t school;
    uint32_t group0;   // first group (4 fish) of the tile within its school
    uint32_t n_fish;   // fish in the tile (the school's last group may be partial)
    uint32_t k0, k1;   // the school's Philox key
    uint32_t pad;
};
static_assert(sizeof(Tile) == 32, "one 32-byte load per tile");

struct BatchArgs {
    float *x, *y, *w, *prev, *cur;  // packed columns
    const Tile* tiles;              // [n_tiles]
    const uint32_t* tile_begin;     // [S+1] first tile of each school
    uint32_t n_tiles;
    uint32_t n_schools;
    float H, S, wmin, wmax, wlo, whi;
    uint32_t rule;                  // swim rule flags (FSB_SWIM_*)
    Ctrl* ctrl;
    uint32_t* sync;                 // barrier words
    uint32_t* step;                 // device iteration counter (advanced by each launch)
    uint32_t* school_max;           // [3][S] bits of M of iteration s in slot s % 3 (deep
                                    // kernel: [3 kMaxDepth][S], slot s % (3 kBatchDepth))
    double* tile_part;              // [2][3][tile_cap] per-tile binary64 sums, slot s & 1 (deep
                                    // kernel: [2 kMaxDepth][3][tile_cap], slot s % (2 kBatchDepth))
    uint32_t tile_cap;
    uint32_t max_slots;             // slots of the per-school max ring the layout holds
    float* school_naive;            // [2][S][4] float32 atomic sums of the naive mode
    fsb_record* rec;                // [hist_len][S]
    uint32_t hist_len;
    uint32_t steps;                 // iterations per launch
    uint32_t spin_limit;            // barrier polls before giving up
    // Tile schedule.  n_chunks == 0: static, chunk c = tiles [c * static_chunk,
    // (c + 1) * static_chunk) to wavefront c mod W.  Otherwise wavefronts take
    // chunk c = [chunk_start[c], chunk_start[c+1]) in the order an atomic
    // counter hands them out; the counter of sweep phase p is
    // queue[(p & 1) * kLineWords].
    uint32_t static_chunk;          // >= 1
    const uint32_t* chunk_start;    // [n_chunks + 1]
    uint32_t n_chunks;
    uint32_t* queue;                // two counters, one 256-byte line each
    // Deep kernel's look-ahead skip test (plain swim): schools of at least
    // look_min_tiles tiles skip the objectives of fish whose move cannot reach
    // look_theta times the school's smallest current maximum (0 = never).
    float look_theta;
    uint32_t look_min_tiles;
    uint32_t* school_flag;          // [S] 1: the school's next maxima must be recomputed
};

// Fraction of a school's current maxima under which the batched look-ahead
// skips an objective.  A school of 2^16 fish or more; smaller schools' maxima
// vary by several percent between iterations and are not skipped.
constexpr float kBatchLookTheta = 0.98f;
constexpr uint64_t kBatchLookFish = 1ull << 16;
// theta of the batched look-ahead: kBatchLookTheta, or as FSB_LOOKAHEAD_FILTER
// (read once) says: "off" 0, "redo" 2 (every guess fails, for tests).
float batch_look_theta();

// Workspace of a batch (offsets in bytes).
struct BatchLayout {
    size_t ctrl, sync, tile_begin, tiles, tile_part, school_max, school_naive, rec, chunks,
        queue, school_flag, total;
    uint32_t tile_cap;
};

// `deep`: room for the deep kernel's per-iteration rings (it needs
// compensated sums and no weighted rule; other configurations never run it).
inline BatchLayout batch_layout(uint32_t n_schools, uint64_t tile_cap, uint32_t history_len,
                                bool deep) {
    BatchLayout L;
    const size_t S = n_schools;
    const size_t part_slots = deep ? 2 * kMaxDepth : 2, max_slots = deep ? 3 * kMaxDepth : 3;
    L.tile_cap = (uint32_t)tile_cap;
    L.ctrl = 0;
    L.sync = align_up(sizeof(Ctrl), kAlign);
    L.tile_begin = align_up(L.sync + kSyncWords * sizeof(uint32_t), kAlign);
    L.tiles = align_up(L.tile_begin + (S + 1) * 4, kAlign);
    L.tile_part = align_up(L.tiles + tile_cap * sizeof(Tile), kAlign);
    L.school_max = align_up(L.tile_part + part_slots * 3 * tile_cap * sizeof(double), kAlign);
    L.school_naive = align_up(L.school_max + max_slots * S * 4, kAlign);
    L.rec = align_up(L.school_naive + 2 * S * 4 * sizeof(float), kAlign);
    L.chunks = align_up(L.rec + (size_t)history_len * S * sizeof(fsb_record), kAlign);
    L.queue = align_up(L.chunks + (tile_cap + 1) * sizeof(uint32_t), kAlign);
    L.school_flag = align_up(L.queue + 2 * kLineWords * sizeof(uint32_t), kAlign);
    L.total = align_up(L.school_flag + S * sizeof(uint32_t), kAlign);
    return L;
}

// Launch shapes of the batch kernel.
constexpr uint32_t kBatchBlocks[2] = {256, 1024};
constexpr uint32_t kBatchFishPerLane[3] = {4, 8, 16};
constexpr uint32_t kBatchMinTileFish = 64 * 4;

// Batch kernel variants.
constexpr uint32_t kBatchPrev = 0;  // x, y, w, prev live: 32 B/fish per iteration
constexpr uint32_t kBatchLean = 1;  // x, y, w live, each swim done twice: 24 B
constexpr uint32_t kBatchDeep = 2;  // kBatchDepth iterations per barrier (256-thread blocks,
                                    // compensated sums, no weighted rule): 24 B per superstep
constexpr uint32_t kBatchDepth = 8;

hipError_t launch_batch_init(const BatchArgs& a, uint32_t block, hipStream_t stream);
hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t stream);
// Persistent launch of a.steps iterations; `streaming` selects non-temporal
// column access, `variant` one of kBatch*.  Cooperative, so the grid is
// guaranteed co-resident.
hipError_t launch_batch(const BatchArgs& a, uint32_t block, uint32_t fish_per_lane,
                        uint32_t naive, uint32_t streaming, uint32_t variant, uint32_t grid,
                        hipStream_t stream);
// Largest co-resident grid for a shape and variant (0 if it cannot run).
hipError_t batch_resident_grid(uint32_t block, uint32_t fish_per_lane, uint32_t naive,
                               uint32_t variant, uint32_t* out_grid);

}  // namespace fsb
