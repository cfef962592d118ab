// fsb_batch_api.cpp -- C ABI of batched schools (include/fsb.h, fsb_batch_*):
// argument checks, tile tables, graph capture and replay of the persistent
// batched kernel, result read-back and the launch-shape autotuner.
#include <hip/hip_runtime_api.h>

#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fsb.h"
#include "fsb_host.hpp"
#include "fsb_internal.hpp"
#include "fsb_plan.hpp"

using namespace fsb;

struct fsb_batch {
    fsb_config cfg;
    uint32_t n;
    std::vector<uint64_t> start, size, seed;
    uint64_t total_fish;
    fsb_state st;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    hipStream_t capture;  // non-null stream used only to capture graphs
    BatchLayout L;
    BatchArgs args;
    uint64_t t;
    bool has_result;
    fsb_tuning tuning;
    uint32_t table_fpl;   // fish per lane of the uploaded tile table (0 = none)
    uint32_t n_tiles;
    // uploaded chunk table: schedule, chunk size, wavefronts, tile table it cuts
    uint32_t chunk_sched, chunk_tiles, chunk_waves, chunk_fpl;
    hipGraphExec_t graph;
    uint32_t graph_steps, graph_grid, graph_block, graph_fpl, graph_variant, graph_sched,
        graph_chunks, graph_static;
    uint32_t profile_every;  // time every n-th launch (0 = off)
    uint64_t launches;
    Timer timer;
    ~fsb_batch() {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (capture) (void)hipStreamDestroy(capture);
    }
};

namespace {

// The deep variant needs compensated sums and positions that do not depend on
// weights (no weighted rule); the workspace of such a batch holds its rings.
bool deep_capable(const fsb_config& c) {
    return c.reduce_mode == FSB_REDUCE_COMPENSATED && !(c.swim_rule & FSB_SWIM_WEIGHTED);
}

// The kernel variant (kBatch*) of the tuning.  Variant 0: deep where it can
// run (256-thread blocks), else lean once the 32-byte variant's live columns
// reach the 256 MiB last-level cache (the single-school rule, measured the
// same way).
uint32_t batch_variant(const fsb_batch* b) {
    if (b->tuning.variant == FSB_RUN_FUSED_DEEP) return kBatchDeep;
    if (b->tuning.variant == FSB_RUN_FUSED_LEAN) return kBatchLean;
    if (b->tuning.variant == FSB_RUN_FUSED_PREV) return kBatchPrev;
    if (deep_capable(b->cfg) && b->tuning.block_size == 256) return kBatchDeep;
    return b->total_fish * 16ull >= (256ull << 20) ? kBatchLean : kBatchPrev;
}

// Build and upload the tile table for `fpl` fish per lane (synchronises).
int upload_tiles(fsb_batch* b, uint32_t fpl) {
    if (b->table_fpl == fpl) return FSB_OK;
    std::vector<Tile> tiles;
    std::vector<uint32_t> begin;
    build_tile_table(b->n, b->start.data(), b->size.data(), b->seed.data(), fpl, tiles, begin);
    if (tiles.size() > b->L.tile_cap) return fail(FSB_ERR_INVALID_ARG, "tile table exceeds its capacity");
    char* base = static_cast<char*>(b->ws);
    FSB_HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    FSB_HIP_TRY(hipMemcpy(base + b->L.tiles, tiles.data(), tiles.size() * sizeof(Tile),
                          hipMemcpyHostToDevice),
                "tile table upload");
    FSB_HIP_TRY(hipMemcpy(base + b->L.tile_begin, begin.data(), begin.size() * 4,
                          hipMemcpyHostToDevice),
                "tile index upload");
    b->table_fpl = fpl;
    b->n_tiles = (uint32_t)tiles.size();
    b->args.n_tiles = b->n_tiles;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return FSB_OK;
}

// Schedule of a grid of `waves` wavefronts: the static chunk size, or the
// chunk table of the dynamic and guided schedules (synchronises when it
// uploads one).
int set_schedule(fsb_batch* b, uint32_t waves) {
    const fsb_tuning& tu = b->tuning;
    if (tu.schedule == FSB_SCHED_STATIC) {
        b->args.n_chunks = 0;
        b->args.static_chunk =
            tu.chunk_tiles ? tu.chunk_tiles : (b->n_tiles + waves - 1) / waves;
        if (b->args.static_chunk == 0) b->args.static_chunk = 1;
        return FSB_OK;
    }
    if (b->chunk_sched == tu.schedule && b->chunk_tiles == tu.chunk_tiles &&
        b->chunk_waves == waves && b->chunk_fpl == b->table_fpl)
        return FSB_OK;
    std::vector<uint32_t> start;
    build_chunk_starts(b->n_tiles, tu.schedule, tu.chunk_tiles, waves, start);
    if (start.size() > (size_t)b->L.tile_cap + 1)
        return fail(FSB_ERR_INVALID_ARG, "chunk table exceeds its capacity");
    char* base = static_cast<char*>(b->ws);
    FSB_HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    FSB_HIP_TRY(hipMemcpy(base + b->L.chunks, start.data(), start.size() * 4, hipMemcpyHostToDevice),
                "chunk table upload");
    b->args.n_chunks = (uint32_t)(start.size() - 1);
    b->chunk_sched = tu.schedule;
    b->chunk_tiles = tu.chunk_tiles;
    b->chunk_waves = waves;
    b->chunk_fpl = b->table_fpl;
    return FSB_OK;
}

int grid_for(fsb_batch* b, const fsb_tuning& tu, uint32_t* grid) {
    const uint32_t naive = b->cfg.reduce_mode == FSB_REDUCE_NAIVE_F32;
    uint32_t g = 0;
    const fsb_tuning saved = b->tuning;
    b->tuning = tu;
    const uint32_t variant = batch_variant(b);
    b->tuning = saved;
    if (variant == kBatchDeep && !deep_capable(b->cfg))
        return fail(FSB_ERR_UNSUPPORTED,
                    "the deep variant needs compensated sums and no weighted swim rule");
    FSB_HIP_TRY(batch_resident_grid(tu.block_size, tu.fish_per_thread, naive, variant, &g),
                "occupancy query");
    if (tu.blocks_per_cu) {
        int dev = 0, cus = 0;
        FSB_HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
        FSB_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                    "hipDeviceGetAttribute");
        const uint64_t want = (uint64_t)cus * tu.blocks_per_cu;
        if (want < g) g = (uint32_t)want;
    }
    if (g == 0) return fail(FSB_ERR_UNSUPPORTED, "the batched kernel cannot be resident on this device");
    // no more blocks than there are tiles to share among their waves
    const uint64_t waves_per_block = tu.block_size / 64;
    const uint64_t useful = (b->n_tiles + waves_per_block - 1) / waves_per_block;
    if (useful < g) g = (uint32_t)(useful > 0 ? useful : 1);
    *grid = g;
    return FSB_OK;
}

BatchArgs launch_args(const fsb_batch* b, uint32_t steps, uint32_t grid) {
    BatchArgs a = b->args;
    a.steps = steps;
    a.spin_limit = barrier_spin_limit();
    // the deep variant's look-ahead skip test: plain swim, schools of at least
    // kBatchLookFish fish (in whole tiles of this shape)
    const uint32_t tile_fish = 64u * b->tuning.fish_per_thread;
    a.look_theta = batch_variant(b) == kBatchDeep && !(b->cfg.swim_rule & FSB_SWIM_GREEDY)
                       ? batch_look_theta()
                       : 0.0f;
    a.look_min_tiles = (uint32_t)((kBatchLookFish + tile_fish - 1) / tile_fish);
    return a;
}

int launch_once(fsb_batch* b, uint32_t steps, uint32_t grid) {
    const uint32_t naive = b->cfg.reduce_mode == FSB_REDUCE_NAIVE_F32;
    const uint32_t nt = b->total_fish * 16ull > (256ull << 20);
    const BatchArgs a = launch_args(b, steps, grid);
    hipError_t e = launch_batch(a, b->tuning.block_size, b->tuning.fish_per_thread, naive, nt,
                                batch_variant(b), grid, b->stream);
    if (e != hipSuccess) return persistent_launch_fail(e, "batched kernel launch");
    return FSB_OK;
}

// Capture [reset, persistent launch of `steps` iterations] once per shape.
int ensure_graph(fsb_batch* b, uint32_t steps, uint32_t grid) {
    if (b->graph && b->graph_steps == steps && b->graph_grid == grid &&
        b->graph_block == b->tuning.block_size && b->graph_fpl == b->tuning.fish_per_thread &&
        b->graph_variant == batch_variant(b) && b->graph_sched == b->tuning.schedule &&
        b->graph_chunks == b->args.n_chunks && b->graph_static == b->args.static_chunk)
        return FSB_OK;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    if (!b->capture) FSB_HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "hipStreamCreate");
    const uint32_t naive = b->cfg.reduce_mode == FSB_REDUCE_NAIVE_F32;
    const uint32_t nt = b->total_fish * 16ull > (256ull << 20);
    const BatchArgs a = launch_args(b, steps, grid);
    FSB_HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = launch_batch(a, b->tuning.block_size, b->tuning.fish_per_thread, naive, nt,
                                batch_variant(b), grid, b->capture);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e != hipSuccess ? e : e2, "graph capture of the batched launch");
    }
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph_steps = steps;
    b->graph_grid = grid;
    b->graph_block = b->tuning.block_size;
    b->graph_fpl = b->tuning.fish_per_thread;
    b->graph_variant = batch_variant(b);
    b->graph_sched = b->tuning.schedule;
    b->graph_chunks = b->args.n_chunks;
    b->graph_static = b->args.static_chunk;
    return FSB_OK;
}

template <class F>
int timed(fsb_batch* b, const char* what, F&& fn) {
    std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
    if (b->profile_every && b->launches++ % b->profile_every == 0) {
        FSB_HIP_TRY(b->timer.next(&ev), "hipEventCreate");
        FSB_HIP_TRY(hipEventRecord(ev->first, b->stream), "hipEventRecord");
    }
    int rc = fn();
    if (rc) return rc;
    if (ev) FSB_HIP_TRY(hipEventRecord(ev->second, b->stream), "hipEventRecord");
    (void)what;
    return FSB_OK;
}

int run(fsb_batch* b, uint64_t n_steps) {
    if (n_steps == 0) return FSB_OK;
    if (n_steps > kStepLimit - b->t) return fail(FSB_ERR_INVALID_ARG, "iteration index would pass 2^32");
    int rc = upload_tiles(b, b->tuning.fish_per_thread);
    if (rc) return rc;
    uint32_t grid = 0;
    rc = grid_for(b, b->tuning, &grid);
    if (rc) return rc;
    rc = set_schedule(b, grid * (b->tuning.block_size / 64));
    if (rc) return rc;
    const uint64_t K = b->tuning.steps_per_launch < n_steps ? b->tuning.steps_per_launch : n_steps;
    const uint64_t full = n_steps / K, rest = n_steps % K;
    if (full) {
        rc = ensure_graph(b, (uint32_t)K, grid);
        if (rc) return rc;
        for (uint64_t i = 0; i < full; ++i) {
            rc = timed(b, "graph launch", [&] {
                hipError_t e = hipGraphLaunch(b->graph, b->stream);
                return e == hipSuccess ? FSB_OK : hip_fail(e, "hipGraphLaunch");
            });
            if (rc) return rc;
        }
    }
    if (rest) {
        rc = timed(b, "batched launch", [&] { return launch_once(b, (uint32_t)rest, grid); });
        if (rc) return rc;
    }
    b->t += n_steps;
    b->has_result = true;
    return FSB_OK;
}

int check_error(fsb_batch* b) {
    uint32_t err = 0;
    FSB_HIP_TRY(hipMemcpyDtoHAsync(&err, reinterpret_cast<hipDeviceptr_t>(&b->args.ctrl->error),
                                   sizeof(err), b->stream),
                "hipMemcpyDtoHAsync");
    FSB_HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    if (err & kErrBarrierTimeout) return fail(FSB_ERR_DEVICE, "a persistent kernel's grid barrier timed out");
    if (err) return fail(FSB_ERR_DEVICE, "kernel error flags " + std::to_string(err));
    return FSB_OK;
}

int read_records(fsb_batch* b, uint64_t step, std::vector<fsb_record>& out) {
    out.resize(b->n);
    const fsb_record* src = b->args.rec + (size_t)(step % b->cfg.history_len) * b->n;
    FSB_HIP_TRY(hipMemcpyDtoHAsync(out.data(), reinterpret_cast<hipDeviceptr_t>(const_cast<fsb_record*>(src)),
                                   out.size() * sizeof(fsb_record), b->stream),
                "hipMemcpyDtoHAsync");
    int rc = check_error(b);
    if (rc) return rc;
    for (uint32_t s = 0; s < b->n; ++s)
        if (out[s].step_lo != (uint32_t)step)
            return fail(FSB_ERR_STATE, "record ring slot holds another iteration");
    return FSB_OK;
}

// ---- autotune cache --------------------------------------------------------

std::string cache_key(const fsb_batch* b) {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the school sizes
    for (uint32_t s = 0; s < b->n; ++s) {
        h ^= b->size[s];
        h *= 1099511628211ull;
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|%u|%" PRIu64 "|%016" PRIx64 "|%u", arch.c_str(), b->n,
                  b->total_fish, h, b->cfg.reduce_mode);
    return buf;
}

bool cache_lookup(const std::string& key, fsb_tuning* out) {
    const char* path = std::getenv("FSB_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        fsb_tuning t;
        if (parse_cache_line(line, key, &t)) {  // the last matching line wins
            *out = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string& key, const fsb_tuning& t) {
    const char* path = std::getenv("FSB_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fputs(format_cache_line(key, t).c_str(), f);
    std::fclose(f);
}

// Time `steps` iterations with tuning `tu` (one warm launch of 1 iteration
// first, so table upload and graph capture are not timed).
int probe(fsb_batch* b, const fsb_tuning& tu, uint64_t steps, double* ms_per_step) {
    b->tuning = tu;
    int rc = run(b, 1);
    if (rc) return rc;
    hipEvent_t e0, e1;
    FSB_HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    rc = FSB_OK;
    if ((e = hipEventRecord(e0, b->stream)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
    if (!rc) rc = run(b, steps);
    if (!rc && (e = hipEventRecord(e1, b->stream)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
    if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    if (!rc && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) rc = check_error(b);
    *ms_per_step = ms / (double)steps;
    return rc;
}

}  // namespace

extern "C" {

int fsb_batch_workspace_bytes(const fsb_config* common, uint32_t n_schools, const uint64_t* starts,
                              const uint64_t* sizes, size_t* out_bytes) {
    int rc = check_config(common, false);
    if (rc) return rc;
    if (!out_bytes) return fail(FSB_ERR_INVALID_ARG, "out_bytes is NULL");
    uint64_t cap = 0, total = 0;
    rc = check_schools(n_schools, starts, sizes, &cap, &total);
    if (rc) return rc;
    *out_bytes = batch_layout(n_schools, cap, common->history_len, deep_capable(*common)).total;
    return FSB_OK;
}

int fsb_batch_init(const fsb_config* common, uint32_t n_schools, const uint64_t* starts,
                   const uint64_t* sizes, const uint64_t* seeds, fsb_state packed,
                   uint64_t packed_len, void* workspace, size_t workspace_bytes, void* stream,
                   fsb_batch** out) {
    int rc = check_config(common, false);
    if (rc) return rc;
    if (common->reduce_mode == FSB_REDUCE_CRITICAL_F32)
        return fail(FSB_ERR_UNSUPPORTED, "the critical reduction is a plain-path ablation only");
    if (!out) return fail(FSB_ERR_INVALID_ARG, "out is NULL");
    if (!seeds) return fail(FSB_ERR_INVALID_ARG, "seeds is NULL");
    uint64_t cap = 0, total = 0;
    rc = check_schools(n_schools, starts, sizes, &cap, &total);
    if (rc) return rc;
    const uint64_t end = starts[n_schools - 1] + sizes[n_schools - 1];
    if (packed_len < end) return fail(FSB_ERR_INVALID_ARG, "packed columns are shorter than the last school");
    rc = check_columns(packed, packed_len);
    if (rc) return rc;
    const BatchLayout L = batch_layout(n_schools, cap, common->history_len, deep_capable(*common));
    rc = check_workspace(workspace, workspace_bytes, L.total);
    if (rc) return rc;

    fsb_batch* b = new (std::nothrow) fsb_batch();
    if (!b) return fail(FSB_ERR_INVALID_ARG, "out of host memory");
    b->cfg = *common;
    b->n = n_schools;
    b->start.assign(starts, starts + n_schools);
    b->size.assign(sizes, sizes + n_schools);
    b->seed.assign(seeds, seeds + n_schools);
    b->total_fish = total;
    b->st = packed;
    b->ws = workspace;
    b->ws_bytes = workspace_bytes;
    b->stream = static_cast<hipStream_t>(stream);
    b->L = L;
    b->tuning = fsb_tuning{deep_capable(*common) ? 256u : 1024u, 8, 100, 0, 0, FSB_SCHED_STATIC, 0};

    char* base = static_cast<char*>(workspace);
    BatchArgs& a = b->args;
    a = BatchArgs{};
    a.x = packed.x;
    a.y = packed.y;
    a.w = packed.w;
    a.prev = packed.prev;
    a.cur = packed.cur;
    a.tiles = reinterpret_cast<const Tile*>(base + L.tiles);
    a.tile_begin = reinterpret_cast<const uint32_t*>(base + L.tile_begin);
    a.n_schools = n_schools;
    a.H = common->pond_half;
    a.S = common->swim_step;
    a.wmin = common->w_min;
    a.wmax = common->w_max;
    a.wlo = common->w_init_lo;
    a.whi = common->w_init_hi;
    a.rule = common->swim_rule;
    a.ctrl = reinterpret_cast<Ctrl*>(base + L.ctrl);
    a.sync = reinterpret_cast<uint32_t*>(base + L.sync);
    a.step = &a.ctrl->step;
    a.school_max = reinterpret_cast<uint32_t*>(base + L.school_max);
    a.tile_part = reinterpret_cast<double*>(base + L.tile_part);
    a.tile_cap = L.tile_cap;
    a.max_slots = deep_capable(*common) ? 3 * kMaxDepth : 3;
    a.school_naive = reinterpret_cast<float*>(base + L.school_naive);
    a.rec = reinterpret_cast<fsb_record*>(base + L.rec);
    a.hist_len = common->history_len;
    a.chunk_start = reinterpret_cast<const uint32_t*>(base + L.chunks);
    a.queue = reinterpret_cast<uint32_t*>(base + L.queue);
    a.school_flag = reinterpret_cast<uint32_t*>(base + L.school_flag);

    auto cleanup = [&](int code) {
        delete b;
        return code;
    };
    rc = upload_tiles(b, b->tuning.fish_per_thread);
    if (rc) return cleanup(rc);
    SchoolArgs sa{};
    sa.ctrl = a.ctrl;
    hipError_t e = launch_reset(sa, b->stream);
    if (e == hipSuccess) e = launch_batch_init(a, 256, b->stream);
    if (e != hipSuccess) return cleanup(hip_fail(e, "batch init launch"));
    *out = b;
    return FSB_OK;
}

int fsb_batch_run(fsb_batch* b, uint64_t n_steps, const fsb_tuning* tuning) {
    if (!b) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (tuning) {
        int rc = check_tuning(tuning);
        if (rc) return rc;
        b->tuning = *tuning;
    }
    return run(b, n_steps);
}

int fsb_batch_results(fsb_batch* b, double* out_xy, double* out_sums, float* out_max) {
    if (!b) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (!b->has_result) return fail(FSB_ERR_STATE, "no iteration has completed");
    std::vector<fsb_record> r;
    int rc = read_records(b, b->t - 1, r);
    if (rc) return rc;
    for (uint32_t s = 0; s < b->n; ++s) {
        if (out_xy) {
            out_xy[2 * s] = r[s].sum_wx / r[s].sum_w;
            out_xy[2 * s + 1] = r[s].sum_wy / r[s].sum_w;
        }
        if (out_sums) {
            out_sums[3 * s] = r[s].sum_w;
            out_sums[3 * s + 1] = r[s].sum_wx;
            out_sums[3 * s + 2] = r[s].sum_wy;
        }
        if (out_max) out_max[s] = r[s].max_delta;
    }
    return FSB_OK;
}

int fsb_batch_barycentre(fsb_batch* b, double* out_xy, double* out_sums) {
    if (!b) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (!out_xy) return fail(FSB_ERR_INVALID_ARG, "out_xy is NULL");
    return fsb_batch_results(b, out_xy, out_sums, nullptr);
}

int fsb_batch_history(fsb_batch* b, uint64_t step, fsb_record* out) {
    if (!b || !out) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    if (step >= b->t || b->t - step > b->cfg.history_len)
        return fail(FSB_ERR_INVALID_ARG, "iteration is not in the record ring");
    std::vector<fsb_record> r;
    int rc = read_records(b, step, r);
    if (rc) return rc;
    std::memcpy(out, r.data(), r.size() * sizeof(fsb_record));
    return FSB_OK;
}

int fsb_autotune(fsb_batch* b, uint64_t probe_steps, fsb_tuning* out) {
    if (!b || !out) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    if (probe_steps == 0) return fail(FSB_ERR_INVALID_ARG, "probe_steps must be >= 1");
    const std::string key = cache_key(b);
    fsb_tuning best;
    if (cache_lookup(key, &best)) {
        b->tuning = best;
        *out = best;
        return FSB_OK;
    }
    double best_ms = 1e300;
    best = b->tuning;
    // shapes with the variant the library would pick, then the other variant
    const uint32_t lib_variant =
        b->total_fish * 16ull >= (256ull << 20) ? FSB_RUN_FUSED_LEAN : FSB_RUN_FUSED_PREV;
    for (uint32_t block : kBatchBlocks)
        for (uint32_t fpl : kBatchFishPerLane) {
            fsb_tuning tu{block, fpl, (uint32_t)probe_steps, 0, lib_variant, FSB_SCHED_STATIC, 0};
            double ms = 0.0;
            int rc = probe(b, tu, probe_steps, &ms);
            if (rc == FSB_ERR_UNSUPPORTED) continue;
            if (rc) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best = tu;
            }
        }
    {
        fsb_tuning tu = best;
        tu.variant = lib_variant == FSB_RUN_FUSED_LEAN ? FSB_RUN_FUSED_PREV : FSB_RUN_FUSED_LEAN;
        double ms = 0.0;
        int rc = probe(b, tu, probe_steps, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = tu;
        }
    }
    // the deep variant (256-thread blocks), where it can run
    if (deep_capable(b->cfg))
        for (uint32_t fpl : kBatchFishPerLane) {
            fsb_tuning tu{256, fpl, (uint32_t)probe_steps, 0, FSB_RUN_FUSED_DEEP, FSB_SCHED_STATIC, 0};
            double ms = 0.0;
            int rc = probe(b, tu, probe_steps, &ms);
            if (rc == FSB_ERR_UNSUPPORTED) continue;
            if (rc) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best = tu;
            }
        }
    // work-queue schedules against the static one (one tile per chunk is
    // left out: at CFG5 scale its one atomic per tile saturates the counter)
    const fsb_tuning queues[5] = {{0, 0, 0, 0, 0, FSB_SCHED_DYNAMIC, 4},
                                  {0, 0, 0, 0, 0, FSB_SCHED_DYNAMIC, 8},
                                  {0, 0, 0, 0, 0, FSB_SCHED_DYNAMIC, 16},
                                  {0, 0, 0, 0, 0, FSB_SCHED_DYNAMIC, 64},
                                  {0, 0, 0, 0, 0, FSB_SCHED_GUIDED, 4}};
    const fsb_tuning shape = best;
    for (const fsb_tuning& q : queues) {
        fsb_tuning tu = shape;
        tu.schedule = q.schedule;
        tu.chunk_tiles = q.chunk_tiles;
        double ms = 0.0;
        int rc = probe(b, tu, probe_steps, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = tu;
        }
    }
    // iterations per launch for the best shape: short launches against one
    // launch of probe_steps (each launch re-reads the state once more in its
    // prologue and pays one graph launch)
    const uint64_t shorter[2] = {probe_steps / 8, probe_steps / 2};
    for (uint64_t k : shorter) {
        if (k == 0 || k == probe_steps) continue;
        fsb_tuning tu = best;
        tu.steps_per_launch = (uint32_t)k;
        double ms = 0.0;
        int rc = probe(b, tu, probe_steps, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = tu;
        }
    }
    // a chosen single launch covers runs of any length with the same shape
    if (best.steps_per_launch == probe_steps && probe_steps < 1000) best.steps_per_launch = 1000;
    b->tuning = best;
    cache_store(key, best);
    *out = best;
    return FSB_OK;
}

int fsb_batch_get_tuning(const fsb_batch* b, fsb_tuning* out) {
    if (!b || !out) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    *out = b->tuning;
    return FSB_OK;
}

int fsb_batch_step_index(const fsb_batch* b, uint64_t* out_t) {
    if (!b || !out_t) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    *out_t = b->t;
    return FSB_OK;
}

int fsb_batch_sync(fsb_batch* b) {
    if (!b) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    return check_error(b);
}

int fsb_batch_destroy(fsb_batch* b) {
    if (!b) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    // The graph exec, the capture stream and the timer's events are released
    // only once the handle's stream has drained: a replay still in flight
    // reads the exec's kernel arguments, and the timer's events are still to
    // be recorded.  The handle is freed even if the stream reports an error.
    const hipError_t e = hipStreamSynchronize(b->stream);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize before destroying the batch");
    return FSB_OK;
}

int fsb_batch_profile_enable(fsb_batch* b, int every) {
    if (!b) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (every < 0) return fail(FSB_ERR_INVALID_ARG, "every must be >= 0");
    b->profile_every = (uint32_t)every;
    b->launches = 0;
    return FSB_OK;
}

int fsb_batch_kernel_times(fsb_batch* b, uint64_t* count, double* ms) {
    if (!b || !count || !ms) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    FSB_HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    *count = b->timer.used;
    FSB_HIP_TRY(b->timer.total(ms), "hipEventElapsedTime");
    b->timer.used = 0;
    return FSB_OK;
}

}  // extern "C"
