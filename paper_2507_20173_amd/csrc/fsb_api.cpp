// fsb_api.cpp -- the C ABI of libfsb (declared in include/fsb.h): argument
// checks, handles, launch sequencing, result read-back, kernel timing.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "fsb.h"
#include "fsb_host.hpp"
#include "fsb_internal.hpp"
#include "fsb_probe.hpp"

using namespace fsb;

struct fsb_school {
    fsb_config cfg;
    fsb_state st;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    Layout L;
    SchoolArgs args;
    uint64_t t;            // next iteration
    uint64_t first_valid;  // first iteration whose record this handle wrote
    bool has_result;       // an iteration completed since init/attach/set
    bool pending;          // last feed pass's partials not yet combined
    uint32_t pending_t;
    uint32_t pending_grid;
    uint32_t profile_every;  // time every n-th launch of each kind (0 = off)
    uint64_t launches[FSB_KERNEL_KINDS];
    uint32_t resident[2];  // co-resident grid of the persistent kernel (per reduce mode; 0 = unknown)
    uint32_t resident_regs[2];  // the same for the register-resident kernel
    uint32_t resident_deep[3];  // the same for the deep kernel of depth 2, 4, 8 (compensated sums only)
    Timer timers[FSB_KERNEL_KINDS];
};

namespace {

// Launch `fn` bracketed by the kind's events when profiling is on.
template <class F>
int timed(fsb_school* h, int kind, const char* what, F&& fn) {
    std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
    if (h->profile_every && h->launches[kind]++ % h->profile_every == 0) {
        FSB_HIP_TRY(h->timers[kind].next(&ev), "hipEventCreate");
        FSB_HIP_TRY(hipEventRecord(ev->first, h->stream), "hipEventRecord");
    }
    FSB_HIP_TRY(fn(), what);
    if (ev) FSB_HIP_TRY(hipEventRecord(ev->second, h->stream), "hipEventRecord");
    return FSB_OK;
}

// The same for a launch that records the events itself (the plain passes):
// fn(start, stop) gets the kind's next pair, or two nulls when this launch is
// not timed.
template <class F>
int timed_by_launch(fsb_school* h, int kind, const char* what, F&& fn) {
    std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
    if (h->profile_every && h->launches[kind]++ % h->profile_every == 0)
        FSB_HIP_TRY(h->timers[kind].next(&ev), "hipEventCreate");
    FSB_HIP_TRY(fn(ev ? ev->first : nullptr, ev ? ev->second : nullptr), what);
    return FSB_OK;
}

SchoolArgs make_args(const fsb_config& c, const fsb_state& st, void* ws, const Layout& L) {
    SchoolArgs a{};
    char* base = static_cast<char*>(ws);
    a.x = st.x;
    a.y = st.y;
    a.w = st.w;
    a.prev = st.prev;
    a.cur = st.cur;
    a.n = c.n_fish;
    a.k0 = (uint32_t)c.seed;
    a.k1 = (uint32_t)(c.seed >> 32);
    a.H = c.pond_half;
    a.S = c.swim_step;
    a.wmin = c.w_min;
    a.wmax = c.w_max;
    a.rule = c.swim_rule;
    a.ctrl = reinterpret_cast<Ctrl*>(base + L.ctrl);
    a.hist = reinterpret_cast<fsb_record*>(base + L.hist);
    a.hist_len = c.history_len;
    a.blockmax = reinterpret_cast<uint32_t*>(base + L.blockmax);
    a.partials = reinterpret_cast<double*>(base + L.partials);
    a.deep = reinterpret_cast<double*>(base + L.deep);
    a.sync = reinterpret_cast<uint32_t*>(base + L.sync);
    return a;
}

// A handle's fields for a school whose arguments have been checked (no
// allocation: the handle may live on the caller's stack).
void fill_school(fsb_school* h, const fsb_config& cfg, const fsb_state& state, void* ws,
                 size_t ws_bytes, void* stream, const Layout& L, uint64_t t) {
    h->cfg = cfg;
    h->st = state;
    h->ws = ws;
    h->ws_bytes = ws_bytes;
    h->stream = static_cast<hipStream_t>(stream);
    h->L = L;
    h->args = make_args(cfg, state, ws, L);
    h->t = t;
    h->first_valid = t;
    h->has_result = false;
    h->pending = false;
    h->profile_every = 0;
}

int new_school(const fsb_config* cfg, fsb_state state, void* ws, size_t ws_bytes, void* stream,
               uint64_t t, fsb_school** out) {
    int rc = check_config(cfg, true);
    if (rc) return rc;
    if (!out) return fail(FSB_ERR_INVALID_ARG, "out is NULL");
    rc = check_columns(state, cfg->n_fish);
    if (rc) return rc;
    const Layout L = school_layout(cfg->history_len);
    rc = check_workspace(ws, ws_bytes, L.total);
    if (rc) return rc;
    if (t >= kStepLimit) return fail(FSB_ERR_INVALID_ARG, "iteration index must be < 2^32");
    fsb_school* h = new (std::nothrow) fsb_school();
    if (!h) return fail(FSB_ERR_INVALID_ARG, "out of host memory");
    fill_school(h, *cfg, state, ws, ws_bytes, stream, L, t);
    hipError_t e = launch_reset(h->args, h->stream);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "reset launch");
    }
    *out = h;
    return FSB_OK;
}

// Write the pending record (iteration pending_t) with a one-block launch.
int finish_pending(fsb_school* h) {
    if (!h->pending) return FSB_OK;
    const uint32_t naive = h->cfg.reduce_mode != FSB_REDUCE_COMPENSATED;
    FSB_HIP_TRY(launch_combine(h->args, h->pending_t, h->pending_grid, naive, h->stream),
                "combine launch");
    h->pending = false;
    return FSB_OK;
}

int check_device_error(fsb_school* h) {
    uint32_t err = 0;
    FSB_HIP_TRY(hipMemcpyDtoHAsync(&err, reinterpret_cast<hipDeviceptr_t>(&h->args.ctrl->error),
                                   sizeof(err), h->stream),
                "hipMemcpyDtoHAsync");
    FSB_HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (err & kErrBarrierTimeout)
        return fail(FSB_ERR_DEVICE, "a persistent kernel's grid barrier timed out");
    if (err) return fail(FSB_ERR_DEVICE, "kernel error flags " + std::to_string(err));
    return FSB_OK;
}

int do_step(fsb_school* h, const float* dx, const float* dy) {
    if (h->t >= kStepLimit) return fail(FSB_ERR_INVALID_ARG, "iteration index reached 2^32");
    StepArgs s{};
    s.t = (uint32_t)h->t;
    s.swim_grid = plain_grid(h->cfg.n_fish);
    s.combine = h->pending ? 1u : 0u;
    s.prev_t = h->pending_t;
    s.prev_grid = h->pending_grid;
    s.naive = h->cfg.reduce_mode != FSB_REDUCE_COMPENSATED;
    s.critical = h->cfg.reduce_mode == FSB_REDUCE_CRITICAL_F32;
    s.dx = dx;
    s.dy = dy;
    int rc = timed_by_launch(h, FSB_KERNEL_SWIM_EVAL, "swim pass launch",
                             [&](hipEvent_t e0, hipEvent_t e1) {
                                 return launch_swim_eval(h->args, s, h->stream, e0, e1);
                             });
    if (rc) return rc;
    h->pending = false;
    const uint32_t fgrid = feed_grid(h->cfg.n_fish);
    s.combine = 0u;  // the swim pass wrote the pending record
    rc = timed_by_launch(h, FSB_KERNEL_FEED_BARY, "feed pass launch",
                         [&](hipEvent_t e0, hipEvent_t e1) {
                             return launch_feed_bary(h->args, s, fgrid, h->stream, e0, e1);
                         });
    if (rc) return rc;
    h->pending = true;
    h->pending_t = (uint32_t)h->t;
    h->pending_grid = fgrid;
    h->t += 1;
    h->has_result = true;
    return FSB_OK;
}

// FSB_RUN_PLAIN over n_steps >= 2 iterations, one launch per iteration: the
// swim pass of the first, then for each next iteration t the pipelined pass
// (feed of t - 1, swim of t), then the feed pass of the last, which also
// stores cur.  Every launch first writes the record its predecessor left
// pending.  The critical ablation keeps fsb_step's two passes.
int run_plain(fsb_school* h, uint64_t n_steps) {
    if (n_steps < 2 || h->cfg.reduce_mode == FSB_REDUCE_CRITICAL_F32) {
        for (uint64_t k = 0; k < n_steps; ++k) {
            int rc = do_step(h, nullptr, nullptr);
            if (rc) return rc;
        }
        return FSB_OK;
    }
    const uint64_t n = h->cfg.n_fish;
    StepArgs s{};
    s.naive = h->cfg.reduce_mode != FSB_REDUCE_COMPENSATED;
    auto pending_into = [&](StepArgs& a) {
        a.combine = h->pending ? 1u : 0u;
        a.prev_t = h->pending_t;
        a.prev_grid = h->pending_grid;
    };
    const uint64_t t0 = h->t;
    s.t = (uint32_t)t0;
    s.swim_grid = plain_grid(n);
    pending_into(s);
    int rc = timed_by_launch(h, FSB_KERNEL_SWIM_EVAL, "swim pass launch",
                             [&](hipEvent_t e0, hipEvent_t e1) {
                                 return launch_swim_eval(h->args, s, h->stream, e0, e1);
                             });
    if (rc) return rc;
    h->pending = false;
    h->has_result = true;
    uint32_t swum_by = s.swim_grid;  // grid whose block maxima the next launch reads
    const uint32_t pgrid = pipe_grid(n);
    for (uint64_t k = 1; k < n_steps; ++k) {
        s.t = (uint32_t)(t0 + k);
        s.swim_grid = swum_by;
        pending_into(s);
        rc = timed_by_launch(h, FSB_KERNEL_FEED_SWIM, "pipelined pass launch",
                             [&](hipEvent_t e0, hipEvent_t e1) {
                                 return launch_feed_swim(h->args, s, pgrid, h->stream, e0, e1);
                             });
        if (rc) return rc;
        h->pending = true;
        h->pending_t = (uint32_t)(t0 + k - 1);
        h->pending_grid = pgrid;
        swum_by = pgrid;
    }
    s.t = (uint32_t)(t0 + n_steps - 1);
    s.swim_grid = swum_by;
    pending_into(s);
    const uint32_t fgrid = feed_grid(n);
    rc = timed_by_launch(h, FSB_KERNEL_FEED_BARY, "feed pass launch",
                         [&](hipEvent_t e0, hipEvent_t e1) {
                             return launch_feed_bary(h->args, s, fgrid, h->stream, e0, e1, true);
                         });
    if (rc) return rc;
    h->pending = true;
    h->pending_t = s.t;
    h->pending_grid = fgrid;
    h->t = t0 + n_steps;
    return FSB_OK;
}

// FSB_RUN_FUSED without the deep kernel (naive sums or the weighted rule) on
// a school too large for registers: the lean variant trades a second swim per fish for a
// quarter less traffic.  Measured on MI355X it wins once the 32-byte
// variant's live columns (16 B/fish) no longer fit the 256 MiB last-level
// cache with room to spare (N >= 2^24); below that the cache feeds both and
// the extra arithmetic costs more than the saved bytes.
bool lean_pays(uint64_t n) { return n * 16ull >= (256ull << 20); }

// n_steps iterations in one persistent launch (cooperative, so the grid is
// guaranteed co-resident or the launch fails).
int run_fused(fsb_school* h, uint64_t n_steps, uint32_t mode) {
    if (n_steps == 0) return FSB_OK;
    if (h->cfg.reduce_mode == FSB_REDUCE_CRITICAL_F32)
        return fail(FSB_ERR_UNSUPPORTED, "the critical reduction is a plain-path ablation only");
    const uint32_t naive = h->cfg.reduce_mode == FSB_REDUCE_NAIVE_F32;
    if (h->resident[naive] == 0)
        FSB_HIP_TRY(fused_resident_grid(naive, &h->resident[naive]), "occupancy query");
    if (h->resident[naive] == 0)
        return fail(FSB_ERR_UNSUPPORTED, "the persistent kernel cannot be resident on this device");
    // FSB_RUN_FUSED takes the deep kernel whenever it can run (compensated sums,
    // no weighted rule): measured on MI355X it is the fastest persistent form at
    // every size from 2^10 to 2^26 fish (3.9 us per iteration at 2^16 against
    // 5.6 for registers; 205 us at 2^26 against 332 for lean).  Otherwise the
    // register-resident kernel for a school it holds (1.4-1.6x faster than the
    // streaming variants from 2^12 to 2^21 fish), else lean or store-prev.
    const bool deep_ok = !naive && !(h->cfg.swim_rule & FSB_SWIM_WEIGHTED);
    if (mode == FSB_RUN_FUSED && deep_ok) mode = FSB_RUN_FUSED_DEEP;
    uint32_t groups = 0, grid = 0;
    if (mode == FSB_RUN_FUSED_REGS || mode == FSB_RUN_FUSED) {
        if (h->resident_regs[naive] == 0)
            FSB_HIP_TRY(regs_resident_grid(naive, &h->resident_regs[naive]), "occupancy query");
        grid = regs_plan(h->cfg.n_fish, h->resident_regs[naive], &groups);
        if (groups == 0 && mode == FSB_RUN_FUSED_REGS)
            return fail(FSB_ERR_UNSUPPORTED, "school too large to be held in registers (" +
                                                 std::to_string(h->cfg.n_fish) + " fish)");
    }
    // The deep kernel, if asked for.
    uint32_t depth = 0;
    if (mode == FSB_RUN_FUSED_DEEP) {
        if (!deep_ok)
            return fail(FSB_ERR_UNSUPPORTED,
                        "the deep kernel needs compensated sums and positions that do not depend "
                        "on weights (no weighted swim rule)");
        depth = deep_depth(h->cfg.n_fish);
        uint32_t& resident = h->resident_deep[depth == 2 ? 0 : depth == 4 ? 1 : 2];
        if (resident == 0) FSB_HIP_TRY(deep_resident_grid(depth, &resident), "occupancy query");
        if (resident == 0)
            return fail(FSB_ERR_UNSUPPORTED, "the deep kernel cannot be resident on this device");
        grid = deep_grid(h->cfg.n_fish, depth, resident);
    }
    int rc = finish_pending(h);
    if (rc) return rc;
    if (groups == 0 && depth == 0) grid = fused_grid(h->cfg.n_fish, h->resident[naive]);
    FusedArgs f{};
    f.regs = groups;
    f.deep = depth;
    f.look_theta = depth ? look_theta(h->cfg.n_fish) : 0.0f;
    f.t0 = (uint32_t)h->t;
    f.steps = (uint32_t)n_steps;
    f.naive = naive;
    f.spin_limit = barrier_spin_limit();
    // Non-temporal streaming once the four live columns outgrow the 256 MB
    // last-level cache (below that, keeping lines cached is faster).
    f.streaming = h->cfg.n_fish * 16ull > (256ull << 20);
    f.lean = mode == FSB_RUN_FUSED_LEAN || (mode == FSB_RUN_FUSED && lean_pays(h->cfg.n_fish));
    std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
    if (h->profile_every && h->launches[FSB_KERNEL_FUSED]++ % h->profile_every == 0) {
        FSB_HIP_TRY(h->timers[FSB_KERNEL_FUSED].next(&ev), "hipEventCreate");
        FSB_HIP_TRY(hipEventRecord(ev->first, h->stream), "hipEventRecord");
    }
    hipError_t e = launch_fused(h->args, f, grid, h->stream);
    if (e != hipSuccess) return persistent_launch_fail(e, "persistent kernel launch");
    if (ev) FSB_HIP_TRY(hipEventRecord(ev->second, h->stream), "hipEventRecord");
    // The deep kernel writes every record itself; the others leave the last
    // iteration's partials for a combine launch.
    h->pending = depth == 0;
    h->pending_t = (uint32_t)(h->t + n_steps - 1);
    h->pending_grid = grid;
    h->t += n_steps;
    h->has_result = true;
    return FSB_OK;
}

int read_record(fsb_school* h, uint64_t step, fsb_record* r) {
    const fsb_record* src = h->args.hist + (step % h->cfg.history_len);
    FSB_HIP_TRY(hipMemcpyDtoHAsync(r, reinterpret_cast<hipDeviceptr_t>(const_cast<fsb_record*>(src)),
                                   sizeof(*r), h->stream),
                "hipMemcpyDtoHAsync");
    return FSB_OK;
}

}  // namespace

extern "C" {

const char* fsb_strerror(int code) {
    switch (code) {
        case FSB_OK: return "ok";
        case FSB_ERR_INVALID_ARG: return "invalid argument";
        case FSB_ERR_HIP: return "HIP runtime error";
        case FSB_ERR_UNSUPPORTED: return "unsupported configuration";
        case FSB_ERR_STATE: return "call not valid in the current state";
        case FSB_ERR_DEVICE: return "a kernel reported a failure";
        default: return "unknown error code";
    }
}

const char* fsb_last_error(void) { return last_error().c_str(); }

int fsb_abi_version(void) { return FSB_ABI_VERSION; }

int fsb_workspace_bytes(const fsb_config* cfg, size_t* out_bytes) {
    int rc = check_config(cfg, false);
    if (rc) return rc;
    if (!out_bytes) return fail(FSB_ERR_INVALID_ARG, "out_bytes is NULL");
    *out_bytes = school_layout(cfg->history_len).total;
    return FSB_OK;
}

int fsb_init(const fsb_config* cfg, fsb_state state, void* workspace, size_t workspace_bytes,
             void* stream, fsb_school** out) {
    fsb_school* h = nullptr;
    int rc = new_school(cfg, state, workspace, workspace_bytes, stream, 0, &h);
    if (rc) return rc;
    rc = timed(h, FSB_KERNEL_INIT, "init launch", [&] {
        return launch_init(h->args, cfg->w_init_lo, cfg->w_init_hi, h->stream);
    });
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return FSB_OK;
}

int fsb_attach(const fsb_config* cfg, fsb_state state, void* workspace, size_t workspace_bytes,
               void* stream, uint64_t t, fsb_school** out) {
    return new_school(cfg, state, workspace, workspace_bytes, stream, t, out);
}

int fsb_step(fsb_school* h) {
    if (!h) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    return do_step(h, nullptr, nullptr);
}

int fsb_step_displaced(fsb_school* h, const float* dx, const float* dy) {
    if (!h) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (!dx || !dy) return fail(FSB_ERR_INVALID_ARG, "displacement arrays must not be NULL");
    if (!aligned(dx, 16) || !aligned(dy, 16))
        return fail(FSB_ERR_INVALID_ARG, "displacement arrays must be 16-byte aligned");
    return do_step(h, dx, dy);
}

int fsb_run(fsb_school* h, uint64_t n_steps, uint32_t mode) {
    if (!h) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (mode > FSB_RUN_PLAIN_SPLIT) return fail(FSB_ERR_INVALID_ARG, "unknown run mode");
    if (n_steps > kStepLimit - h->t) return fail(FSB_ERR_INVALID_ARG, "iteration index would pass 2^32");
    if (mode == FSB_RUN_PLAIN) return run_plain(h, n_steps);
    if (mode != FSB_RUN_PLAIN_SPLIT) return run_fused(h, n_steps, mode);
    for (uint64_t k = 0; k < n_steps; ++k) {
        int rc = do_step(h, nullptr, nullptr);
        if (rc) return rc;
    }
    return FSB_OK;
}

int fsb_barycentre(fsb_school* h, double out_xy[2], double* out_sums3) {
    if (!h || !out_xy) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    if (!h->has_result) return fail(FSB_ERR_STATE, "no iteration has completed");
    int rc = finish_pending(h);
    if (rc) return rc;
    fsb_record r;
    rc = read_record(h, h->t - 1, &r);
    if (rc) return rc;
    rc = check_device_error(h);
    if (rc) return rc;
    out_xy[0] = r.sum_wx / r.sum_w;
    out_xy[1] = r.sum_wy / r.sum_w;
    if (out_sums3) {
        out_sums3[0] = r.sum_w;
        out_sums3[1] = r.sum_wx;
        out_sums3[2] = r.sum_wy;
    }
    return FSB_OK;
}

int fsb_max_delta(fsb_school* h, float* out_max) {
    if (!h || !out_max) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    if (!h->has_result) return fail(FSB_ERR_STATE, "no iteration has completed");
    int rc = finish_pending(h);
    if (rc) return rc;
    fsb_record r;
    rc = read_record(h, h->t - 1, &r);
    if (rc) return rc;
    rc = check_device_error(h);
    if (rc) return rc;
    *out_max = r.max_delta;
    return FSB_OK;
}

int fsb_history(fsb_school* h, uint64_t first, uint64_t count, fsb_record* out) {
    if (!h || (!out && count)) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    const uint64_t lo = h->t > h->cfg.history_len ? h->t - h->cfg.history_len : 0;
    const uint64_t oldest = lo > h->first_valid ? lo : h->first_valid;
    if (first < oldest || first > h->t || count > h->t - first)
        return fail(FSB_ERR_INVALID_ARG, "requested iterations are not in the record ring");
    int rc = finish_pending(h);
    if (rc) return rc;
    for (uint64_t k = 0; k < count; ++k) {
        rc = read_record(h, first + k, out + k);
        if (rc) return rc;
    }
    rc = check_device_error(h);
    if (rc) return rc;
    for (uint64_t k = 0; k < count; ++k)
        if (out[k].step_lo != (uint32_t)(first + k))
            return fail(FSB_ERR_STATE, "record ring slot holds another iteration");
    return FSB_OK;
}

int fsb_sync(fsb_school* h) {
    if (!h) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    int rc = finish_pending(h);
    if (rc) return rc;
    return check_device_error(h);
}

int fsb_step_index(const fsb_school* h, uint64_t* out_t) {
    if (!h || !out_t) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    *out_t = h->t;
    return FSB_OK;
}

int fsb_set_step_index(fsb_school* h, uint64_t t) {
    if (!h) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (t >= kStepLimit) return fail(FSB_ERR_INVALID_ARG, "iteration index must be < 2^32");
    int rc = finish_pending(h);
    if (rc) return rc;
    h->t = t;
    h->first_valid = t;
    h->has_result = false;
    return FSB_OK;
}

int fsb_destroy(fsb_school* h) {
    if (!h) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    // The timers' events are released only once the handle's stream has
    // drained (a timed launch may still be in flight); the handle is freed
    // even if the stream reports an error.
    const hipError_t e = hipStreamSynchronize(h->stream);
    delete h;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize before destroying the school");
    return FSB_OK;
}

int fsb_run_static(const fsb_config* cfg, fsb_state state, uint64_t t, uint64_t n_steps,
                   uint32_t mode, fsb_record* records, uint32_t* status, void* stream) {
    // Every check comes before the first HIP call.
    int rc = check_config(cfg, true);
    if (rc) return rc;
    rc = check_columns(state, cfg->n_fish);
    if (rc) return rc;
    if (!records) return fail(FSB_ERR_INVALID_ARG, "records is NULL");
    if (!aligned(records, alignof(fsb_record)))
        return fail(FSB_ERR_INVALID_ARG, "records is not 8-byte aligned");
    if (status && !aligned(status, 4)) return fail(FSB_ERR_INVALID_ARG, "status is not 4-byte aligned");
    if (mode > FSB_RUN_PLAIN_SPLIT) return fail(FSB_ERR_INVALID_ARG, "unknown run mode");
    if (t >= kStepLimit || n_steps > kStepLimit - t)
        return fail(FSB_ERR_INVALID_ARG, "iterations must stay below 2^32");
    if (kStaticLayout.total > kStaticScratchBytes)  // the layout is fixed; checked at compile time
        return fail(FSB_ERR_UNSUPPORTED, "the static scratch is smaller than a school's workspace");
    void* ws = nullptr;
    FSB_HIP_TRY(static_scratch(&ws), "address of the static scratch");
    // A handle on the stack over the scratch, with the caller's ring.
    fsb_school h{};
    fill_school(&h, *cfg, state, ws, kStaticScratchBytes, stream, kStaticLayout, t);
    h.args.hist = records;
    FSB_HIP_TRY(launch_reset(h.args, h.stream), "reset launch");
    rc = n_steps ? fsb_run(&h, n_steps, mode) : FSB_OK;
    if (!rc) rc = finish_pending(&h);
    if (!rc && status) FSB_HIP_TRY(launch_copy_error(h.args, status, h.stream), "status copy");
    return rc;
}

int fsb_profile_enable(fsb_school* h, int every) {
    if (!h) return fail(FSB_ERR_INVALID_ARG, "handle is NULL");
    if (every < 0) return fail(FSB_ERR_INVALID_ARG, "every must be >= 0");
    h->profile_every = (uint32_t)every;
    for (int k = 0; k < FSB_KERNEL_KINDS; ++k) h->launches[k] = 0;
    return FSB_OK;
}

int fsb_barrier_probe(fsb_school* h, uint32_t grid, uint32_t n_barriers, double* out_us,
                      uint32_t* out_max) {
    if (!h || !out_us) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    if (n_barriers == 0) return fail(FSB_ERR_INVALID_ARG, "n_barriers must be >= 1");
    if (h->resident[0] == 0)
        FSB_HIP_TRY(fused_resident_grid(0, &h->resident[0]), "occupancy query");
    if (h->resident[0] == 0)
        return fail(FSB_ERR_UNSUPPORTED, "the persistent kernel cannot be resident on this device");
    if (grid == 0) grid = fused_grid(h->cfg.n_fish, h->resident[0]);
    if (grid > h->resident[0])
        return fail(FSB_ERR_INVALID_ARG, "grid exceeds the co-resident maximum (" +
                                             std::to_string(h->resident[0]) + " blocks)");
    int rc = finish_pending(h);
    if (rc) return rc;
    FusedArgs f{};
    f.steps = n_barriers;
    f.spin_limit = barrier_spin_limit();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
    if (e == hipSuccess) {
        e = launch_barrier_probe(h->args, f, grid, h->stream);
        if (e != hipSuccess) rc = persistent_launch_fail(e, "barrier probe launch");
    } else {
        rc = hip_fail(e, "hipEvent");
    }
    float ms = 0.0f;
    if (!rc && (e = hipEventRecord(e1, h->stream)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
    if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
    if (!rc && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = check_device_error(h);
    if (rc) return rc;
    if (out_max) {
        FSB_HIP_TRY(hipMemcpyDtoH(out_max, reinterpret_cast<hipDeviceptr_t>(&h->args.ctrl->probe_max),
                                  sizeof(uint32_t)),
                    "hipMemcpyDtoH");
    }
    *out_us = ms * 1e3 / (double)n_barriers;
    return FSB_OK;
}

int fsb_valu_probe(uint32_t kind, uint32_t blocks, uint32_t iters, void* out, size_t out_bytes,
                   void* stream, double* out_ms, uint64_t* out_lane_instructions) {
    // Vector instructions per lane and round of each probe kind (the assembly
    // of the probe kernels is checked for exactly these).
    static const uint64_t per_round[FSB_PROBE_KINDS] = {8, 80, 80};
    if (kind >= FSB_PROBE_KINDS) return fail(FSB_ERR_INVALID_ARG, "unknown probe kind");
    if (blocks == 0 || iters == 0) return fail(FSB_ERR_INVALID_ARG, "blocks and iters must be >= 1");
    if (!out || !out_ms || !out_lane_instructions) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    if (!aligned(out, 4)) return fail(FSB_ERR_INVALID_ARG, "out is not 4-byte aligned");
    if (out_bytes < (size_t)blocks * kProbeThreads * 4)
        return fail(FSB_ERR_INVALID_ARG, "out must hold blocks x 256 words");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = FSB_OK;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_valu_probe(kind, blocks, iters, out, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = hip_fail(e, "VALU probe");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    *out_ms = ms;
    *out_lane_instructions = (uint64_t)blocks * kProbeThreads * iters * per_round[kind];
    return FSB_OK;
}

int fsb_sweep_probe(float* cols[4], uint64_t n, uint32_t grid, uint32_t streamed, void* stream,
                    double* out_ms) {
    if (!cols || !out_ms) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    if (n == 0 || n % 4) return fail(FSB_ERR_INVALID_ARG, "n must be a positive multiple of 4");
    for (int k = 0; k < 4; ++k) {
        if (!cols[k]) return fail(FSB_ERR_INVALID_ARG, "NULL column");
        if (!aligned(cols[k], 16)) return fail(FSB_ERR_INVALID_ARG, "columns must be 16-byte aligned");
    }
    if (grid == 0) grid = 512;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = FSB_OK;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_sweep_probe(cols, n, grid, streamed != 0, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = hip_fail(e, "sweep probe");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    *out_ms = ms;
    return FSB_OK;
}

int fsb_eval_sqrt(const float* in, float* out, uint64_t n, void* stream) {
    if (n == 0) return FSB_OK;
    if (!in || !out) return fail(FSB_ERR_INVALID_ARG, "NULL array");
    if (!aligned(in, 4) || !aligned(out, 4)) return fail(FSB_ERR_INVALID_ARG, "arrays must be 4-byte aligned");
    FSB_HIP_TRY(launch_eval_sqrt(in, out, n, static_cast<hipStream_t>(stream)), "sqrt launch");
    return FSB_OK;
}

int fsb_kernel_times(fsb_school* h, uint64_t counts[FSB_KERNEL_KINDS], double ms[FSB_KERNEL_KINDS]) {
    if (!h || !counts || !ms) return fail(FSB_ERR_INVALID_ARG, "NULL argument");
    FSB_HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    for (int k = 0; k < FSB_KERNEL_KINDS; ++k) {
        counts[k] = h->timers[k].used;
        FSB_HIP_TRY(h->timers[k].total(&ms[k]), "hipEventElapsedTime");
        h->timers[k].used = 0;
    }
    return FSB_OK;
}

}  // extern "C"
