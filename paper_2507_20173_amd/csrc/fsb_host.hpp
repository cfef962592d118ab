// fsb_host.hpp -- host-side helpers shared by the C ABI translation units:
// error reporting, argument checks and HIP-event kernel timers.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "fsb.h"
#include "fsb_internal.hpp"

namespace fsb {

// Message of the last failure on this thread (shared by every translation unit).
inline std::string& last_error() {
    thread_local std::string msg;
    return msg;
}

inline int fail(int code, const std::string& msg) {
    last_error() = msg;
    return code;
}

inline int hip_fail(hipError_t e, const char* what) {
    last_error() = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return FSB_ERR_HIP;
}

// A failed persistent (cooperative) launch.  Two statuses mean that the grid
// cannot be guaranteed co-resident, which the caller can act on, rather than
// a runtime failure: the grid is larger than the device holds at once, or
// (hipErrorIllegalState) the runtime refuses cooperative launches while
// another process has work on the same GPU.  Both become
// FSB_ERR_UNSUPPORTED with a message naming the cause; the plain mode
// (per-iteration launches) is unaffected.  Every other status is FSB_ERR_HIP.
inline int persistent_launch_fail(hipError_t e, const char* what) {
    if (e == hipErrorCooperativeLaunchTooLarge)
        return fail(FSB_ERR_UNSUPPORTED,
                    std::string(what) + ": the persistent grid cannot be co-resident on this device");
    if (e == hipErrorIllegalState)
        return fail(FSB_ERR_UNSUPPORTED,
                    std::string(what) + ": the runtime refused the cooperative launch (another "
                                        "process is using the GPU); FSB_RUN_PLAIN still works");
    return hip_fail(e, what);
}

#define FSB_HIP_TRY(expr, what)                 \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr uint64_t kMaxFish = 1ull << 40;
constexpr uint32_t kMaxHistory = 1u << 24;
constexpr uint64_t kStepLimit = 1ull << 32;  // iteration index fills one counter word

inline int check_config(const fsb_config* c, bool need_fish) {
    if (!c) return fail(FSB_ERR_INVALID_ARG, "config is NULL");
    if (need_fish && c->n_fish == 0) return fail(FSB_ERR_INVALID_ARG, "n_fish must be >= 1");
    if (c->n_fish > kMaxFish) return fail(FSB_ERR_INVALID_ARG, "n_fish exceeds 2^40");
    if (!(std::isfinite(c->pond_half) && c->pond_half > 0.0f && c->pond_half <= 0x1p63f))
        return fail(FSB_ERR_INVALID_ARG, "pond_half must be in (0, 2^63]");
    if (!(std::isfinite(c->swim_step) && c->swim_step >= 0.0f))
        return fail(FSB_ERR_INVALID_ARG, "swim_step must be finite and >= 0");
    if (c->swim_step != 0.0f && c->swim_step < 0x1p-103f)
        return fail(FSB_ERR_INVALID_ARG, "swim_step must be 0 or at least 2^-103");
    if (!(std::isfinite(c->w_init_lo) && std::isfinite(c->w_init_hi) && c->w_init_lo <= c->w_init_hi))
        return fail(FSB_ERR_INVALID_ARG, "need finite w_init_lo <= w_init_hi");
    if (!(std::isfinite(c->w_min) && std::isfinite(c->w_max) && c->w_min <= c->w_max))
        return fail(FSB_ERR_INVALID_ARG, "need finite w_min <= w_max");
    for (float v : {c->w_init_lo, c->w_init_hi, c->w_min, c->w_max})
        if (!(v >= -0x1p24f && v <= 0x1p24f))
            return fail(FSB_ERR_INVALID_ARG, "weight bounds must lie in [-2^24, 2^24]");
    if (c->reduce_mode != FSB_REDUCE_COMPENSATED && c->reduce_mode != FSB_REDUCE_NAIVE_F32 &&
        c->reduce_mode != FSB_REDUCE_CRITICAL_F32)
        return fail(FSB_ERR_INVALID_ARG, "unknown reduce_mode");
    if (c->history_len == 0 || c->history_len > kMaxHistory)
        return fail(FSB_ERR_INVALID_ARG, "history_len must be in [1, 2^24]");
    if (c->swim_rule & ~(FSB_SWIM_GREEDY | FSB_SWIM_WEIGHTED))
        return fail(FSB_ERR_INVALID_ARG, "unknown swim_rule flags");
    if ((c->swim_rule & FSB_SWIM_WEIGHTED) && !(c->w_min > 0.0f && c->w_init_lo > 0.0f))
        return fail(FSB_ERR_INVALID_ARG, "the weighted swim rule needs w_min > 0 and w_init_lo > 0");
    return FSB_OK;
}

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline int check_columns(const fsb_state& s, uint64_t n) {
    const float* cols[5] = {s.x, s.y, s.w, s.prev, s.cur};
    const char* names[5] = {"x", "y", "w", "prev", "cur"};
    for (int i = 0; i < 5; ++i) {
        if (!cols[i]) return fail(FSB_ERR_INVALID_ARG, std::string("column ") + names[i] + " is NULL");
        if (!aligned(cols[i], 16))
            return fail(FSB_ERR_INVALID_ARG, std::string("column ") + names[i] + " is not 16-byte aligned");
    }
    const uintptr_t bytes = (uintptr_t)n * sizeof(float);
    for (int i = 0; i < 5; ++i)
        for (int j = i + 1; j < 5; ++j) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(cols[i]);
            const uintptr_t b = reinterpret_cast<uintptr_t>(cols[j]);
            if (a < b + bytes && b < a + bytes)
                return fail(FSB_ERR_INVALID_ARG, std::string("columns ") + names[i] + " and " +
                                                     names[j] + " overlap");
        }
    return FSB_OK;
}

inline int check_workspace(void* ws, size_t bytes, size_t need) {
    if (!ws) return fail(FSB_ERR_INVALID_ARG, "workspace is NULL");
    if (!aligned(ws, kAlign)) return fail(FSB_ERR_INVALID_ARG, "workspace is not 256-byte aligned");
    if (bytes < need)
        return fail(FSB_ERR_INVALID_ARG, "workspace too small: " + std::to_string(bytes) + " < " +
                                             std::to_string(need) + " bytes");
    return FSB_OK;
}

// Pairs of HIP events bracketing launches of one kernel kind.
struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
    ~Timer() {
        for (auto& p : pool) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    }
    hipError_t next(std::pair<hipEvent_t, hipEvent_t>** out) {
        if (used == pool.size()) {
            std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
            hipError_t e = hipEventCreate(&p.first);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&p.second);
            if (e != hipSuccess) {
                (void)hipEventDestroy(p.first);
                return e;
            }
            pool.push_back(p);
        }
        *out = &pool[used++];
        return hipSuccess;
    }
    hipError_t total(double* ms) {
        double sum = 0.0;
        for (size_t i = 0; i < used; ++i) {
            float v = 0.0f;
            hipError_t e = hipEventElapsedTime(&v, pool[i].first, pool[i].second);
            if (e != hipSuccess) return e;
            sum += v;
        }
        *ms = sum;
        return hipSuccess;
    }
};


}  // namespace fsb
