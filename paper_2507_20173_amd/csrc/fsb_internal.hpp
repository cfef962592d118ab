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
    uint32_t reserved0[2];
    float naive_acc[2][4];    // float32 atomic sums of the naive mode, slot t & 1
    uint32_t pad[52];
};
static_assert(sizeof(Ctrl) == 256, "Ctrl is one aligned block");

constexpr uint32_t kErrBarrierTimeout = 1u;

// Synchronisation words of the persistent kernel's two-level grid barrier,
// each on its own 256-byte line (word offsets into the sync area).
constexpr uint32_t kLineWords = 64;
constexpr uint32_t kSyncRootCount = 0;                  // group leaders arrived
constexpr uint32_t kSyncPhase = 1 * kLineWords;         // completed barriers
constexpr uint32_t kSyncRootMax = 2 * kLineWords;       // max over group maxima
constexpr uint32_t kSyncMaxPub = 3 * kLineWords;        // published M, slot s & 1
constexpr uint32_t kSyncGroups = 4 * kLineWords;        // group g: [count, max] at + g * line
constexpr uint32_t kMaxGroups = 64;
constexpr uint32_t kSyncWords = kSyncGroups + kMaxGroups * kLineWords;

// Workspace of one school:
//   [Ctrl][history ring][block maxima u32 x kMaxGrid]
//   [block partials f64 x 3 x kMaxGrid x 2 (slot t & 1)][barrier sync area]
struct Layout {
    size_t ctrl, hist, blockmax, partials, sync, total;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline Layout school_layout(uint32_t history_len) {
    Layout L;
    L.ctrl = 0;
    L.hist = align_up(L.ctrl + sizeof(Ctrl), kAlign);
    L.blockmax = align_up(L.hist + (size_t)history_len * sizeof(fsb_record), kAlign);
    L.partials = align_up(L.blockmax + kMaxGrid * sizeof(uint32_t), kAlign);
    L.sync = align_up(L.partials + 2 * 3 * (size_t)kMaxGrid * sizeof(double), kAlign);
    L.total = align_up(L.sync + kSyncWords * sizeof(uint32_t), kAlign);
    return L;
}

// Everything a single-school kernel needs, passed by value.
struct SchoolArgs {
    float *x, *y, *w, *prev, *cur;
    uint64_t n;           // fish
    uint32_t k0, k1;      // Philox key (seed lo, hi)
    float H, S, wmin, wmax;
    Ctrl *ctrl;
    fsb_record *hist;
    uint32_t hist_len;
    uint32_t *blockmax;   // [kMaxGrid] per-block max |diff| bits of the swim pass
    double *partials;     // [2][3][kMaxGrid] per-block binary64 sums
    uint32_t *sync;       // [kSyncWords] persistent-kernel barrier words
};

// Step-specific arguments of the plain passes.
struct StepArgs {
    uint32_t t;           // iteration index (low 32 bits; host keeps t < 2^32)
    uint32_t swim_grid;   // blocks of the swim pass (feed pass reads that many maxima)
    uint32_t combine;     // swim pass block 0 first writes the pending record
    uint32_t prev_t;      // iteration whose record is pending
    uint32_t prev_grid;   // blocks that produced its partials
    uint32_t naive;       // FSB_REDUCE_NAIVE_F32
    const float *dx;      // test hook: displacements instead of draws (or null)
    const float *dy;
};

// Arguments of the persistent multi-iteration kernel.
struct FusedArgs {
    uint32_t t0;          // first iteration of the launch
    uint32_t steps;       // iterations in the launch, >= 1
    uint32_t naive;
    uint32_t group_size;  // blocks per barrier group
    uint32_t groups;      // barrier groups (<= kMaxGroups)
    uint32_t streaming;   // non-temporal loads/stores (state larger than the last-level cache)
};

// Launchers (fsb_kernels.hip).  All enqueue on `stream` and return the HIP
// status of the launch.
uint32_t plain_grid(uint64_t n);
hipError_t launch_reset(const SchoolArgs& a, hipStream_t stream);
hipError_t launch_init(const SchoolArgs& a, float wlo, float whi, hipStream_t stream);
hipError_t launch_swim_eval(const SchoolArgs& a, const StepArgs& s, hipStream_t stream);
hipError_t launch_feed_bary(const SchoolArgs& a, const StepArgs& s, uint32_t grid,
                            hipStream_t stream);
hipError_t launch_combine(const SchoolArgs& a, uint32_t t, uint32_t grid, uint32_t naive,
                          hipStream_t stream);
// Largest co-resident grid of the persistent kernel (0 if it cannot run).
hipError_t fused_resident_grid(uint32_t naive, uint32_t* out_grid);
// Grid the persistent kernel uses for n fish given the resident maximum.
uint32_t fused_grid(uint64_t n, uint32_t resident);
// Barrier grouping of a persistent grid.
void fused_groups(uint32_t grid, uint32_t* group_size, uint32_t* groups);
hipError_t launch_fused(const SchoolArgs& a, const FusedArgs& f, uint32_t grid,
                        hipStream_t stream);

}  // namespace fsb
