// fsb_kernels.hip -- HIP kernels of the FSB iteration for gfx950 (MI355X).
//
// Plain iteration t = two streaming passes over the SoA columns:
//   swim pass  (reads x, y; writes x, y, prev, cur; 24 B/fish)
//     draws, swim + pond clamp, objective, |diff|; each block stores its max
//     |diff| bit pattern (non-negative floats order like their bits, so the
//     max is exact and independent of order).  Block 0 first writes the
//     pending record of the previous iteration from its block partials.
//   feed pass  (reads prev, w, x, y; writes w; 20 B/fish)
//     every block reduces the swim pass's block maxima to M, feeds, and
//     accumulates sum w, sum w*x, sum w*y per lane in compensated float32,
//     merges lanes with TwoSum and waves in binary64: one binary64 partial
//     per block.
// Pipelined plain iterations (a run of n >= 2 iterations, one launch each):
//   swim pass of the first iteration, then for each next iteration t
//   feed-swim pass (reads x, y, w, prev; writes x, y, w, prev; 32 B/fish)
//     every block reduces the previous launch's block maxima to M_{t-1},
//     feeds each fish with it, adds the fed weight and the position to
//     iteration t-1's sums, then swims the fish for iteration t: prev_t is
//     the objective of the position it swims from (cur of t-1, recomputed),
//     so cur is not stored; each block stores its max |diff| of t.
//   and the feed pass of the last iteration, which also writes cur.
//   Block maxima and partials sit in slot t & 1, so a launch reads the
//   previous launch's while it writes its own.
// Persistent iteration (one cooperative launch for many iterations, one grid
// barrier per iteration; 32 B/fish per iteration):
//   prologue   swim t0 from (x, y), keep (x, y, prev), block max -> M_t0
//   sweep s    read (x, y, w, prev); cur = |p| recomputed; feed with M_s;
//              partial sums of s; then swim s+1 and its max -> M_{s+1};
//              write (x, y, w, prev); grid barrier.  The last sweep writes
//              (w, cur) instead, leaving the five columns complete.
//   The record of s is written after the barrier by block s % grid.
// Critical mode (an ablation of the reduction, plain passes only): every fish
// folds its |diff| into one shared max word and its three terms into three
// shared float32 sums with its own device-scope atomic, the way a critical
// section entered once per fish serialises the update; no tree at all.
// No kernel reads a cur it has not written in the same launch: a fish's
// objective is the distance of its position, so it is recomputed from (x, y)
// with the same binary32 operations that produced the stored value (the state
// after every iteration satisfies cur == sqrtf(x*x + y*y)); only the deep
// kernels read cur back, between their own supersteps.
// Records are combined in a fixed order, so every sum is deterministic for a
// given launch shape.  Each thread handles groups of four consecutive fish
// (one float4 per column): two Philox calls, for fish pairs 2g and 2g+1.
// The n % 4 fish past the last full group are handled one by one by the last
// block.  A thread keeps the same fish in every sweep of a launch.
#include <hip/hip_ext.h>

#include <cstdlib>
#include <cstring>
#include <mutex>

#include "fsb_sweep.hpp"

namespace fsb {

constexpr int kBlock = 256;
constexpr int kUnroll = 2;  // groups in flight per thread (persistent kernels)
// Plain passes: grid caps and groups in flight per thread, measured at
// N = 2^24 (swim caps 2048-8192 within 1.5%; feed best at 512-768 blocks,
// 20% slower at 256, 5% at 1024-2048: each of its blocks first reads every
// swim block's max).
constexpr uint32_t kSwimGridCap = 4096;
constexpr uint32_t kFeedGridCap = 512;
// The pipelined pass runs the feed pass's grid: each iteration's sums then
// come from the same lanes in the same order whichever pass feeds it, so a
// pipelined run's records equal fsb_step's bit for bit.  It is also its
// fastest grid (measured at N = 2^24 and 2^26: 256 blocks 27% and 17%
// slower, 768 3% and 2%, 1024-4096 6-11%).
constexpr uint32_t kPipeGridCap = kFeedGridCap;
constexpr int kSwimUnroll = 1;
constexpr int kFeedUnroll = 1;

__device__ __forceinline__ double* partial_slot(const SchoolArgs& a, uint32_t t, int k) {
    return a.partials + ((size_t)(t & 1u) * 3 + k) * kMaxGrid;
}

// Per-block max |diff| bits of the swim of iteration t.
__device__ __forceinline__ uint32_t* blockmax_slot(const SchoolArgs& a, uint32_t t) {
    return a.blockmax + (size_t)(t & 1u) * kMaxGrid;
}

// The deep kernel's partials of iteration t: slot t mod kDeepSlots.
__device__ __forceinline__ double* deep_slot(const SchoolArgs& a, uint32_t t, int k) {
    return a.deep + ((size_t)(t % kDeepSlots) * 3 + k) * kMaxBarrierBlocks;
}

// Block-wide reduction of the lane sums: binary64 partial of this block for
// iteration t (compensated mode) or float32 atomics into slot t & 1 (naive).
template <bool kNaive, int BLOCK = kBlock>
__device__ __forceinline__ void block_sums(const SchoolArgs& a, LaneSums<kNaive>& ls, uint32_t t) {
    constexpr int W = BLOCK / kWave;
    __shared__ CSum wave_cs[3][W];
    __shared__ float wave_fs[3][W];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if constexpr (kNaive) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float v = wave_sum_f32(ls.f[k]);
            if (lane == 0) wave_fs[k][wid] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 0; k < 3; ++k) {
                float v = wave_fs[k][0];
                for (int w = 1; w < W; ++w) v += wave_fs[k][w];
                atomicAdd(&a.ctrl->naive_acc[t & 1u][k], v);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const CSum v = wave_csum(ls.c[k]);
            if (lane == 0) wave_cs[k][wid] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 0; k < 3; ++k) {
                double v = 0.0;
                for (int w = 0; w < W; ++w) v += csum_value(wave_cs[k][w]);
                partial_slot(a, t, k)[blockIdx.x] = v;
            }
        }
    }
}

// The same for KD iterations of the deep kernel at once (its binary64 lane
// sums, merged in binary64): ls[j] holds iteration t0 + j, for j < kd.
template <int KD, int BLOCK>
__device__ __forceinline__ void block_sums_deep(const SchoolArgs& a, LaneSumsF64 (&ls)[KD],
                                                uint32_t t0, uint32_t kd) {
    constexpr int W = BLOCK / kWave;
    __shared__ double wave_v[KD][3][W];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < KD; ++j) {
        if ((uint32_t)j >= kd) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double v = wave_sum_f64(ls[j].v[k]);
            if (lane == 0) wave_v[j][k][wid] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kd * 3) {  // one thread per (iteration, sum)
        const uint32_t j = threadIdx.x / 3, k = threadIdx.x % 3;
        double v = 0.0;
        for (int w = 0; w < W; ++w) v += wave_v[j][k][w];
        deep_slot(a, t0 + j, (int)k)[blockIdx.x] = v;
    }
}

// Block max of per-thread maxima (every thread gets it).
template <int BLOCK = kBlock>
__device__ __forceinline__ uint32_t block_max(uint32_t v) {
    constexpr int W = BLOCK / kWave;
    __shared__ uint32_t wave_best[W];
    v = wave_max_u32(v);
    if (threadIdx.x % kWave == 0) wave_best[threadIdx.x / kWave] = v;
    __syncthreads();
    uint32_t m = wave_best[0];
    for (int w = 1; w < W; ++w) m = max(m, wave_best[w]);
    return m;
}

// Block maxima of KD per-thread values at once (thread 0 gets them; the
// caller passes a barrier, which synchronises, before the next call).
template <int KD, int BLOCK>
__device__ __forceinline__ void block_max_k(const uint32_t (&v)[KD], uint32_t (&out)[KD]) {
    constexpr int W = BLOCK / kWave;
    __shared__ uint32_t wave_best[KD][W];
#pragma unroll
    for (int j = 0; j < KD; ++j) {
        const uint32_t m = wave_max_u32(v[j]);
        if (threadIdx.x % kWave == 0) wave_best[j][threadIdx.x / kWave] = m;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KD; ++j) {
        uint32_t m = wave_best[j][0];
        for (int w = 1; w < W; ++w) m = max(m, wave_best[j][w]);
        out[j] = m;
    }
}

// Critical-mode updates of a shared word by every lane.  The address is
// hidden from the compiler's uniformity analysis: otherwise it may turn
// per-lane atomics on one address into a wave reduction followed by a single
// atomic, which is the tree the critical mode is there to leave out.  The
// global address space keeps them global (not flat) atomics.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* per_lane(T* p) {
    auto q = (__attribute__((address_space(1))) T*)p;
    asm volatile("" : "+v"(q));
    return q;
}
__device__ __forceinline__ void lane_atomic_max(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_max(per_lane(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lane_atomic_add(float* p, float v) {
    __hip_atomic_fetch_add(per_lane(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Control-word resets (kernels rather than memsets, so they are graph-safe).
// ---------------------------------------------------------------------------
__global__ void reset_kernel(Ctrl* ctrl) {
    uint32_t* p = reinterpret_cast<uint32_t*>(ctrl);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctrl) / 4; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Initial state: counter (pair, 0, init) -> position, (pair, 1, init) -> weight.
// ---------------------------------------------------------------------------
struct InitArgs {
    SchoolArgs a;
    float wlo, whi;
};

__device__ __forceinline__ void init_fish(const InitArgs& ia, uint32_t pa, uint32_t pb,
                                          uint32_t qa, float& x, float& y, float& w,
                                          float& c) {
    x = ia.a.H * signed_unit(pa);
    y = ia.a.H * signed_unit(pb);
    const float span = ia.whi - ia.wlo;
    w = ia.wlo + span * unit(qa);
    c = distance(x, y);
}

__global__ __launch_bounds__(kBlock) void init_kernel(InitArgs ia) {
    const SchoolArgs& a = ia.a;
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < n4; g += stride) {
        const Words p0 = pair_words(2 * g, 0, kDomainInit, a.k0, a.k1);
        const Words p1 = pair_words(2 * g + 1, 0, kDomainInit, a.k0, a.k1);
        const Words q0 = pair_words(2 * g, 1, kDomainInit, a.k0, a.k1);
        const Words q1 = pair_words(2 * g + 1, 1, kDomainInit, a.k0, a.k1);
        float4 X, Y, W, C;
        init_fish(ia, p0.r0, p0.r1, q0.r0, X.x, Y.x, W.x, C.x);
        init_fish(ia, p0.r2, p0.r3, q0.r2, X.y, Y.y, W.y, C.y);
        init_fish(ia, p1.r0, p1.r1, q1.r0, X.z, Y.z, W.z, C.z);
        init_fish(ia, p1.r2, p1.r3, q1.r2, X.w, Y.w, W.w, C.w);
        st4(a.x, g, X);
        st4(a.y, g, Y);
        st4(a.w, g, W);
        st4(a.prev, g, C);
        st4(a.cur, g, C);
    }
    if (blockIdx.x == gridDim.x - 1) {
        const uint64_t i = 4 * n4 + threadIdx.x;
        if (i < a.n) {
            const Words p = pair_words(i >> 1, 0, kDomainInit, a.k0, a.k1);
            const Words q = pair_words(i >> 1, 1, kDomainInit, a.k0, a.k1);
            const bool odd = i & 1;
            float x, y, w, c;
            init_fish(ia, odd ? p.r2 : p.r0, odd ? p.r3 : p.r1, odd ? q.r2 : q.r0, x, y, w, c);
            a.x[i] = x;
            a.y[i] = y;
            a.w[i] = w;
            a.prev[i] = c;
            a.cur[i] = c;
        }
    }
}

// ---------------------------------------------------------------------------
// Record of iteration t from its block partials (one whole block calls this).
// ---------------------------------------------------------------------------
template <int BLOCK = kBlock>
__device__ void combine_block(const SchoolArgs& a, uint32_t t, uint32_t grid, uint32_t naive,
                              uint32_t max_bits, bool deep = false) {
    constexpr int W = BLOCK / kWave;
    __shared__ double part[3][W];
    if (!naive) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (uint32_t b = threadIdx.x; b < grid; b += BLOCK)
            for (int k = 0; k < 3; ++k)
                acc[k] += (deep ? deep_slot(a, t, k) : partial_slot(a, t, k))[b];
        for (int k = 0; k < 3; ++k) {
            acc[k] = wave_sum_f64(acc[k]);
            if (threadIdx.x % kWave == 0) part[k][threadIdx.x / kWave] = acc[k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        fsb_record r;
        double s[3];
        for (int k = 0; k < 3; ++k) {
            if (!naive) {
                s[k] = 0.0;
                for (int w = 0; w < W; ++w) s[k] += part[k][w];
            } else {
                s[k] = (double)a.ctrl->naive_acc[t & 1u][k];
                a.ctrl->naive_acc[t & 1u][k] = 0.0f;
            }
        }
        r.sum_w = s[0];
        r.sum_wx = s[1];
        r.sum_wy = s[2];
        r.max_delta = __uint_as_float(max_bits);
        r.step_lo = t;
        a.hist[t % a.hist_len] = r;
        a.ctrl->crit_max[t & 1u] = 0u;  // critical mode: slot free for iteration t + 2
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void combine_kernel(SchoolArgs a, uint32_t t, uint32_t grid,
                                                         uint32_t naive) {
    combine_block(a, t, grid, naive, a.ctrl->last_max);
}

// ---------------------------------------------------------------------------
// Plain swim pass.
// ---------------------------------------------------------------------------
// Cache policy of the plain passes (chosen on the host from the footprint).
// cur is only written by these passes, and always streamed.  kCached keeps x, y, prev and w in
// the last-level cache, kStreamW streams w too (touched by the feed pass
// alone) so x, y, prev stay resident, and kStreamAll streams every column
// once even those three cannot fit.
constexpr int kCached = 0, kStreamW = 1, kStreamAll = 2;

template <bool kInject, int kPolicy, bool kCritical>
__global__ __launch_bounds__(kBlock) void swim_eval_kernel(SchoolArgs a, StepArgs s) {
    constexpr bool NT = kPolicy == kStreamAll;
    uint32_t* const crit = &a.ctrl->crit_max[s.t & 1u];
    if (s.combine && blockIdx.x == 0)
        combine_block(a, s.prev_t, s.prev_grid, s.naive, a.ctrl->last_max);

    const float H = a.H;
    const SwimRule rule{a.rule, a.wmin};
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t best = 0u;
    for (uint64_t g0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g0 < n4;
         g0 += kSwimUnroll * stride) {
        float4 X[kSwimUnroll], Y[kSwimUnroll], Wt[kSwimUnroll];
#pragma unroll
        for (int u = 0; u < kSwimUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g < n4) {
                X[u] = ldv<NT>(a.x, g);
                Y[u] = ldv<NT>(a.y, g);
                Wt[u] = swim_weights<NT>(rule, a.w, g);
            }
        }
#pragma unroll
        for (int u = 0; u < kSwimUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g >= n4) break;
            float dx[4], dy[4];
            if constexpr (kInject) {
                const float4 DX = ld4(s.dx, g), DY = ld4(s.dy, g);
                dx[0] = DX.x; dx[1] = DX.y; dx[2] = DX.z; dx[3] = DX.w;
                dy[0] = DY.x; dy[1] = DY.y; dy[2] = DY.z; dy[3] = DY.w;
            } else {
                group_draws(a.S, a.k0, a.k1, g, s.t, dx, dy);
            }
            float4 nx = X[u], ny = Y[u], c, nc;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                lane_of(c, k) = distance(lane_of(nx, k), lane_of(ny, k));
                lane_of(nc, k) = swim(rule, lane_of(nx, k), lane_of(ny, k), dx[k], dy[k], H,
                                      lane_of(c, k), lane_of(Wt[u], k));
                const uint32_t d = mag_bits(lane_of(c, k) - lane_of(nc, k));
                if constexpr (kCritical) lane_atomic_max(crit, d);
                else best = max(best, d);
            }
            stv<NT>(a.x, g, nx);
            stv<NT>(a.y, g, ny);
            stv<NT>(a.prev, g, c);
            stv<true>(a.cur, g, nc);
        }
    }
    if (blockIdx.x == gridDim.x - 1) {
        const uint64_t i = 4 * n4 + threadIdx.x;
        if (i < a.n) {
            float dx, dy;
            if constexpr (kInject) {
                dx = s.dx[i];
                dy = s.dy[i];
            } else {
                fish_draw(a.S, a.k0, a.k1, i, s.t, dx, dy);
            }
            float x = a.x[i], y = a.y[i];
            const float c = distance(x, y);
            const float wt = (rule.flags & kSwimWeighted) ? a.w[i] : 1.0f;
            const float nc = swim(rule, x, y, dx, dy, H, c, wt);
            const uint32_t d = mag_bits(c - nc);
            if constexpr (kCritical) lane_atomic_max(crit, d);
            else best = max(best, d);
            a.x[i] = x;
            a.y[i] = y;
            a.prev[i] = c;
            a.cur[i] = nc;
        }
    }
    if constexpr (!kCritical) {
        const uint32_t m = block_max(best);
        if (threadIdx.x == 0) blockmax_slot(a, s.t)[blockIdx.x] = m;
    }
}

// ---------------------------------------------------------------------------
// Plain feed pass.
// ---------------------------------------------------------------------------
// Reduction of the feed pass: compensated tree, naive float32 tree with one
// atomic per block, or critical (one atomic per fish, max and sums).
constexpr int kRedCompensated = 0, kRedNaive = 1, kRedCritical = 2;

// M of iteration t: the max of the `count` block maxima its swim stored (every
// thread of the block gets it).  Four maxima per load, all loads of a thread
// issued before any is used.
__device__ __forceinline__ uint32_t school_max(const SchoolArgs& a, uint32_t t, uint32_t count) {
    const uint32_t* bm = blockmax_slot(a, t);
    const uint32_t n_vec = count / 4;
    const uint4* bm4 = reinterpret_cast<const uint4*>(bm);
    constexpr uint32_t kPer = kMaxGrid / 4 / kBlock;  // vector loads per thread, at most
    uint4 v[kPer];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        const uint32_t i = threadIdx.x + j * kBlock;
        v[j] = i < n_vec ? bm4[i] : make_uint4(0u, 0u, 0u, 0u);
    }
    uint32_t mb = 0u;
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) mb = max(mb, max(max(v[j].x, v[j].y), max(v[j].z, v[j].w)));
    for (uint32_t b = 4 * n_vec + threadIdx.x; b < count; b += kBlock) mb = max(mb, bm[b]);
    return block_max(mb);
}

// kWriteCur: also store each fish's objective in cur (the closing pass of a
// pipelined run).  With s.combine, block 0 first writes the pending record.
template <int kRed, int kPolicy, bool kWriteCur>
__global__ __launch_bounds__(kBlock) void feed_bary_kernel(SchoolArgs a, StepArgs s) {
    constexpr bool NT = kPolicy == kStreamAll;
    constexpr bool NTW = kPolicy != kCached;
    constexpr bool kNaive = kRed != kRedCompensated;
    if (s.combine && blockIdx.x == 0)
        combine_block(a, s.prev_t, s.prev_grid, s.naive, a.ctrl->last_max);
    // M = max over the swim's block maxima (critical mode: the shared word).
    uint32_t mb;
    if constexpr (kRed == kRedCritical) mb = a.ctrl->crit_max[s.t & 1u];
    else mb = school_max(a, s.t, s.swim_grid);
    if (threadIdx.x == 0 && blockIdx.x == 0) a.ctrl->last_max = mb;
    const float M = __uint_as_float(mb);

    const float wmin = a.wmin, wmax = a.wmax;
    LaneSums<kNaive> ls;
    float* const acc = a.ctrl->naive_acc[s.t & 1u];
    // One fish's terms: into the lane's sums, or (critical) straight into the
    // shared float32 sums.
    auto add = [&](float nw, float x, float y) {
        if constexpr (kRed == kRedCritical) {
            lane_atomic_add(acc + 0, nw);
            lane_atomic_add(acc + 1, nw * x);
            lane_atomic_add(acc + 2, nw * y);
        } else {
            ls.add(nw, x, y);
        }
    };
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g0 < n4;
         g0 += kFeedUnroll * stride) {
        float4 P[kFeedUnroll], W[kFeedUnroll], X[kFeedUnroll], Y[kFeedUnroll];
#pragma unroll
        for (int u = 0; u < kFeedUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g < n4) {
                P[u] = ldv<NT>(a.prev, g);
                W[u] = ldv<NTW>(a.w, g);
                X[u] = ldv<NT>(a.x, g);
                Y[u] = ldv<NT>(a.y, g);
            }
        }
#pragma unroll
        for (int u = 0; u < kFeedUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g >= n4) break;
            float4 nw, C;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                lane_of(C, k) = distance(lane_of(X[u], k), lane_of(Y[u], k));
                const float diff = lane_of(P[u], k) - lane_of(C, k);
                lane_of(nw, k) = feed(lane_of(W[u], k), diff, M, wmin, wmax);
                if constexpr (kRed == kRedCritical) add(lane_of(nw, k), lane_of(X[u], k), lane_of(Y[u], k));
            }
            if constexpr (kRed != kRedCritical) ls.add4(nw, X[u], Y[u]);
            stv<NTW>(a.w, g, nw);
            if constexpr (kWriteCur) stv<true>(a.cur, g, C);
        }
    }
    if (blockIdx.x == gridDim.x - 1) {
        const uint64_t i = 4 * n4 + threadIdx.x;
        if (i < a.n) {
            const float x = a.x[i], y = a.y[i];
            const float c = distance(x, y);
            const float nw = feed(a.w[i], a.prev[i] - c, M, wmin, wmax);
            a.w[i] = nw;
            if constexpr (kWriteCur) a.cur[i] = c;
            add(nw, x, y);
        }
    }
    if constexpr (kRed != kRedCritical) block_sums<kNaive>(a, ls, s.t);
}

// ---------------------------------------------------------------------------
// Pipelined pass: the feed of iteration t - 1 and the swim of iteration t.
// ---------------------------------------------------------------------------
// Within a run, the feed of t - 1 and the swim of t touch each fish one after
// the other, so one launch does both and the columns are read and written
// once per iteration (x, y, w, prev: 32 B per fish) instead of twice.  Every
// operation of a fish is the plain passes', in their order: the objective of
// the position (cur of t - 1), the feed with M_{t-1}, the fed weight and the
// position into iteration t-1's sums, then the swim of t from that position
// (the weighted rule sees the fed weight, as the swim pass reads it).  The
// objective swum from is prev_t; the new one is only compared with it, and
// the run's closing feed pass stores cur from the final positions.
template <bool kNaive, int kPolicy>
__global__ __launch_bounds__(kBlock) void feed_swim_kernel(SchoolArgs a, StepArgs s) {
    constexpr bool NT = kPolicy == kStreamAll;
    constexpr bool NTW = kPolicy != kCached;
    const uint32_t tf = s.t - 1u;  // iteration fed
    if (s.combine && blockIdx.x == 0)
        combine_block(a, s.prev_t, s.prev_grid, s.naive, a.ctrl->last_max);
    const uint32_t mb = school_max(a, tf, s.swim_grid);
    if (threadIdx.x == 0 && blockIdx.x == 0) a.ctrl->last_max = mb;
    const float M = __uint_as_float(mb);

    const float H = a.H, wmin = a.wmin, wmax = a.wmax;
    const SwimRule rule{a.rule, a.wmin};
    LaneSums<kNaive> ls;
    uint32_t best = 0u;
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < n4; g += stride) {
        float4 X = ldv<NT>(a.x, g), Y = ldv<NT>(a.y, g);
        float4 W = ldv<NTW>(a.w, g), P = ldv<NT>(a.prev, g);
        float dx[4], dy[4];
        group_draws(a.S, a.k0, a.k1, g, s.t, dx, dy);
        float4 C, nw;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lane_of(C, k) = distance(lane_of(X, k), lane_of(Y, k));
            lane_of(nw, k) = feed(lane_of(W, k), lane_of(P, k) - lane_of(C, k), M, wmin, wmax);
        }
        ls.add4(nw, X, Y);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float nc = swim(rule, lane_of(X, k), lane_of(Y, k), dx[k], dy[k], H,
                                  lane_of(C, k), lane_of(nw, k));
            best = max(best, mag_bits(lane_of(C, k) - nc));
        }
        stv<NT>(a.x, g, X);
        stv<NT>(a.y, g, Y);
        stv<NTW>(a.w, g, nw);
        stv<NT>(a.prev, g, C);
    }
    if (blockIdx.x == gridDim.x - 1) {
        const uint64_t i = 4 * n4 + threadIdx.x;
        if (i < a.n) {
            float x = a.x[i], y = a.y[i];
            const float c = distance(x, y);
            const float nw = feed(a.w[i], a.prev[i] - c, M, wmin, wmax);
            ls.add(nw, x, y);
            float dx, dy;
            fish_draw(a.S, a.k0, a.k1, i, s.t, dx, dy);
            const float nc = swim(rule, x, y, dx, dy, H, c, nw);
            best = max(best, mag_bits(c - nc));
            a.x[i] = x;
            a.y[i] = y;
            a.w[i] = nw;
            a.prev[i] = c;
        }
    }
    block_sums<kNaive>(a, ls, tf);
    __syncthreads();  // block_max's staging words were read by school_max
    const uint32_t m = block_max(best);
    if (threadIdx.x == 0) blockmax_slot(a, s.t)[blockIdx.x] = m;
}

// ---------------------------------------------------------------------------
// Persistent multi-iteration kernel (1024 threads: one block per CU, so the
// barrier has few participants).
// ---------------------------------------------------------------------------
constexpr int kFusedBlock = 1024;

template <bool kNaive, bool kNT>
__global__ __launch_bounds__(kFusedBlock) void fused_kernel(SchoolArgs a, FusedArgs f) {
    constexpr int B = kFusedBlock;
    __shared__ uint32_t M_sh;
    const float H = a.H, wmin = a.wmin, wmax = a.wmax;
    const SwimRule rule{a.rule, a.wmin};
    const uint32_t grid = gridDim.x;
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)grid * B;
    const uint64_t gbase = (uint64_t)blockIdx.x * B + threadIdx.x;
    const uint64_t tail_i = 4 * n4 + threadIdx.x;
    const bool has_tail = blockIdx.x == grid - 1 && tail_i < a.n;
    const Barrier bar{a.sync, a.ctrl, f.spin_limit};
    uint32_t phase = 0;

    // Prologue: swim t0, keep (x, y, prev), M_t0.
    {
        uint32_t best = 0u;
        for (uint64_t g = gbase; g < n4; g += stride) {
            float4 X = ldv<kNT>(a.x, g), Y = ldv<kNT>(a.y, g), C;
            float4 Wt = swim_weights<kNT>(rule, a.w, g);
            float dx[4], dy[4];
            group_draws(a.S, a.k0, a.k1, g, f.t0, dx, dy);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lane_of(C, q) = distance(lane_of(X, q), lane_of(Y, q));
                const float nc = swim(rule, lane_of(X, q), lane_of(Y, q), dx[q], dy[q], H,
                                      lane_of(C, q), lane_of(Wt, q));
                best = max(best, mag_bits(lane_of(C, q) - nc));
            }
            stv<kNT>(a.x, g, X);
            stv<kNT>(a.y, g, Y);
            stv<kNT>(a.prev, g, C);
        }
        if (has_tail) {
            float dx, dy;
            fish_draw(a.S, a.k0, a.k1, tail_i, f.t0, dx, dy);
            float x = a.x[tail_i], y = a.y[tail_i];
            const float c = distance(x, y);
            const float wt = (rule.flags & kSwimWeighted) ? a.w[tail_i] : 1.0f;
            const float nc = swim(rule, x, y, dx, dy, H, c, wt);
            best = max(best, mag_bits(c - nc));
            a.x[tail_i] = x;
            a.y[tail_i] = y;
            a.prev[tail_i] = c;
        }
        const uint32_t m = block_max<B>(best);
        if (!barrier_max(bar, m, phase, &M_sh)) return;
    }

    uint32_t M_prev = 0u;  // M of the previous sweep, for its record
    for (uint32_t k = 0; k < f.steps; ++k) {
        const uint32_t s = f.t0 + k;
        const bool last = k + 1 == f.steps;
        const uint32_t M_bits = M_sh;
        const float M = __uint_as_float(M_bits);
        // Record of the previous iteration, by a rotating block.
        if (k > 0 && blockIdx.x == (s - 1u) % grid) combine_block<B>(a, s - 1u, grid, f.naive, M_prev);
        M_prev = M_bits;

        LaneSums<kNaive> ls;
        uint32_t best = 0u;
        for (uint64_t g0 = gbase; g0 < n4; g0 += kUnroll * stride) {
            float4 X[kUnroll], Y[kUnroll], W[kUnroll], P[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t g = g0 + u * stride;
                if (g < n4) {
                    X[u] = ldv<kNT>(a.x, g);
                    Y[u] = ldv<kNT>(a.y, g);
                    W[u] = ldv<kNT>(a.w, g);
                    P[u] = ldv<kNT>(a.prev, g);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t g = g0 + u * stride;
                if (g >= n4) break;
                float4 C;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    lane_of(C, q) = distance(lane_of(X[u], q), lane_of(Y[u], q));
                    const float diff = lane_of(P[u], q) - lane_of(C, q);
                    lane_of(W[u], q) = feed(lane_of(W[u], q), diff, M, wmin, wmax);
                }
                ls.add4(W[u], X[u], Y[u]);
                stv<kNT>(a.w, g, W[u]);
                if (last) {
                    stv<kNT>(a.cur, g, C);
                } else {
                    float dx[4], dy[4];
                    group_draws(a.S, a.k0, a.k1, g, s + 1u, dx, dy);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float nc = swim(rule, lane_of(X[u], q), lane_of(Y[u], q), dx[q],
                                              dy[q], H, lane_of(C, q), lane_of(W[u], q));
                        best = max(best, mag_bits(lane_of(C, q) - nc));
                    }
                    stv<kNT>(a.x, g, X[u]);
                    stv<kNT>(a.y, g, Y[u]);
                    stv<kNT>(a.prev, g, C);
                }
            }
        }
        if (has_tail) {
            float x = a.x[tail_i], y = a.y[tail_i];
            const float c = distance(x, y);
            const float nw = feed(a.w[tail_i], a.prev[tail_i] - c, M, wmin, wmax);
            a.w[tail_i] = nw;
            ls.add(nw, x, y);
            if (last) {
                a.cur[tail_i] = c;
            } else {
                float dx, dy;
                fish_draw(a.S, a.k0, a.k1, tail_i, s + 1u, dx, dy);
                const float nc = swim(rule, x, y, dx, dy, H, c, nw);
                best = max(best, mag_bits(c - nc));
                a.x[tail_i] = x;
                a.y[tail_i] = y;
                a.prev[tail_i] = c;
            }
        }
        block_sums<kNaive, B>(a, ls, s);
        if (last) {
            if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->last_max = M_sh;
        } else {
            const uint32_t m = block_max<B>(best);
            if (!barrier_max(bar, m, phase, &M_sh)) return;
        }
    }
}

// ---------------------------------------------------------------------------
// Lean persistent kernel: keeps only (x, y, w) live, 24 B/fish per iteration.
// Positions stay one swim behind: sweep s reads the positions before swim s,
// redoes that swim (the same draws and binary32 ops, so the same bits), feeds
// with M_s, adds the partial sums of s, then swims s+1 on a copy only to get
// its max.  Each swim is computed twice, which the VALU can afford; the last
// sweep also writes (prev, cur), leaving the five columns complete.
// ---------------------------------------------------------------------------
template <bool kNaive, bool kNT>
__global__ __launch_bounds__(kFusedBlock) void fused_lean_kernel(SchoolArgs a, FusedArgs f) {
    constexpr int B = kFusedBlock;
    __shared__ uint32_t M_sh;
    const float H = a.H, wmin = a.wmin, wmax = a.wmax;
    const SwimRule rule{a.rule, a.wmin};
    const uint32_t grid = gridDim.x;
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)grid * B;
    const uint64_t gbase = (uint64_t)blockIdx.x * B + threadIdx.x;
    const uint64_t tail_i = 4 * n4 + threadIdx.x;
    const bool has_tail = blockIdx.x == grid - 1 && tail_i < a.n;
    const Barrier bar{a.sync, a.ctrl, f.spin_limit};
    uint32_t phase = 0;

    // Prologue: M_t0 from a look-ahead swim of t0; nothing is stored.
    {
        uint32_t best = 0u;
        for (uint64_t g = gbase; g < n4; g += stride) {
            const float4 X = ldv<kNT>(a.x, g), Y = ldv<kNT>(a.y, g);
            float4 Wt = swim_weights<kNT>(rule, a.w, g);
            float dx[4], dy[4];
            group_draws(a.S, a.k0, a.k1, g, f.t0, dx, dy);
            float4 nx = X, ny = Y;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float c = distance(lane_of(nx, q), lane_of(ny, q));
                const float nc = swim(rule, lane_of(nx, q), lane_of(ny, q), dx[q], dy[q], H, c,
                                      lane_of(Wt, q));
                best = max(best, mag_bits(c - nc));
            }
        }
        if (has_tail) {
            float dx, dy;
            fish_draw(a.S, a.k0, a.k1, tail_i, f.t0, dx, dy);
            float x = a.x[tail_i], y = a.y[tail_i];
            const float c = distance(x, y);
            const float wt = (rule.flags & kSwimWeighted) ? a.w[tail_i] : 1.0f;
            const float nc = swim(rule, x, y, dx, dy, H, c, wt);
            best = max(best, mag_bits(c - nc));
        }
        const uint32_t m = block_max<B>(best);
        if (!barrier_max(bar, m, phase, &M_sh)) return;
    }

    uint32_t M_prev = 0u;  // M of the previous sweep, for its record
    for (uint32_t k = 0; k < f.steps; ++k) {
        const uint32_t s = f.t0 + k;
        const bool last = k + 1 == f.steps;
        const uint32_t M_bits = M_sh;
        const float M = __uint_as_float(M_bits);
        if (k > 0 && blockIdx.x == (s - 1u) % grid) combine_block<B>(a, s - 1u, grid, f.naive, M_prev);
        M_prev = M_bits;

        LaneSums<kNaive> ls;
        uint32_t best = 0u;
        for (uint64_t g0 = gbase; g0 < n4; g0 += kUnroll * stride) {
            float4 X[kUnroll], Y[kUnroll], W[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t g = g0 + u * stride;
                if (g < n4) {
                    X[u] = ldv<kNT>(a.x, g);
                    Y[u] = ldv<kNT>(a.y, g);
                    W[u] = ldv<kNT>(a.w, g);
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t g = g0 + u * stride;
                if (g >= n4) break;
                float dx[4], dy[4];
                group_draws(a.S, a.k0, a.k1, g, s, dx, dy);
                float4 C0, C1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    lane_of(C0, q) = distance(lane_of(X[u], q), lane_of(Y[u], q));
                    lane_of(C1, q) = swim(rule, lane_of(X[u], q), lane_of(Y[u], q), dx[q], dy[q],
                                          H, lane_of(C0, q), lane_of(W[u], q));
                    const float diff = lane_of(C0, q) - lane_of(C1, q);
                    lane_of(W[u], q) = feed(lane_of(W[u], q), diff, M, wmin, wmax);
                }
                ls.add4(W[u], X[u], Y[u]);
                stv<kNT>(a.x, g, X[u]);
                stv<kNT>(a.y, g, Y[u]);
                stv<kNT>(a.w, g, W[u]);
                if (last) {
                    stv<kNT>(a.prev, g, C0);
                    stv<kNT>(a.cur, g, C1);
                } else {
                    group_draws(a.S, a.k0, a.k1, g, s + 1u, dx, dy);
                    float4 nx = X[u], ny = Y[u];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float nc = swim(rule, lane_of(nx, q), lane_of(ny, q), dx[q], dy[q],
                                              H, lane_of(C1, q), lane_of(W[u], q));
                        best = max(best, mag_bits(lane_of(C1, q) - nc));
                    }
                }
            }
        }
        if (has_tail) {
            float dx, dy;
            fish_draw(a.S, a.k0, a.k1, tail_i, s, dx, dy);
            float x = a.x[tail_i], y = a.y[tail_i];
            const float w0 = a.w[tail_i];
            const float c0 = distance(x, y);
            const float c1 = swim(rule, x, y, dx, dy, H, c0, w0);
            const float nw = feed(w0, c0 - c1, M, wmin, wmax);
            a.x[tail_i] = x;
            a.y[tail_i] = y;
            a.w[tail_i] = nw;
            ls.add(nw, x, y);
            if (last) {
                a.prev[tail_i] = c0;
                a.cur[tail_i] = c1;
            } else {
                fish_draw(a.S, a.k0, a.k1, tail_i, s + 1u, dx, dy);
                const float nc = swim(rule, x, y, dx, dy, H, c1, nw);
                best = max(best, mag_bits(c1 - nc));
            }
        }
        block_sums<kNaive, B>(a, ls, s);
        if (last) {
            if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->last_max = M_sh;
        } else {
            const uint32_t m = block_max<B>(best);
            if (!barrier_max(bar, m, phase, &M_sh)) return;
        }
    }
}

// ---------------------------------------------------------------------------
// Deep persistent kernel: KD iterations per grid barrier.  Without the
// weighted rule a fish's positions do not depend on its weight (the draws
// depend on (seed, fish, t) only, and the greedy test on objectives only), so
// the differences of KD iterations ahead can be formed before any of their
// maxima is known.  A superstep of kd <= KD iterations s0 .. s0 + kd - 1
// reads (x, y, w, cur) once: it replays swims s0 .. s0 + kd - 1 from the
// stored positions, feeding with the maxima M_s0 .. published by the previous
// barrier and adding each iteration's partial sums; then, from a copy of the
// final positions, it swims the next superstep's iterations only for their
// maxima; it writes (x, y, w, cur) once.  cur carries the objective of the
// stored positions from one superstep to the next, which saves forming it
// again (a square root per fish and superstep) for 8 B; the first superstep
// of a launch forms it from the positions.  One barrier reduces all the
// maxima.  Columns: 32 B per fish per superstep, 32 / KD per fish-iteration;
// each swim is computed twice, as in the lean kernel.  Every operation of a fish is the
// plain path's, in the same order, so the bits are the same.  Compensated
// sums only; the host never picks it under the weighted rule.  The rule is a
// template argument (kRule: 0 or kSwimGreedy), so the plain swim carries no
// run-time tests or selects of the other rules.  Blocks of 512 threads for
// KD = 8 (two waves per SIMD, 256 registers each: the eight unrolled swims and
// eight sets of lane sums take ~230) and of 768 threads for KD <= 4 (three
// waves per SIMD, at most 168 registers: four take ~150).
// ---------------------------------------------------------------------------
template <int KD>
constexpr int kDeepBlockOf = KD == 8 ? 512 : 768;

template <int KD, bool kNT, uint32_t kRule>
__global__ __launch_bounds__(kDeepBlockOf<KD>) void fused_deep_kernel(SchoolArgs a, FusedArgs f) {
    static_assert((kRule & kSwimWeighted) == 0, "the deep kernel never runs the weighted rule");
    constexpr int B = kDeepBlockOf<KD>;
    __shared__ uint32_t M_sh[KD];
    const float H = a.H, wmin = a.wmin, wmax = a.wmax;
    const SwimRule rule{kRule, a.wmin};
    const uint32_t grid = gridDim.x;
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)grid * B;
    const uint64_t gbase = (uint64_t)blockIdx.x * B + threadIdx.x;
    const uint64_t tail_i = 4 * n4 + threadIdx.x;
    const bool has_tail = blockIdx.x == grid - 1 && tail_i < a.n;
    const Barrier bar{a.sync, a.ctrl, f.spin_limit};
    uint32_t phase = 0;

    // Look-ahead maxima of iterations t .. t + kd - 1 from positions (x, y)
    // with objective c, into best[] (nothing is stored).
    auto look_ahead = [&](float x, float y, float c, uint64_t fish, uint32_t t, uint32_t kd,
                          uint32_t (&best)[KD]) {
#pragma unroll
        for (int j = 0; j < KD; ++j) {
            if ((uint32_t)j >= kd) break;
            float dx, dy;
            fish_draw(a.S, a.k0, a.k1, fish, t + j, dx, dy);
            const float nc = swim(rule, x, y, dx, dy, H, c, 1.0f);
            best[j] = max(best[j], mag_bits(c - nc));
            c = nc;
        }
    };

    // Exact maxima of iterations t .. t + kd0 - 1 from the stored positions,
    // reduced by one grid barrier: the prologue's, and the recomputation when
    // a skip test guessed too high (below).
    auto exact_maxima = [&](uint32_t t, uint32_t kd0) -> bool {
        uint32_t best[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) best[j] = 0u;
        for (uint64_t g = gbase; g < n4; g += stride) {
            float4 X = ldv<kNT>(a.x, g), Y = ldv<kNT>(a.y, g);
            float4 C;
#pragma unroll
            for (int q = 0; q < 4; ++q) lane_of(C, q) = distance(lane_of(X, q), lane_of(Y, q));
#pragma unroll
            for (int j = 0; j < KD; ++j) {
                if ((uint32_t)j >= kd0) break;
                float dx[4], dy[4];
                group_draws(a.S, a.k0, a.k1, g, t + j, dx, dy);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float nc = swim(rule, lane_of(X, q), lane_of(Y, q), dx[q], dy[q], H,
                                          lane_of(C, q), 1.0f);
                    best[j] = max(best[j], mag_bits(lane_of(C, q) - nc));
                    lane_of(C, q) = nc;
                }
            }
        }
        if (has_tail) {
            const float x = a.x[tail_i], y = a.y[tail_i];
            look_ahead(x, y, distance(x, y), tail_i, t, kd0, best);
        }
        uint32_t m[KD];
        block_max_k<KD, B>(best, m);
        return barrier_maxima<KD>(bar, m, phase, M_sh);
    };
    if (!exact_maxima(f.t0, min((uint32_t)KD, f.steps))) return;

    uint32_t M_prev[KD];
    uint32_t kd_prev = 0;
    for (uint32_t k0 = 0; k0 < f.steps; k0 += KD) {
        const uint32_t s0 = f.t0 + k0;
        const uint32_t kd = min((uint32_t)KD, f.steps - k0);
        const uint32_t kd_next = min((uint32_t)KD, f.steps - k0 - kd);
        const bool last = kd_next == 0;
        float M[KD];
        uint32_t M_bits[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) {
            M_bits[j] = uniform(M_sh[j]);
            M[j] = __uint_as_float(M_bits[j]);
        }
        // Records of the previous superstep, each by a rotating block.
        for (uint32_t j = 0; j < kd_prev; ++j) {
            const uint32_t t = s0 - kd_prev + j;
            if (blockIdx.x == t % grid) combine_block<B>(a, t, grid, 0u, M_prev[j], true);
        }
#pragma unroll
        for (int j = 0; j < KD; ++j) M_prev[j] = M_bits[j];
        kd_prev = kd;

        // Under the plain swim, the look-ahead forms a fish's objectives only
        // when its move could reach T, a guess just below this superstep's
        // maxima (the maxima of a large school change little between
        // iterations); the other fish cannot carry the maxima if these are at
        // least T, which the barrier's published maxima then show, else they
        // are recomputed exactly.
        bool filtered = false;
        float T = 0.0f, skip_limit = 0.0f;
        if constexpr (kRule == 0) {
            if (f.look_theta > 0.0f && !last) {
                float m_min = M[0];
#pragma unroll
                for (int j = 1; j < KD; ++j)
                    if ((uint32_t)j < kd) m_min = fminf(m_min, M[j]);
                T = f.look_theta * m_min;
                skip_limit = look_skip_limit(T, H, a.S);
                filtered = true;
            }
        }

        LaneSumsF64 ls[KD];
        uint32_t best[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) best[j] = 0u;
        for (uint64_t g = gbase; g < n4; g += stride) {
            float4 X = ldv<kNT>(a.x, g), Y = ldv<kNT>(a.y, g), W = ldv<kNT>(a.w, g);
            float4 C, P;
            if (k0 == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) lane_of(C, q) = distance(lane_of(X, q), lane_of(Y, q));
            } else {
                C = ldv<kNT>(a.cur, g);  // stored by the previous superstep (below)
            }
#pragma unroll
            for (int j = 0; j < KD; ++j) {
                if ((uint32_t)j >= kd) break;
                float dx[4], dy[4];
                group_draws(a.S, a.k0, a.k1, g, s0 + j, dx, dy);
                P = C;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    lane_of(C, q) = swim(rule, lane_of(X, q), lane_of(Y, q), dx[q], dy[q], H,
                                         lane_of(P, q), 1.0f);
                    lane_of(W, q) = feed(lane_of(W, q), lane_of(P, q) - lane_of(C, q), M[j], wmin,
                                         wmax);
                }
                ls[j].add4(W, X, Y);
            }
            stv<kNT>(a.x, g, X);
            stv<kNT>(a.y, g, Y);
            stv<kNT>(a.w, g, W);
            stv<kNT>(a.cur, g, C);
            if (last) {
                stv<kNT>(a.prev, g, P);
            } else if (filtered) {
                // The plain swim's own operations; C[q] is the objective of
                // the current position only while fresh[q] holds.
                bool fresh[4] = {true, true, true, true};
#pragma unroll
                for (int j = 0; j < KD; ++j) {
                    if ((uint32_t)j >= kd_next) break;
                    float dx[4], dy[4];
                    group_draws(a.S, a.k0, a.k1, g, s0 + kd + j, dx, dy);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float ox = lane_of(X, q), oy = lane_of(Y, q);
                        lane_of(X, q) = clamp_to(ox + dx[q], -H, H);
                        lane_of(Y, q) = clamp_to(oy + dy[q], -H, H);
                        if (__builtin_fmaf(dx[q], dx[q], dy[q] * dy[q]) >= skip_limit) {
                            float oc = lane_of(C, q);
                            if (!fresh[q]) oc = distance(ox, oy);
                            const float nc = distance(lane_of(X, q), lane_of(Y, q));
                            best[j] = max(best[j], mag_bits(oc - nc));
                            lane_of(C, q) = nc;
                            fresh[q] = true;
                        } else {
                            fresh[q] = false;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < KD; ++j) {
                    if ((uint32_t)j >= kd_next) break;
                    float dx[4], dy[4];
                    group_draws(a.S, a.k0, a.k1, g, s0 + kd + j, dx, dy);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float nc = swim(rule, lane_of(X, q), lane_of(Y, q), dx[q], dy[q], H,
                                              lane_of(C, q), 1.0f);
                        best[j] = max(best[j], mag_bits(lane_of(C, q) - nc));
                        lane_of(C, q) = nc;
                    }
                }
            }
        }
        if (has_tail) {
            float x = a.x[tail_i], y = a.y[tail_i], w = a.w[tail_i];
            float c = distance(x, y), p = c;
#pragma unroll
            for (int j = 0; j < KD; ++j) {
                if ((uint32_t)j >= kd) break;
                float dx, dy;
                fish_draw(a.S, a.k0, a.k1, tail_i, s0 + j, dx, dy);
                p = c;
                c = swim(rule, x, y, dx, dy, H, p, 1.0f);
                w = feed(w, p - c, M[j], wmin, wmax);
                ls[j].add(w, x, y);
            }
            a.x[tail_i] = x;
            a.y[tail_i] = y;
            a.w[tail_i] = w;
            if (last) {
                a.prev[tail_i] = p;
                a.cur[tail_i] = c;
            } else {
                look_ahead(x, y, c, tail_i, s0 + kd, kd_next, best);
            }
        }
        block_sums_deep<KD, B>(a, ls, s0, kd);
        // The barrier that ends the superstep: the next maxima (none after the
        // last superstep, whose barrier only makes its partials visible).
        uint32_t m[KD];
        block_max_k<KD, B>(best, m);
        if (!barrier_maxima<KD>(bar, m, phase, M_sh)) return;
        if (filtered) {
            // Every skipped fish's |diff| is below T: a published maximum of at
            // least T is exact.  Any below T: recompute them all exactly (the
            // same decision in every block: all see the same published words).
            bool redo = false;
            for (uint32_t j = 0; j < kd_next; ++j) redo |= __uint_as_float(M_sh[j]) < T;
            if (redo && !exact_maxima(s0 + kd, kd_next)) return;
        }
        if (last) {
            for (uint32_t j = 0; j < kd; ++j) {
                const uint32_t t = s0 + j;
                if (blockIdx.x == t % grid) combine_block<B>(a, t, grid, 0u, M_prev[j], true);
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->last_max = M_prev[kd - 1];
        }
    }
}

// ---------------------------------------------------------------------------
// Register-resident persistent kernel: for schools small enough, every fish's
// (x, y, w, prev, cur) stays in registers for the whole launch, so an
// iteration moves no column bytes at all: the columns are read once at the
// start and written once at the end.  Thread i of the grid holds groups
// i, i + T, ..., i + (KG - 1) T (T threads in the grid; groups past the end
// are skipped).  Like the 32-byte variant, sweep s feeds with M_s from the
// stored prev and cur, then swims s+1 for M_{s+1}; cur is the look-ahead
// swim's own result, so each fish-iteration costs one draw and one square
// root.  The tail fish (n mod 4) go through memory as in fused_kernel.
// Blocks of 512 threads, one per CU: two waves per SIMD, so each thread may
// use 256 registers.  Four groups (80 registers of state) compile to 209
// registers with no spill; eight would spill.
// ---------------------------------------------------------------------------
constexpr int kRegsBlock = 512;
constexpr uint32_t kRegsMaxGroups = 4;

template <int KG, bool kNaive>
__global__ __launch_bounds__(kRegsBlock) void fused_regs_kernel(SchoolArgs a, FusedArgs f) {
    constexpr int B = kRegsBlock;
    __shared__ uint32_t M_sh;
    const float H = a.H, wmin = a.wmin, wmax = a.wmax;
    const SwimRule rule{a.rule, a.wmin};
    const uint32_t grid = gridDim.x;
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)grid * B;
    const uint64_t gbase = (uint64_t)blockIdx.x * B + threadIdx.x;
    const uint64_t tail_i = 4 * n4 + threadIdx.x;
    const bool has_tail = blockIdx.x == grid - 1 && tail_i < a.n;
    const Barrier bar{a.sync, a.ctrl, f.spin_limit};
    uint32_t phase = 0;

    float4 X[KG], Y[KG], W[KG], P[KG], C[KG];
    // Prologue: load, swim t0 (P = objective before it, C = after), M_t0.
    {
        uint32_t best = 0u;
#pragma unroll
        for (int j = 0; j < KG; ++j) {
            const uint64_t g = gbase + j * stride;
            if (g >= n4) break;
            X[j] = ldv<false>(a.x, g);
            Y[j] = ldv<false>(a.y, g);
            W[j] = ldv<false>(a.w, g);
            float dx[4], dy[4];
            group_draws(a.S, a.k0, a.k1, g, f.t0, dx, dy);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lane_of(P[j], q) = distance(lane_of(X[j], q), lane_of(Y[j], q));
                lane_of(C[j], q) = swim(rule, lane_of(X[j], q), lane_of(Y[j], q), dx[q], dy[q], H,
                                        lane_of(P[j], q), lane_of(W[j], q));
                best = max(best, mag_bits(lane_of(P[j], q) - lane_of(C[j], q)));
            }
        }
        if (has_tail) {
            float dx, dy;
            fish_draw(a.S, a.k0, a.k1, tail_i, f.t0, dx, dy);
            float x = a.x[tail_i], y = a.y[tail_i];
            const float c = distance(x, y);
            const float wt = (rule.flags & kSwimWeighted) ? a.w[tail_i] : 1.0f;
            const float nc = swim(rule, x, y, dx, dy, H, c, wt);
            best = max(best, mag_bits(c - nc));
            a.x[tail_i] = x;
            a.y[tail_i] = y;
            a.prev[tail_i] = c;
        }
        const uint32_t m = block_max<B>(best);
        if (!barrier_max(bar, m, phase, &M_sh)) return;
    }

    uint32_t M_prev = 0u;  // M of the previous sweep, for its record
    for (uint32_t k = 0; k < f.steps; ++k) {
        const uint32_t s = f.t0 + k;
        const bool last = k + 1 == f.steps;
        const uint32_t M_bits = M_sh;
        const float M = __uint_as_float(M_bits);
        if (k > 0 && blockIdx.x == (s - 1u) % grid) combine_block<B>(a, s - 1u, grid, f.naive, M_prev);
        M_prev = M_bits;

        LaneSums<kNaive> ls;
        uint32_t best = 0u;
#pragma unroll
        for (int j = 0; j < KG; ++j) {
            const uint64_t g = gbase + j * stride;
            if (g >= n4) break;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                lane_of(W[j], q) = feed(lane_of(W[j], q), lane_of(P[j], q) - lane_of(C[j], q), M,
                                        wmin, wmax);
            ls.add4(W[j], X[j], Y[j]);
            if (last) {
                stv<false>(a.x, g, X[j]);
                stv<false>(a.y, g, Y[j]);
                stv<false>(a.w, g, W[j]);
                stv<false>(a.prev, g, P[j]);
                stv<false>(a.cur, g, C[j]);
            } else {
                float dx[4], dy[4];
                group_draws(a.S, a.k0, a.k1, g, s + 1u, dx, dy);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    lane_of(P[j], q) = lane_of(C[j], q);
                    lane_of(C[j], q) = swim(rule, lane_of(X[j], q), lane_of(Y[j], q), dx[q], dy[q],
                                            H, lane_of(P[j], q), lane_of(W[j], q));
                    best = max(best, mag_bits(lane_of(P[j], q) - lane_of(C[j], q)));
                }
            }
        }
        if (has_tail) {
            float x = a.x[tail_i], y = a.y[tail_i];
            const float c = distance(x, y);
            const float nw = feed(a.w[tail_i], a.prev[tail_i] - c, M, wmin, wmax);
            a.w[tail_i] = nw;
            ls.add(nw, x, y);
            if (last) {
                a.cur[tail_i] = c;
            } else {
                float dx, dy;
                fish_draw(a.S, a.k0, a.k1, tail_i, s + 1u, dx, dy);
                const float nc = swim(rule, x, y, dx, dy, H, c, nw);
                best = max(best, mag_bits(c - nc));
                a.x[tail_i] = x;
                a.y[tail_i] = y;
                a.prev[tail_i] = c;
            }
        }
        block_sums<kNaive, B>(a, ls, s);
        if (last) {
            if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->last_max = M_sh;
        } else {
            const uint32_t m = block_max<B>(best);
            if (!barrier_max(bar, m, phase, &M_sh)) return;
        }
    }
}

// Instrumentation: f.steps barriers of the persistent kernels' kind with no
// other work, each folding max(block index + k) over the grid, so the
// synchronisation a persistent iteration adds can be timed on its own (and
// its max checked: grid - 1 + f.steps - 1 after the last one).
__global__ __launch_bounds__(kFusedBlock) void barrier_probe_kernel(SchoolArgs a, FusedArgs f) {
    __shared__ uint32_t M_sh;
    const Barrier bar{a.sync, a.ctrl, f.spin_limit};
    uint32_t phase = 0;
    for (uint32_t k = 0; k < f.steps; ++k)
        if (!barrier_max(bar, blockIdx.x + k, phase, &M_sh)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->probe_max = M_sh;
}

// The kernels' square root over an array (instrumentation and tests).
__global__ __launch_bounds__(kBlock) void eval_sqrt_kernel(const float* in, float* out,
                                                            uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        out[i] = sqrt_rn(in[i]);
}

// Clears the barrier's words before a persistent launch (barrier numbers
// restart at 1 in every launch).
__global__ void reset_sync_kernel(uint32_t* sync) {
    for (uint32_t i = threadIdx.x; i < kSyncWords; i += blockDim.x) sync[i] = 0u;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point.  In host code the array's name
// is only a stand-in for the symbol: kernels get the device address that
// hipGetSymbolAddress returns for the current device, never the name itself.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // with device `dev` current
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

__global__ void copy_error_kernel(const Ctrl* ctrl, uint32_t* out) {
    if (threadIdx.x == 0) *out = ctrl->error;
}

hipError_t launch_copy_error(const SchoolArgs& a, uint32_t* out, hipStream_t stream) {
    hipLaunchKernelGGL(copy_error_kernel, dim3(1), dim3(64), 0, stream, a.ctrl, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static uint32_t capped_grid(uint64_t n, uint32_t cap) {
    const uint64_t groups = n >> 2;
    uint64_t g = (groups + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

uint32_t plain_grid(uint64_t n) { return capped_grid(n, kSwimGridCap); }
uint32_t feed_grid(uint64_t n) { return capped_grid(n, kFeedGridCap); }
uint32_t pipe_grid(uint64_t n) { return capped_grid(n, kPipeGridCap); }

hipError_t launch_reset(const SchoolArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, stream, a.ctrl);
    return hipGetLastError();
}

hipError_t launch_init(const SchoolArgs& a, float wlo, float whi, hipStream_t stream) {
    InitArgs ia{a, wlo, whi};
    hipLaunchKernelGGL(init_kernel, dim3(plain_grid(a.n)), dim3(kBlock), 0, stream, ia);
    return hipGetLastError();
}

// Footprint rule of the plain passes' cache policy (256 MiB last-level cache).
constexpr uint64_t kLastLevelCache = 256ull << 20;

int plain_policy(uint64_t n) {
    if (n * 16ull <= kLastLevelCache) return kCached;
    if (n * 12ull <= kLastLevelCache) return kStreamW;
    return kStreamAll;
}

template <bool kInject, bool kCritical>
const void* swim_fn(int pol) {
    switch (pol) {
        case kCached:
            return reinterpret_cast<const void*>(swim_eval_kernel<kInject, kCached, kCritical>);
        case kStreamW:
            return reinterpret_cast<const void*>(swim_eval_kernel<kInject, kStreamW, kCritical>);
        default:
            return reinterpret_cast<const void*>(swim_eval_kernel<kInject, kStreamAll, kCritical>);
    }
}

template <int kRed, bool kWriteCur>
const void* feed_fn(int pol) {
    switch (pol) {
        case kCached:
            return reinterpret_cast<const void*>(feed_bary_kernel<kRed, kCached, kWriteCur>);
        case kStreamW:
            return reinterpret_cast<const void*>(feed_bary_kernel<kRed, kStreamW, kWriteCur>);
        default:
            return reinterpret_cast<const void*>(feed_bary_kernel<kRed, kStreamAll, kWriteCur>);
    }
}

template <bool kNaive>
const void* feed_swim_fn(int pol) {
    switch (pol) {
        case kCached: return reinterpret_cast<const void*>(feed_swim_kernel<kNaive, kCached>);
        case kStreamW: return reinterpret_cast<const void*>(feed_swim_kernel<kNaive, kStreamW>);
        default: return reinterpret_cast<const void*>(feed_swim_kernel<kNaive, kStreamAll>);
    }
}

// With start and stop events, the launch itself records them (hipExtLaunchKernel):
// the elapsed time is the kernel's own, with no marker packets of its own in
// the stream to stretch it.
hipError_t launch_plain(const void* fn, uint32_t grid, const SchoolArgs& a, const StepArgs& s,
                        hipStream_t stream, hipEvent_t start, hipEvent_t stop) {
    SchoolArgs aa = a;
    StepArgs ss = s;
    void* args[] = {&aa, &ss};
    if (start && stop)
        return hipExtLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, stream, start, stop, 0);
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, stream);
}

hipError_t launch_swim_eval(const SchoolArgs& a, const StepArgs& s, hipStream_t stream,
                            hipEvent_t start, hipEvent_t stop) {
    const int pol = plain_policy(a.n);
    const void* fn = s.critical ? (s.dx ? swim_fn<true, true>(pol) : swim_fn<false, true>(pol))
                                : (s.dx ? swim_fn<true, false>(pol) : swim_fn<false, false>(pol));
    return launch_plain(fn, s.swim_grid, a, s, stream, start, stop);
}

hipError_t launch_feed_bary(const SchoolArgs& a, const StepArgs& s, uint32_t grid,
                            hipStream_t stream, hipEvent_t start, hipEvent_t stop,
                            bool write_cur) {
    const int pol = plain_policy(a.n);
    if (s.critical && write_cur) return hipErrorInvalidValue;  // critical runs never pipeline
    const void* fn = s.critical ? feed_fn<kRedCritical, false>(pol)
                     : s.naive  ? (write_cur ? feed_fn<kRedNaive, true>(pol)
                                             : feed_fn<kRedNaive, false>(pol))
                                : (write_cur ? feed_fn<kRedCompensated, true>(pol)
                                             : feed_fn<kRedCompensated, false>(pol));
    return launch_plain(fn, grid, a, s, stream, start, stop);
}

hipError_t launch_feed_swim(const SchoolArgs& a, const StepArgs& s, uint32_t grid,
                            hipStream_t stream, hipEvent_t start, hipEvent_t stop) {
    if (s.critical || s.dx || s.t == 0) return hipErrorInvalidValue;
    const int pol = plain_policy(a.n);
    const void* fn = s.naive ? feed_swim_fn<true>(pol) : feed_swim_fn<false>(pol);
    return launch_plain(fn, grid, a, s, stream, start, stop);
}

hipError_t launch_combine(const SchoolArgs& a, uint32_t t, uint32_t grid, uint32_t naive,
                          hipStream_t stream) {
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(kBlock), 0, stream, a, t, grid, naive);
    return hipGetLastError();
}

template <bool kNaive, bool kNT>
const void* fused_fn(uint32_t lean) {
    return lean ? reinterpret_cast<const void*>(fused_lean_kernel<kNaive, kNT>)
                : reinterpret_cast<const void*>(fused_kernel<kNaive, kNT>);
}

const void* pick_fused(uint32_t naive, uint32_t streaming, uint32_t lean) {
    if (naive) return streaming ? fused_fn<true, true>(lean) : fused_fn<true, false>(lean);
    return streaming ? fused_fn<false, true>(lean) : fused_fn<false, false>(lean);
}

template <bool kNT, uint32_t kRule>
const void* deep_fn(uint32_t depth) {
    switch (depth) {
        case 2: return reinterpret_cast<const void*>(fused_deep_kernel<2, kNT, kRule>);
        case 4: return reinterpret_cast<const void*>(fused_deep_kernel<4, kNT, kRule>);
        default: return reinterpret_cast<const void*>(fused_deep_kernel<8, kNT, kRule>);
    }
}

// The deep kernel of a cache policy, depth and swim rule (greedy or plain;
// the host never asks for the weighted rule).
const void* pick_deep(uint32_t streaming, uint32_t depth, uint32_t rule) {
    if (rule & kSwimGreedy)
        return streaming ? deep_fn<true, kSwimGreedy>(depth) : deep_fn<false, kSwimGreedy>(depth);
    return streaming ? deep_fn<true, 0u>(depth) : deep_fn<false, 0u>(depth);
}

hipError_t deep_resident_grid(uint32_t depth, uint32_t* out_grid) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int per_cu = 1 << 30;
    for (uint32_t nt = 0; nt < 2; ++nt)  // both cache policies and both rules must fit
        for (uint32_t rule : {0u, kSwimGreedy}) {
            int b = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, pick_deep(nt, depth, rule),
                                                             (int)deep_block(depth), 0);
            if (e != hipSuccess) return e;
            per_cu = b < per_cu ? b : per_cu;
        }
    uint64_t g = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 0);
    if (g > kMaxBarrierBlocks) g = kMaxBarrierBlocks;
    *out_grid = (uint32_t)g;
    return hipSuccess;
}

uint32_t deep_grid(uint64_t n, uint32_t depth, uint32_t resident) {
    const uint64_t block = deep_block(depth);
    uint64_t g = ((n >> 2) + block - 1) / block;
    if (g < 1) g = 1;
    if (g > resident) g = resident;
    return (uint32_t)g;
}

float look_theta(uint64_t n) {
    static const int mode = [] {
        const char* v = std::getenv("FSB_LOOKAHEAD_FILTER");
        if (v && std::strcmp(v, "off") == 0) return 0;
        if (v && std::strcmp(v, "redo") == 0) return 2;
        return 1;
    }();
    if (mode == 0) return 0.0f;
    if (mode == 2) return 2.0f;
    return n >= kLookFilterFish ? kLookTheta : 0.0f;
}

uint32_t deep_depth(uint64_t n) {
    static const uint32_t forced = [] {
        const char* v = std::getenv("FSB_DEEP_DEPTH");
        const unsigned long d = v && *v ? std::strtoul(v, nullptr, 10) : 0;
        return d == 2 || d == 4 || d == 8 ? (uint32_t)d : 0u;
    }();
    if (forced) return forced;
    return n > kDeepWideFish ? 4u : 8u;
}

template <bool kNaive>
const void* regs_fn(uint32_t groups) {
    switch (groups) {
        case 1: return reinterpret_cast<const void*>(fused_regs_kernel<1, kNaive>);
        case 2: return reinterpret_cast<const void*>(fused_regs_kernel<2, kNaive>);
        default: return reinterpret_cast<const void*>(fused_regs_kernel<4, kNaive>);
    }
}

const void* pick_regs(uint32_t naive, uint32_t groups) {
    return naive ? regs_fn<true>(groups) : regs_fn<false>(groups);
}

hipError_t regs_resident_grid(uint32_t naive, uint32_t* out_grid) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int per_cu = 1 << 30;
    for (uint32_t groups : {1u, 2u, 4u}) {  // every instance must fit
        int b = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, pick_regs(naive, groups), kRegsBlock,
                                                         0);
        if (e != hipSuccess) return e;
        per_cu = b < per_cu ? b : per_cu;
    }
    uint64_t g = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 0);
    if (g > kMaxBarrierBlocks) g = kMaxBarrierBlocks;
    if (g > kMaxGrid) g = kMaxGrid;
    *out_grid = (uint32_t)g;
    return hipSuccess;
}

uint32_t regs_plan(uint64_t n, uint32_t resident, uint32_t* groups) {
    const uint64_t n4 = n >> 2;
    *groups = 0;
    if (resident == 0) return 0;
    const uint64_t threads = (uint64_t)resident * kRegsBlock;
    const uint64_t per = (n4 + threads - 1) / threads;  // groups per thread needed
    if (per > kRegsMaxGroups) return 0;
    uint32_t kg = 1;
    while (kg < per) kg *= 2;
    uint64_t g = (n4 + (uint64_t)kg * kRegsBlock - 1) / ((uint64_t)kg * kRegsBlock);
    if (g < 1) g = 1;
    if (g > resident) g = resident;
    *groups = kg;
    return (uint32_t)g;
}

hipError_t fused_resident_grid(uint32_t naive, uint32_t* out_grid) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int per_cu = 1 << 30;
    for (uint32_t v = 0; v < 4; ++v) {  // every variant must fit
        int b = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, pick_fused(naive, v & 1, v >> 1),
                                                         kFusedBlock, 0);
        if (e != hipSuccess) return e;
        per_cu = b < per_cu ? b : per_cu;
    }

    uint64_t g = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 0);
    if (g > kMaxBarrierBlocks) g = kMaxBarrierBlocks;
    if (g > kMaxGrid) g = kMaxGrid;
    *out_grid = (uint32_t)g;
    return hipSuccess;
}

uint32_t fused_grid(uint64_t n, uint32_t resident) {
    const uint64_t groups = n >> 2;
    uint64_t g = (groups + kFusedBlock - 1) / kFusedBlock;
    if (g < 1) g = 1;
    if (g > resident) g = resident;
    return (uint32_t)g;
}

uint32_t barrier_spin_limit() {
    static const uint32_t limit = [] {
        const char* v = std::getenv("FSB_BARRIER_SPIN_LIMIT");
        if (!v || !*v) return kBarrierSpinLimit;
        const unsigned long x = std::strtoul(v, nullptr, 10);
        return x >= 1 && x <= kBarrierSpinLimit ? (uint32_t)x : kBarrierSpinLimit;
    }();
    return limit;
}

hipError_t launch_persistent(const void* fn, dim3 grid, dim3 block, void** args,
                             hipStream_t stream) {
    static const bool regular = [] {
        const char* v = std::getenv("FSB_PERSISTENT_LAUNCH");
        return v && std::strcmp(v, "regular") == 0;
    }();
    if (regular) return hipLaunchKernel(fn, grid, block, args, 0, stream);
    return hipLaunchCooperativeKernel(fn, grid, block, args, 0, stream);
}

hipError_t launch_eval_sqrt(const float* in, float* out, uint64_t n, hipStream_t stream) {
    uint64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(eval_sqrt_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, stream, in, out, n);
    return hipGetLastError();
}

hipError_t launch_barrier_probe(const SchoolArgs& a, const FusedArgs& f, uint32_t grid,
                                hipStream_t stream) {
    hipLaunchKernelGGL(reset_sync_kernel, dim3(1), dim3(256), 0, stream, a.sync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SchoolArgs sa = a;
    FusedArgs fa = f;
    void* args[] = {&sa, &fa};
    return launch_persistent(reinterpret_cast<const void*>(barrier_probe_kernel), dim3(grid),
                             dim3(kFusedBlock), args, stream);
}

hipError_t launch_fused(const SchoolArgs& a, const FusedArgs& f, uint32_t grid,
                        hipStream_t stream) {
    hipLaunchKernelGGL(reset_sync_kernel, dim3(1), dim3(256), 0, stream, a.sync);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SchoolArgs sa = a;
    FusedArgs fa = f;
    void* args[] = {&sa, &fa};
    const void* fn = f.regs   ? pick_regs(f.naive, f.regs)
                     : f.deep ? pick_deep(f.streaming, f.deep, a.rule)
                              : pick_fused(f.naive, f.streaming, f.lean);
    const uint32_t block = f.regs ? kRegsBlock : f.deep ? deep_block(f.deep) : kFusedBlock;
    return launch_persistent(fn, dim3(grid), dim3(block), args, stream);
}

}  // namespace fsb
