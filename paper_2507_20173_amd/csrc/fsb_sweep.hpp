// fsb_sweep.hpp -- pieces shared by the single-school and batched kernels:
// float4 column access, the swim draws of a group of four fish, per-lane
// barycentre sums, and the persistent kernels' grid barrier.
#pragma once

#include "fsb_device.hpp"
#include "fsb_internal.hpp"

namespace fsb {

__device__ __forceinline__ float4 ld4(const float* p, uint64_t g) {
    return reinterpret_cast<const float4*>(p)[g];
}
__device__ __forceinline__ void st4(float* p, uint64_t g, float4 v) {
    reinterpret_cast<float4*>(p)[g] = v;
}
__device__ __forceinline__ float& lane_of(float4& v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Column access, non-temporal when the live state outgrows the cache.
template <bool kNT>
__device__ __forceinline__ float4 ldv(const float* p, uint64_t g) {
    if constexpr (kNT) {
        const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p) + g);
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return ld4(p, g);
    }
}
template <bool kNT>
__device__ __forceinline__ void stv(float* p, uint64_t g, float4 v) {
    if constexpr (kNT) {
        const v4f w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<v4f*>(p) + g);
    } else {
        st4(p, g, v);
    }
}

// Weights a swim of group g reads: the w column under the weighted rule
// (otherwise they are not used).
template <bool kNT>
__device__ __forceinline__ float4 swim_weights(const SwimRule& r, const float* w, uint64_t g) {
    if (r.flags & kSwimWeighted) return ldv<kNT>(w, g);
    return make_float4(1.0f, 1.0f, 1.0f, 1.0f);
}

// Swim displacements of the four fish of group g (fish 4g..4g+3 of a school
// with key (k0, k1)) at iteration t: pairs 2g and 2g+1.
__device__ __forceinline__ void group_draws(float S, uint32_t k0, uint32_t k1, uint64_t g,
                                            uint32_t t, float dx[4], float dy[4]) {
    const Words p0 = pair_words(2 * g, t, kDomainSwim, k0, k1);
    const Words p1 = pair_words(2 * g + 1, t, kDomainSwim, k0, k1);
    const float S23 = S * 0x1p-23f, nS = -S;
    dx[0] = swim_delta(S23, nS, p0.r0); dy[0] = swim_delta(S23, nS, p0.r1);
    dx[1] = swim_delta(S23, nS, p0.r2); dy[1] = swim_delta(S23, nS, p0.r3);
    dx[2] = swim_delta(S23, nS, p1.r0); dy[2] = swim_delta(S23, nS, p1.r1);
    dx[3] = swim_delta(S23, nS, p1.r2); dy[3] = swim_delta(S23, nS, p1.r3);
}

// Swim displacement of fish i of a school at iteration t.
__device__ __forceinline__ void fish_draw(float S, uint32_t k0, uint32_t k1, uint64_t i,
                                          uint32_t t, float& dx, float& dy) {
    const Words p = pair_words(i >> 1, t, kDomainSwim, k0, k1);
    const bool odd = i & 1;
    const float S23 = S * 0x1p-23f, nS = -S;
    dx = swim_delta(S23, nS, odd ? p.r2 : p.r0);
    dy = swim_delta(S23, nS, odd ? p.r3 : p.r1);
}

// Per-lane sums of the barycentre: compensated (TwoSum) or plain float32.
template <bool kNaive>
struct LaneSums {
    CSum c[3] = {{0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}};
    float f[3] = {0.0f, 0.0f, 0.0f};
    // One fish.
    __device__ __forceinline__ void add(float w, float x, float y) {
        const float wx = w * x;
        const float wy = w * y;
        if constexpr (kNaive) {
            f[0] += w;
            f[1] += wx;
            f[2] += wy;
        } else {
            csum_add(c[0], w);
            csum_add(c[1], wx);
            csum_add(c[2], wy);
        }
    }
    // The four fish of a float4 group.  Compensated: each sum's four terms are
    // added pairwise in binary32, (t0 + t1) + (t2 + t3), so every term passes
    // two roundings (error at most gamma_2 times the sum of the group's |terms|,
    // gamma_2 = 2u / (1 - 2u)), and the group total then enters the TwoSum
    // accumulator: one TwoSum per group instead of four.  Naive: one by one.
    __device__ __forceinline__ void add4(float4 w, float4 x, float4 y) {
        if constexpr (kNaive) {
            add(w.x, x.x, y.x);
            add(w.y, x.y, y.y);
            add(w.z, x.z, y.z);
            add(w.w, x.w, y.w);
        } else {
            const float wx0 = w.x * x.x, wx1 = w.y * x.y, wx2 = w.z * x.z, wx3 = w.w * x.w;
            const float wy0 = w.x * y.x, wy1 = w.y * y.y, wy2 = w.z * y.z, wy3 = w.w * y.w;
            csum_add(c[0], (w.x + w.y) + (w.z + w.w));
            csum_add(c[1], (wx0 + wx1) + (wx2 + wx3));
            csum_add(c[2], (wy0 + wy1) + (wy2 + wy3));
        }
    }
};

// Skip threshold of the deep kernels' look-ahead.  A plain swim by (dx, dy)
// from objective c to nc changes it by |RN(c - nc)| <= (sqrt(dx^2 + dy^2) + K)
// (1 + u), u = 2^-24, where K bounds every rounding on the way: each
// coordinate sum x + dx rounds by at most u (H + S) (the clamp only shortens
// the move), and each objective RN(sqrt(RN(RN(x^2) + RN(y^2)))) lies within
// 2.01 u r of the true distance r <= H sqrt 2.  So K = u sqrt 2 (H + S) +
// 4.02 u sqrt 2 H, taken here as 1.5 u (5.1 H + S) + 2^-60.  The fish's test
// value q = fma(dx, dx, RN(dy * dy)) is at least (dx^2 + dy^2) (1 - u)^2.
// Hence q < L, L = RD(((T - 2^-60) / (1 + 2u) - K)^2 (1 - 4u)), implies
// |diff| < T: the fish cannot carry a maximum that is at least T.  L = 0 (no
// fish skipped) when T is too small.
__device__ __forceinline__ float look_skip_limit(float T, float H, float S) {
    const double K = 0x1p-24 * 1.5 * (5.1 * (double)H + (double)S) + 0x1p-60;
    const double root = ((double)T - 0x1p-60) / (1.0 + 0x1p-23) - K;
    if (!(root > 0.0)) return 0.0f;
    const double L = root * root * (1.0 - 0x1p-22);
    float Lf = (float)L;
    if ((double)Lf > L) Lf = __uint_as_float(__float_as_uint(Lf) - 1u);  // round down
    return Lf;
}

// A value the caller knows to be the same in every lane, moved to a scalar
// register: the compiler cannot prove that of a value read from memory, and
// would otherwise hold one copy per lane in vector registers.
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// The deep kernels' lane sums: each float4 group's four terms are added
// pairwise in binary32 exactly as in the compensated LaneSums (error at most
// gamma_2 times the group's |terms|), and the group totals are accumulated in
// binary64, whose rounding (2^-53 relative per add) is far below that of the
// group totals themselves: as accurate as the TwoSum accumulator, in two
// instructions per sum instead of seven, in the same two registers.  The
// wave and block merges that follow stay in binary64.
struct LaneSumsF64 {
    double v[3] = {0.0, 0.0, 0.0};
    __device__ __forceinline__ void add(float w, float x, float y) {
        const float wx = w * x;
        const float wy = w * y;
        v[0] += (double)w;
        v[1] += (double)wx;
        v[2] += (double)wy;
    }
    __device__ __forceinline__ void add4(float4 w, float4 x, float4 y) {
        const float wx0 = w.x * x.x, wx1 = w.y * x.y, wx2 = w.z * x.z, wx3 = w.w * x.w;
        const float wy0 = w.x * y.x, wy1 = w.y * y.y, wy2 = w.z * y.z, wy3 = w.w * y.w;
        v[0] += (double)((w.x + w.y) + (w.z + w.w));
        v[1] += (double)((wx0 + wx1) + (wx2 + wx3));
        v[2] += (double)((wy0 + wy1) + (wy2 + wy3));
    }
};

// ---------------------------------------------------------------------------
// Grid barrier of the persistent kernels, which also reduces a max.
//
// No read-modify-write on the path: every wave waits for its own stores,
// then thread 0 of every block but block 0 release-stores {its max, barrier
// number} into its own slot (agent scope).  Wave 0 of block 0 is the
// collector: each lane polls every 64th slot until all carry the barrier
// number, then the wave folds the maxima and lane 0 release-stores {M,
// barrier number} into the publish word, which the waiting blocks poll (one
// load returns both).  Measured on MI355X with 256 blocks of 1024 threads:
// 6.8 us per barrier, against 9.9 us for a two-level tree of same-address
// atomic counters, which serialise.  Waits are bounded: on timeout, or when
// another block has flagged an error, every block leaves the kernel and the
// host reports FSB_ERR_DEVICE.
// ---------------------------------------------------------------------------
// s_waitcnt immediate for vmcnt(0) with expcnt and lgkmcnt left at their
// maxima (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int kWaitVmcnt0 = 0x0F70;

struct Barrier {
    uint32_t* sync;       // kSyncWords words, zeroed before the launch
    Ctrl* ctrl;           // error flags
    uint32_t spin_limit;  // polls before a wait gives up (kBarrierSpinLimit unless overridden)
};

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void max_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t barrier_word(uint32_t number, uint32_t value) {
    return ((uint64_t)number << 32) | value;
}

// Returns false if the launch must be abandoned.  `m` holds this block's KD
// maxima (read by thread 0); on return M_sh[0..KD) hold the grid maxima.
// `phase` counts the barriers this launch has passed (every thread keeps the
// same count; it starts at 0).  Block b's slot for value j is the 64-bit word
// KD * b + j; the publish words are 0..KD.  A release fence followed by
// relaxed stores of the KD words, read by relaxed polls followed by an
// acquire fence, orders everything before the fence for the reader.
template <int KD>
__device__ __forceinline__ bool barrier_maxima(const Barrier& b, const uint32_t (&m)[KD],
                                               uint32_t& phase, uint32_t* M_sh) {
    __shared__ int ok_sh;
    // Every wave waits until its own stores (tile partials, and columns that
    // a later sweep may hand to another block) are acknowledged by the L2:
    // the workgroup barrier does not wait for them, and thread 0's release
    // below writes back the L2 but waits only for its own wave's stores.  A
    // full agent-scope fence in every wave would write back the L2 once per
    // wave (measured: 37 us per barrier instead of 6).
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    uint64_t* const pub = reinterpret_cast<uint64_t*>(b.sync + kSyncPub);
    uint64_t* const slot = reinterpret_cast<uint64_t*>(b.sync + kSyncSlots);
    const uint32_t target = phase + 1u;
    if (blockIdx.x == 0) {
        if (threadIdx.x < kWave) {
            // collector: every lane is uniform in its decisions below
            uint32_t mx[KD];
#pragma unroll
            for (int j = 0; j < KD; ++j) mx[j] = threadIdx.x == 0 ? m[j] : 0u;
            int ok = 1;
            uint32_t spins = 0;
            for (;;) {
                bool arrived = true;
                uint32_t lm[KD];
#pragma unroll
                for (int j = 0; j < KD; ++j) lm[j] = mx[j];
                for (uint32_t blk = threadIdx.x; blk < gridDim.x; blk += kWave) {
                    if (blk == 0) continue;
#pragma unroll
                    for (int j = 0; j < KD; ++j) {
                        const uint64_t w = __hip_atomic_load(slot + (size_t)blk * KD + j,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if ((uint32_t)(w >> 32) != target) arrived = false;
                        else lm[j] = max(lm[j], (uint32_t)w);
                    }
                }
                if (__all(arrived)) {
#pragma unroll
                    for (int j = 0; j < KD; ++j) mx[j] = lm[j];
                    break;
                }
                if ((spins & 255u) == 0u && ld_agent(&b.ctrl->error)) {
                    ok = 0;
                    break;
                }
                if (++spins > b.spin_limit) {
                    if (threadIdx.x == 0)
                        __hip_atomic_fetch_or(&b.ctrl->error, kErrBarrierTimeout, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
            for (int j = 0; j < KD; ++j) mx[j] = wave_max_u32(mx[j]);
            if (threadIdx.x == 0) {
                if (ok) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
                    for (int j = 0; j < KD; ++j)
                        __hip_atomic_store(pub + j, barrier_word(target, mx[j]), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
                for (int j = 0; j < KD; ++j) M_sh[j] = mx[j];
                ok_sh = ok;
            }
        }
    } else if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
        for (int j = 0; j < KD; ++j)
            __hip_atomic_store(slot + (size_t)blockIdx.x * KD + j, barrier_word(target, m[j]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        uint32_t spins = 0;
        uint64_t w[KD];
        for (;;) {
            bool arrived = true;
#pragma unroll
            for (int j = 0; j < KD; ++j) {
                w[j] = __hip_atomic_load(pub + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint32_t)(w[j] >> 32) != target) arrived = false;
            }
            if (arrived) break;
            if ((spins & 255u) == 0u && ld_agent(&b.ctrl->error)) {
                ok = 0;
                break;
            }
            if (++spins > b.spin_limit) {
                __hip_atomic_fetch_or(&b.ctrl->error, kErrBarrierTimeout, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
        for (int j = 0; j < KD; ++j) M_sh[j] = (uint32_t)w[j];
        ok_sh = ok;
    }
    phase = target;
    __syncthreads();
    return ok_sh != 0;
}

// The one-value barrier of the kernels that reduce one max per iteration.
__device__ __forceinline__ bool barrier_max(const Barrier& b, uint32_t m, uint32_t& phase,
                                           uint32_t* M_sh) {
    const uint32_t mm[1] = {m};
    return barrier_maxima<1>(b, mm, phase, M_sh);
}

// Clears a barrier's words before a persistent launch.
__global__ void reset_sync_kernel(uint32_t* sync);

// Launch of a persistent kernel.  Cooperative by default (the runtime then
// guarantees the grid is co-resident or refuses the launch).  With the
// environment variable FSB_PERSISTENT_LAUNCH=regular (read once) the same
// grid, never larger than the occupancy maximum, is launched ordinarily --
// for profilers that cannot follow cooperative launches; on an otherwise
// idle GPU every block is then resident, and if one were not, the bounded
// barrier would report FSB_ERR_DEVICE rather than hang.
hipError_t launch_persistent(const void* fn, dim3 grid, dim3 block, void** args,
                             hipStream_t stream);

}  // namespace fsb
