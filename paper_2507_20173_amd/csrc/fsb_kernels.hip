// fsb_kernels.hip -- HIP kernels of the FSB iteration for gfx950 (MI355X).
//
// Plain iteration t = two streaming passes over the SoA columns:
//   swim pass  (reads x, y, cur; writes x, y, prev, cur; 28 B/fish)
//     draws, swim + pond clamp, objective, |diff|; each block stores its max
//     |diff| bit pattern (non-negative floats order like their bits, so the
//     max is exact and independent of order).  Block 0 first finishes the
//     previous iteration's record from the feed pass's block partials.
//   feed pass  (reads prev, cur, w, x, y; writes w; 24 B/fish)
//     every block reduces the swim pass's block maxima to M, feeds, and
//     accumulates sum w, sum w*x, sum w*y per lane in compensated float32,
//     merges lanes with TwoSum and waves in binary64; one binary64 partial
//     per block.
// The record of iteration t is written by the next swim pass's block 0 (or by
// a one-block combine launch when the host asks for it), in a fixed order, so
// every sum is deterministic.  No atomics and no fences are needed: the
// stream orders the passes.
// Each thread handles groups of four consecutive fish (one float4 per
// column), i.e. two Philox calls (fish pairs 2g and 2g+1).  Fish beyond the
// last full group (n % 4 of them) are handled one by one by the last block.
#include "fsb_device.hpp"
#include "fsb_internal.hpp"

namespace fsb {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr uint32_t kPlainGridCap = 2048;  // 8 blocks of 4 waves per CU x 256 CUs
constexpr int kUnroll = 2;                // groups in flight per thread

__device__ __forceinline__ float4 ld4(const float* p, uint64_t g) {
    return reinterpret_cast<const float4*>(p)[g];
}
__device__ __forceinline__ void st4(float* p, uint64_t g, float4 v) {
    reinterpret_cast<float4*>(p)[g] = v;
}
__device__ __forceinline__ float& lane_of(float4& v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

// ---------------------------------------------------------------------------
// Control-word reset (a kernel rather than a memset, so it is graph-safe).
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
// Record of iteration t from the feed pass's block partials (one block).
// ---------------------------------------------------------------------------
__device__ void combine_block(const SchoolArgs& a, uint32_t t, uint32_t grid, uint32_t naive) {
    __shared__ double part[3][kWaves];
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (!naive) {
        const double* p = a.partials;  // phase 0
        for (uint32_t b = threadIdx.x; b < grid; b += kBlock) {
            acc0 += p[b];
            acc1 += p[kMaxGrid + b];
            acc2 += p[2 * kMaxGrid + b];
        }
        acc0 = wave_sum_f64(acc0);
        acc1 = wave_sum_f64(acc1);
        acc2 = wave_sum_f64(acc2);
        const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
        if (lane == 0) {
            part[0][wid] = acc0;
            part[1][wid] = acc1;
            part[2][wid] = acc2;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        fsb_record r;
        if (!naive) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int w = 0; w < kWaves; ++w) {
                s0 += part[0][w];
                s1 += part[1][w];
                s2 += part[2][w];
            }
            r.sum_w = s0;
            r.sum_wx = s1;
            r.sum_wy = s2;
        } else {
            r.sum_w = (double)a.ctrl->naive_acc[0];
            r.sum_wx = (double)a.ctrl->naive_acc[1];
            r.sum_wy = (double)a.ctrl->naive_acc[2];
            a.ctrl->naive_acc[0] = 0.0f;
            a.ctrl->naive_acc[1] = 0.0f;
            a.ctrl->naive_acc[2] = 0.0f;
        }
        r.max_delta = __uint_as_float(a.ctrl->last_max);
        r.step_lo = t;
        a.hist[t % a.hist_len] = r;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void combine_kernel(SchoolArgs a, uint32_t t, uint32_t grid,
                                                         uint32_t naive) {
    combine_block(a, t, grid, naive);
}

// ---------------------------------------------------------------------------
// Swim pass.
// ---------------------------------------------------------------------------
template <bool kInject>
__global__ __launch_bounds__(kBlock) void swim_eval_kernel(SchoolArgs a, StepArgs s) {
    __shared__ uint32_t wave_best[kWaves];
    if (s.combine && blockIdx.x == 0) combine_block(a, s.prev_t, s.prev_grid, s.naive);

    const float H = a.H, S = a.S;
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t best = 0u;
    for (uint64_t g0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g0 < n4;
         g0 += kUnroll * stride) {
        float4 X[kUnroll], Y[kUnroll], C[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g < n4) {
                X[u] = ld4(a.x, g);
                Y[u] = ld4(a.y, g);
                C[u] = ld4(a.cur, g);
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g >= n4) break;
            float dx[4], dy[4];
            if constexpr (kInject) {
                const float4 DX = ld4(s.dx, g), DY = ld4(s.dy, g);
                dx[0] = DX.x; dx[1] = DX.y; dx[2] = DX.z; dx[3] = DX.w;
                dy[0] = DY.x; dy[1] = DY.y; dy[2] = DY.z; dy[3] = DY.w;
            } else {
                const Words p0 = pair_words(2 * g, s.t, kDomainSwim, a.k0, a.k1);
                const Words p1 = pair_words(2 * g + 1, s.t, kDomainSwim, a.k0, a.k1);
                dx[0] = S * signed_unit(p0.r0); dy[0] = S * signed_unit(p0.r1);
                dx[1] = S * signed_unit(p0.r2); dy[1] = S * signed_unit(p0.r3);
                dx[2] = S * signed_unit(p1.r0); dy[2] = S * signed_unit(p1.r1);
                dx[3] = S * signed_unit(p1.r2); dy[3] = S * signed_unit(p1.r3);
            }
            float4 nx = X[u], ny = Y[u], nc;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                lane_of(nc, k) = swim(lane_of(nx, k), lane_of(ny, k), dx[k], dy[k], H);
                best = max(best, mag_bits(lane_of(C[u], k) - lane_of(nc, k)));
            }
            st4(a.x, g, nx);
            st4(a.y, g, ny);
            st4(a.prev, g, C[u]);
            st4(a.cur, g, nc);
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
                const Words p = pair_words(i >> 1, s.t, kDomainSwim, a.k0, a.k1);
                const bool odd = i & 1;
                dx = S * signed_unit(odd ? p.r2 : p.r0);
                dy = S * signed_unit(odd ? p.r3 : p.r1);
            }
            float x = a.x[i], y = a.y[i];
            const float c = a.cur[i];
            const float nc = swim(x, y, dx, dy, H);
            best = max(best, mag_bits(c - nc));
            a.x[i] = x;
            a.y[i] = y;
            a.prev[i] = c;
            a.cur[i] = nc;
        }
    }
    best = wave_max_u32(best);
    if (threadIdx.x % kWave == 0) wave_best[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = wave_best[0];
        for (int w = 1; w < kWaves; ++w) m = max(m, wave_best[w]);
        a.blockmax[blockIdx.x] = m;
    }
}

// ---------------------------------------------------------------------------
// Feed pass.
// ---------------------------------------------------------------------------
template <bool kNaive>
__device__ __forceinline__ void accumulate(CSum* cs, float* fs, float w, float x, float y) {
    const float wx = w * x;
    const float wy = w * y;
    if constexpr (kNaive) {
        fs[0] += w;
        fs[1] += wx;
        fs[2] += wy;
    } else {
        csum_add(cs[0], w);
        csum_add(cs[1], wx);
        csum_add(cs[2], wy);
    }
}

template <bool kNaive>
__global__ __launch_bounds__(kBlock) void feed_bary_kernel(SchoolArgs a, StepArgs s) {
    __shared__ uint32_t wave_best[kWaves];
    __shared__ CSum wave_cs[3][kWaves];
    __shared__ float wave_fs[3][kWaves];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;

    // M = max over the swim pass's block maxima.
    uint32_t mb = 0u;
    for (uint32_t b = threadIdx.x; b < s.swim_grid; b += kBlock) mb = max(mb, a.blockmax[b]);
    mb = wave_max_u32(mb);
    if (lane == 0) wave_best[wid] = mb;
    __syncthreads();
    mb = wave_best[0];
    for (int w = 1; w < kWaves; ++w) mb = max(mb, wave_best[w]);
    const float M = __uint_as_float(mb);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->last_max = mb;

    const float wmin = a.wmin, wmax = a.wmax;
    CSum cs[3] = {{0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}};
    float fs[3] = {0.0f, 0.0f, 0.0f};
    const uint64_t n4 = a.n >> 2;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g0 < n4;
         g0 += kUnroll * stride) {
        float4 P[kUnroll], C[kUnroll], W[kUnroll], X[kUnroll], Y[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g < n4) {
                P[u] = ld4(a.prev, g);
                C[u] = ld4(a.cur, g);
                W[u] = ld4(a.w, g);
                X[u] = ld4(a.x, g);
                Y[u] = ld4(a.y, g);
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint64_t g = g0 + u * stride;
            if (g >= n4) break;
            float4 nw;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float diff = lane_of(P[u], k) - lane_of(C[u], k);
                lane_of(nw, k) = feed(lane_of(W[u], k), diff, M, wmin, wmax);
                accumulate<kNaive>(cs, fs, lane_of(nw, k), lane_of(X[u], k), lane_of(Y[u], k));
            }
            st4(a.w, g, nw);
        }
    }
    if (blockIdx.x == gridDim.x - 1) {
        const uint64_t i = 4 * n4 + threadIdx.x;
        if (i < a.n) {
            const float diff = a.prev[i] - a.cur[i];
            const float nw = feed(a.w[i], diff, M, wmin, wmax);
            a.w[i] = nw;
            accumulate<kNaive>(cs, fs, nw, a.x[i], a.y[i]);
        }
    }

    if constexpr (kNaive) {
        // Plain float32 trees, then float32 atomics across blocks.
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            fs[k] = wave_sum_f32(fs[k]);
            if (lane == 0) wave_fs[k][wid] = fs[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 0; k < 3; ++k) {
                float v = wave_fs[k][0];
                for (int w = 1; w < kWaves; ++w) v += wave_fs[k][w];
                atomicAdd(&a.ctrl->naive_acc[k], v);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cs[k] = wave_csum(cs[k]);
            if (lane == 0) wave_cs[k][wid] = cs[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 0; k < 3; ++k) {
                double v = 0.0;
                for (int w = 0; w < kWaves; ++w) v += csum_value(wave_cs[k][w]);
                a.partials[k * kMaxGrid + blockIdx.x] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
uint32_t plain_grid(uint64_t n) {
    const uint64_t groups = n >> 2;
    uint64_t g = (groups + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > kPlainGridCap) g = kPlainGridCap;
    return (uint32_t)g;
}

hipError_t launch_reset(const SchoolArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, stream, a.ctrl);
    return hipGetLastError();
}

hipError_t launch_init(const SchoolArgs& a, float wlo, float whi, hipStream_t stream) {
    InitArgs ia{a, wlo, whi};
    hipLaunchKernelGGL(init_kernel, dim3(plain_grid(a.n)), dim3(kBlock), 0, stream, ia);
    return hipGetLastError();
}

hipError_t launch_swim_eval(const SchoolArgs& a, const StepArgs& s, hipStream_t stream) {
    if (s.dx)
        hipLaunchKernelGGL(swim_eval_kernel<true>, dim3(s.swim_grid), dim3(kBlock), 0, stream, a, s);
    else
        hipLaunchKernelGGL(swim_eval_kernel<false>, dim3(s.swim_grid), dim3(kBlock), 0, stream, a, s);
    return hipGetLastError();
}

hipError_t launch_feed_bary(const SchoolArgs& a, const StepArgs& s, uint32_t grid,
                            hipStream_t stream) {
    if (s.naive)
        hipLaunchKernelGGL(feed_bary_kernel<true>, dim3(grid), dim3(kBlock), 0, stream, a, s);
    else
        hipLaunchKernelGGL(feed_bary_kernel<false>, dim3(grid), dim3(kBlock), 0, stream, a, s);
    return hipGetLastError();
}

hipError_t launch_combine(const SchoolArgs& a, uint32_t t, uint32_t grid, uint32_t naive,
                          hipStream_t stream) {
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(kBlock), 0, stream, a, t, grid, naive);
    return hipGetLastError();
}

}  // namespace fsb
