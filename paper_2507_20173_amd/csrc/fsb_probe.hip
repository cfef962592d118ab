// fsb_probe.hip -- instrumentation kernels that measure the chip rather than
// the method: the plain-VALU ceiling the VALU-bound persistent kernels are
// compared with, and the streaming rate of the plain kernels' access pattern.  Kept out of the kernels' own translation unit, so that the
// measured kernels' code (and the digests that key their counter summaries)
// does not change with it.
#include "fsb_device.hpp"
#include "fsb_probe.hpp"

namespace fsb {

// ---------------------------------------------------------------------------
// VALU ceiling probes (instrumentation).  Every lane runs `iters` rounds of
// independent dependency chains of one kind of vector instruction, enough of
// them that a SIMD's waves issue back to back, and stores one word so that
// nothing is dead.  Instructions per lane and round (checked on the assembly):
//   kProbeFma     8 v_fma_f32 (8 chains)
//   kProbePhilox  80: one Philox4x32-10 call, the kernels' own, on each of 2
//                 counters fed back as the next counter: per call and round
//                 2 v_mad_u64_u32 and 2 v_bitop3_b32 (the key schedule is
//                 uniform and stays on the scalar unit)
//   kProbeMixed   80: one Philox4x32-10 call (40) and 40 v_fma_f32 (8 chains,
//                 5 each), the integer and float mix of the kernels' swims
// ---------------------------------------------------------------------------
constexpr uint32_t kProbeFma = 0, kProbePhilox = 1, kProbeMixed = 2;
constexpr int kProbeCounters = 2;
constexpr int kBlock = kProbeThreads;

typedef float v4f __attribute__((ext_vector_type(4)));
template <bool kNT>
__device__ __forceinline__ float4 ldv4(const float* p, uint64_t g) {
    const v4f* q = reinterpret_cast<const v4f*>(p) + g;
    v4f v;
    if constexpr (kNT) v = __builtin_nontemporal_load(q); else v = *q;
    return make_float4(v.x, v.y, v.z, v.w);
}
template <bool kNT>
__device__ __forceinline__ void stv4(float* p, uint64_t g, float4 v) {
    v4f* q = reinterpret_cast<v4f*>(p) + g;
    const v4f w = {v.x, v.y, v.z, v.w};
    if constexpr (kNT) __builtin_nontemporal_store(w, q); else *q = w;
}
__device__ __forceinline__ float4 plus1(float4 v) {
    return make_float4(v.x + 1.0f, v.y + 1.0f, v.z + 1.0f, v.w + 1.0f);
}

__global__ __launch_bounds__(kBlock) void valu_probe_fma_kernel(float* out, uint32_t iters,
                                                                 float b, float c) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (float)(threadIdx.x + j);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = __builtin_fmaf(v[j], b, c);
    }
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void valu_probe_philox_kernel(uint32_t* out, uint32_t iters,
                                                                    uint32_t k0, uint32_t k1) {
    Words w[kProbeCounters];
#pragma unroll
    for (int j = 0; j < kProbeCounters; ++j)
        w[j] = {blockIdx.x * kBlock + threadIdx.x, (uint32_t)j, iters, 0u};
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kProbeCounters; ++j)
            w[j] = philox4x32_10(w[j].r0, w[j].r1, w[j].r2, w[j].r3, k0, k1);
    }
    uint32_t acc = 0u;
#pragma unroll
    for (int j = 0; j < kProbeCounters; ++j) acc ^= w[j].r0 ^ w[j].r1 ^ w[j].r2 ^ w[j].r3;
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void valu_probe_mixed_kernel(uint32_t* out, uint32_t iters,
                                                                   uint32_t k0, uint32_t k1,
                                                                   float b, float c) {
    Words w = {blockIdx.x * kBlock + threadIdx.x, 7u, iters, 0u};
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (float)(threadIdx.x + j);
    for (uint32_t i = 0; i < iters; ++i) {
        w = philox4x32_10(w.r0, w.r1, w.r2, w.r3, k0, k1);
#pragma unroll
        for (int r = 0; r < 5; ++r)
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = __builtin_fmaf(v[j], b, c);
    }
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = w.r0 ^ w.r1 ^ w.r2 ^ w.r3 ^ __float_as_uint(acc);
}

// ---------------------------------------------------------------------------
// Streaming probe (instrumentation): the plain kernels' access pattern without
// their arithmetic.  Four float32 columns of n floats are read and written in
// place as float4 groups, one group per thread per round, grid-stride (each
// float gains 1.0f, so nothing is dead): 32 B per group of four fish, as the
// pipelined pass moves.  kNT streams every access past the caches.
// ---------------------------------------------------------------------------
template <bool kNT>
__global__ __launch_bounds__(kBlock) void sweep_probe_kernel(float* c0, float* c1, float* c2,
                                                              float* c3, uint64_t n4) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x; g < n4; g += stride) {
        float4 a = ldv4<kNT>(c0, g), b = ldv4<kNT>(c1, g), c = ldv4<kNT>(c2, g), d = ldv4<kNT>(c3, g);
        stv4<kNT>(c0, g, plus1(a));
        stv4<kNT>(c1, g, plus1(b));
        stv4<kNT>(c2, g, plus1(c));
        stv4<kNT>(c3, g, plus1(d));
    }
}

hipError_t launch_sweep_probe(float* const cols[4], uint64_t n, uint32_t grid, bool streamed,
                              hipStream_t stream) {
    const uint64_t n4 = n / 4;
    if (streamed)
        hipLaunchKernelGGL(sweep_probe_kernel<true>, dim3(grid), dim3(kBlock), 0, stream, cols[0],
                           cols[1], cols[2], cols[3], n4);
    else
        hipLaunchKernelGGL(sweep_probe_kernel<false>, dim3(grid), dim3(kBlock), 0, stream, cols[0],
                           cols[1], cols[2], cols[3], n4);
    return hipGetLastError();
}

hipError_t launch_valu_probe(uint32_t kind, uint32_t blocks, uint32_t iters, void* out,
                             hipStream_t stream) {
    if (kind == kProbeFma)
        hipLaunchKernelGGL(valu_probe_fma_kernel, dim3(blocks), dim3(kBlock), 0, stream,
                           static_cast<float*>(out), iters, 1.0f, 0.0f);
    else if (kind == kProbePhilox)
        hipLaunchKernelGGL(valu_probe_philox_kernel, dim3(blocks), dim3(kBlock), 0, stream,
                           static_cast<uint32_t*>(out), iters, 0x12345678u, 0x9ABCDEF0u);
    else if (kind == kProbeMixed)
        hipLaunchKernelGGL(valu_probe_mixed_kernel, dim3(blocks), dim3(kBlock), 0, stream,
                           static_cast<uint32_t*>(out), iters, 0x12345678u, 0x9ABCDEF0u, 1.0f, 0.0f);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fsb
