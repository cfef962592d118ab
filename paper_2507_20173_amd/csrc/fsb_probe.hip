// fsb_probe.hip -- instrumentation kernels that measure the chip rather than
// the method: the plain-VALU ceiling the VALU-bound persistent kernels are
// compared with.  Kept out of the kernels' own translation unit, so that the
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
// ---------------------------------------------------------------------------
constexpr uint32_t kProbeFma = 0, kProbePhilox = 1;
constexpr int kProbeCounters = 2;
constexpr int kBlock = kProbeThreads;

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

hipError_t launch_valu_probe(uint32_t kind, uint32_t blocks, uint32_t iters, void* out,
                             hipStream_t stream) {
    if (kind == kProbeFma)
        hipLaunchKernelGGL(valu_probe_fma_kernel, dim3(blocks), dim3(kBlock), 0, stream,
                           static_cast<float*>(out), iters, 1.0f, 0.0f);
    else if (kind == kProbePhilox)
        hipLaunchKernelGGL(valu_probe_philox_kernel, dim3(blocks), dim3(kBlock), 0, stream,
                           static_cast<uint32_t*>(out), iters, 0x12345678u, 0x9ABCDEF0u);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fsb
