// fsb_probe.hpp -- launcher of the instrumentation kernels in fsb_probe.hip.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace fsb {

// VALU ceiling probe (instrumentation): `blocks` blocks of 256 threads, each
// lane running `iters` rounds of the kind's instruction chains; out holds
// blocks x 256 words.
constexpr uint32_t kProbeThreads = 256;
hipError_t launch_valu_probe(uint32_t kind, uint32_t blocks, uint32_t iters, void* out,
                             hipStream_t stream);
// Streaming probe (instrumentation): four columns of n floats (n a multiple
// of 4, 16-byte aligned) read and written in place once, on `grid` blocks of
// 256 threads; streamed: non-temporal accesses.
hipError_t launch_sweep_probe(float* const cols[4], uint64_t n, uint32_t grid, bool streamed,
                              hipStream_t stream);

}  // namespace fsb
