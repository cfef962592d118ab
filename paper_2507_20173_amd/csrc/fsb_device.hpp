// fsb_device.hpp -- device building blocks of the FSB kernels (gfx950, wave64).
//
// The per-fish arithmetic must be bit-exact and reproducible: every float op
// is binary32 round-to-nearest-even, rounded on its own.  The library is
// compiled with -ffp-contract=off (no a*b+c fusion),
// -fhip-fp32-correctly-rounded-divide-sqrt and without denormal flushing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsb {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Counter (c0..c3), key
// (k0, k1).  A round forms the two 64-bit products A*c0 and B*c2 and
// rebuilds the counter as (hi(B*c2)^c1^k0, lo(B*c2), hi(A*c0)^c3^k1,
// lo(A*c0)); the key moves on by the two Weyl constants after each round.
// Each product is written as one 32x32->64 multiply, which gfx950 does in a
// single v_mad_u64_u32 (measured 1.44x the throughput of separate mul_lo /
// mul_hi), and each three-way XOR is one v_bitop3_b32 (truth table 0x96:
// set for an odd number of set inputs), where the compiler would emit two
// v_xor_b32.  The key is uniform across a launch, so its schedule lives in
// SGPRs.
// ---------------------------------------------------------------------------
struct Words {
    uint32_t r0, r1, r2, r3;
};

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t A = 0xD2511F53u, B = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pA = (uint64_t)A * c0;
        const uint64_t pB = (uint64_t)B * c2;
        c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pB >> 32), c1, k0, 0x96);
        c1 = (uint32_t)pB;
        c2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pA >> 32), c3, k1, 0x96);
        c3 = (uint32_t)pA;
        k0 += WA;
        k1 += WB;
    }
    return {c0, c1, c2, c3};
}

// Counter word 3: the random stream's domain.
constexpr uint32_t kDomainSwim = 0u;
constexpr uint32_t kDomainInit = 1u;

// Both words of one pair-call, for pair index p, sub-stream s, domain d.
__device__ __forceinline__ Words pair_words(uint64_t p, uint32_t s, uint32_t d,
                                            uint32_t k0, uint32_t k1) {
    return philox4x32_10((uint32_t)p, (uint32_t)(p >> 32), s, d, k0, k1);
}

// v(r) = (r >> 8) * 2^-23 - 1, formed as the signed integer
// (r >> 8) - 2^23 scaled by 2^-23: both steps are exact in binary32.
__device__ __forceinline__ float signed_unit(uint32_t r) {
    return (float)((int32_t)(r >> 8) - (1 << 23)) * 0x1p-23f;
}

// u(r) = (r >> 8) * 2^-24, exact.
__device__ __forceinline__ float unit(uint32_t r) {
    return (float)(r >> 8) * 0x1p-24f;
}

// A swim displacement S (x) v(r) in one fused multiply-add.  With
// S23 = S * 2^-23 (exact: the host requires S = 0 or S >= 2^-103) and
// k = r >> 8 (exact in binary32), S23 * k - S equals S * v(r) as a real
// number, and the fma rounds it once, as the product S (x) v(r) does: the
// same binary32 value in three instructions instead of five.
__device__ __forceinline__ float swim_delta(float S23, float negS, uint32_t r) {
    return __builtin_fmaf(S23, (float)(r >> 8), negS);
}

// min(max(v, lo), hi) as one v_med3_f32: the median of (v, lo, hi) is that
// clamp whenever lo <= hi (the host checks every pair of limits) and v is not
// a NaN (positions and weights are finite).
__device__ __forceinline__ float clamp_to(float v, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(v, lo, hi);
}

// Correctly rounded binary32 square root.  For s >= 2^-96 the hardware
// estimate v_sqrt_f32 is within one unit in the last place, and one residual
// test on each neighbour (s - r'*r by fma, whose sign says on which side of
// r' the exact root lies) picks the correctly rounded value: 10 instructions
// against the 16 of the general expansion, which also rescales tiny inputs
// and sorts out zeros and infinities.  Below 2^-96 (and for 0) the general
// sqrtf is taken.  Checked against IEEE sqrt on every non-negative binary32
// value (fsb_eval_sqrt and its test).
__device__ __forceinline__ float sqrt_rn(float s) {
    if (__builtin_expect(s < 0x1p-96f, 0)) return sqrtf(s);
    const float r = __builtin_amdgcn_sqrtf(s);
    const float rm = __uint_as_float(__float_as_uint(r) - 1u);
    const float rp = __uint_as_float(__float_as_uint(r) + 1u);
    const float em = __builtin_fmaf(-rm, r, s);
    const float ep = __builtin_fmaf(-rp, r, s);
    const float t = em <= 0.0f ? rm : r;
    return ep > 0.0f ? rp : t;
}

// Euclidean distance from the pond centre; each op rounded on its own.
__device__ __forceinline__ float distance(float x, float y) {
    const float xx = x * x;
    const float yy = y * y;
    return sqrt_rn(xx + yy);
}

// Swim rules (flags; 0 = the plain random swim).  Weighted: the
// displacement is scaled by wmin / w, w being the weight the fish has when it
// swims (weight affects mobility).  Greedy: a move is kept only if the
// objective strictly decreases; otherwise the fish stays where it was.
constexpr uint32_t kSwimGreedy = 1u, kSwimWeighted = 2u;

struct SwimRule {
    uint32_t flags;  // uniform across a launch
    float wmin;
};

// One fish's swim from objective c: move by (dx, dy) under the rule, inside
// [-H, H]^2, and re-evaluate.  Returns the new objective; x, y are updated in
// place.  w is read only under the weighted rule.
__device__ __forceinline__ float swim(const SwimRule& r, float& x, float& y, float dx, float dy,
                                      float H, float c, float w) {
    if (r.flags & kSwimWeighted) {
        const float m = r.wmin / w;
        dx = dx * m;
        dy = dy * m;
    }
    const float nx = clamp_to(x + dx, -H, H);
    const float ny = clamp_to(y + dy, -H, H);
    const float nc = distance(nx, ny);
    if ((r.flags & kSwimGreedy) && !(nc < c)) return c;
    x = nx;
    y = ny;
    return nc;
}

// Feeding: w + diff / M, kept inside [wmin, wmax]; M == 0 leaves w alone.
__device__ __forceinline__ float feed(float w, float diff, float M, float wmin, float wmax) {
    return M > 0.0f ? clamp_to(w + diff / M, wmin, wmax) : w;
}

// Non-negative floats order like their bit patterns.
__device__ __forceinline__ uint32_t mag_bits(float d) {
    return __float_as_uint(fabsf(d));
}

// ---------------------------------------------------------------------------
// Compensated float32 accumulation: (s, e) with the true sum ~ s + e.  Each
// term goes through Knuth's TwoSum, which is exact whatever the relative
// magnitudes (plain Kahan is not when a term exceeds the running sum, as in
// the signed sums of w*x over a school centred at the origin).
// ---------------------------------------------------------------------------
struct CSum {
    float s, e;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& err) {
    s = a + b;
    const float bv = s - a;
    const float av = s - bv;
    err = (a - av) + (b - bv);
}

__device__ __forceinline__ void csum_add(CSum& c, float v) {
    float s, err;
    two_sum(c.s, v, s, err);
    c.s = s;
    c.e += err;
}

__device__ __forceinline__ CSum csum_merge(CSum a, CSum b) {
    float s, err;
    two_sum(a.s, b.s, s, err);
    return {s, (a.e + b.e) + err};
}

__device__ __forceinline__ double csum_value(CSum c) {
    return (double)c.s + (double)c.e;
}

// ---------------------------------------------------------------------------
// Wave64 reductions (butterfly over lanes; every lane ends with the result).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = max(v, (uint32_t)__shfl_xor((int)v, off, kWave));
    return v;
}

__device__ __forceinline__ CSum wave_csum(CSum c) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        CSum o{__shfl_xor(c.s, off, kWave), __shfl_xor(c.e, off, kWave)};
        c = csum_merge(c, o);
    }
    return c;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace fsb
