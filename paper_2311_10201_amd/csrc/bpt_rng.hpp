// Keyed counter-based coins for the fused BPT kernels.
//
// The paper's traversal flips an independent coin per (traversal, edge)
// (Listing 1's random(0,1) test against e.prob, under the IC model of
// Section 2).  To make every execution order produce identical sets, the
// coin is a pure function of (seed, sample id s, canonical edge id e):
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) with
//   key     = (seed mod 2^32, seed >> 32)
//   counter = (e >> 2, s mod 2^32, s >> 32, 0)
// and the coin word is output word (e & 3).  One Philox block therefore
// serves four consecutive in-edges of a row for one sample, which is how the
// kernels consume it.  Start vertices use the disjoint counter family
// ((s >> 2) mod 2^32, s >> 34, 0, 1), output word (s & 3), scaled to [0, n)
// with a 32x32 -> 64 multiply-shift.
//
// Compiled for both host (C-ABI check helpers) and device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpt {

constexpr uint32_t kPhiloxMulA = 0xD2511F53u;   // multiplier applied to word 0
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;   // multiplier applied to word 2
constexpr uint32_t kPhiloxBumpA = 0x9E3779B9u;  // key schedule increments
constexpr uint32_t kPhiloxBumpB = 0xBB67AE85u;
constexpr uint32_t kAlwaysLive = 0xFFFFFFFFu;   // threshold of p = 1

struct Block4 {
    uint32_t w0, w1, w2, w3;
};

__host__ __device__ __forceinline__ uint32_t mul_hi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
#endif
}

// a ^ b ^ c.  On gfx950 one three-input logic instruction (v_bitop3_b32 with
// the truth table of a three-way xor, 0x96) instead of two xors: a round then
// costs four multiplies and two logic operations.
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

// Ten Philox rounds on counter (c0..c3) with key (k0, k1).  Each round's two
// 32x32 products are taken whole, as 64-bit values: on gfx950 that is one
// v_mad_u64_u32 per product (both halves) instead of a v_mul_hi_u32 and a
// v_mul_lo_u32, and it issues at the full vector rate.
__host__ __device__ __forceinline__ Block4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                    uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pA = (uint64_t)kPhiloxMulA * c0;
        const uint64_t pB = (uint64_t)kPhiloxMulB * c2;
        const uint32_t hiA = (uint32_t)(pA >> 32), loA = (uint32_t)pA;
        const uint32_t hiB = (uint32_t)(pB >> 32), loB = (uint32_t)pB;
        c0 = xor3(hiB, c1, k0);
        c1 = loB;
        c2 = xor3(hiA, c3, k1);
        c3 = loA;
        k0 += kPhiloxBumpA;
        k1 += kPhiloxBumpB;
    }
    return Block4{c0, c1, c2, c3};
}

// The four coin words of edges 4q .. 4q+3 for sample s.
__host__ __device__ __forceinline__ Block4 coin_block(uint32_t quad, uint64_t s, uint32_t k0, uint32_t k1) {
    return philox10(quad, (uint32_t)s, (uint32_t)(s >> 32), 0u, k0, k1);
}

__host__ __device__ __forceinline__ uint32_t pick_word(const Block4& b, uint32_t i) {
    return i == 0 ? b.w0 : (i == 1 ? b.w1 : (i == 2 ? b.w2 : b.w3));
}

__host__ __device__ __forceinline__ uint32_t start_of(uint64_t s, uint32_t n, uint32_t k0, uint32_t k1) {
    const Block4 b = philox10((uint32_t)(s >> 2), (uint32_t)(s >> 34), 0u, 1u, k0, k1);
    return mul_hi32(pick_word(b, (uint32_t)(s & 3)), n);
}

__host__ __device__ __forceinline__ bool coin_live(uint32_t word, uint32_t thr) {
    return word < thr || thr == kAlwaysLive;
}

}  // namespace bpt
