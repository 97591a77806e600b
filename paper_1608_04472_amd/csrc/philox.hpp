// Counter-based sample stream for the samplers: Philox4x64 with 10 rounds,
// from its published description (Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11). Each round multiplies words 0
// and 2 by the two Philox multipliers, swaps and xors the halves with the
// round key, and the key advances by the two Weyl increments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcmi {

struct Block4 {
    uint64_t w[4];
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t key0, uint64_t key1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;  // golden ratio
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;  // sqrt(3) - 1
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t hiA = __umul64hi(kMulA, c0), loA = kMulA * c0;
        const uint64_t hiB = __umul64hi(kMulB, c2), loB = kMulB * c2;
        const uint64_t n0 = hiB ^ c1 ^ key0;
        const uint64_t n2 = hiA ^ c3 ^ key1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        key0 += kWeylA;
        key1 += kWeylB;
    }
    Block4 r;
    r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
    return r;
}

// floor(w * range / 2^64): an unbiased-to-2^-64 map of a 64-bit word onto [0, range).
__device__ __forceinline__ int64_t scale_to_range(uint64_t w, uint64_t range)
{
    return (int64_t)__umul64hi(w, range);
}

}  // namespace bcmi
