// Philox4x32-10 counter-based generator for the device (Salmon, Moraes, Dror,
// Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11, Section 4.2).
//
// State: four 32-bit counter words and a two-word key.  One round multiplies
// counter words 0 and 2 by two fixed odd constants, keeps the low halves as
// the new words 1 and 3, and XORs the high halves with the other two counter
// words and the round key to form the new words 0 and 2.  The key advances by
// two Weyl constants between rounds.  Ten rounds.
//
// The key is uniform across a launch, so its ten round values live in scalar
// registers; per lane a round costs two 32x32->64 products and two 3-way XORs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srk {

struct PhiloxKey {
    uint32_t k0, k1;
};

__host__ __device__ constexpr uint32_t philox_m0() { return 0xD2511F53u; }
__host__ __device__ constexpr uint32_t philox_m1() { return 0xCD9E8D57u; }
__host__ __device__ constexpr uint32_t philox_w0() { return 0x9E3779B9u; }
__host__ __device__ constexpr uint32_t philox_w1() { return 0xBB67AE85u; }

__host__ __device__ inline PhiloxKey make_key(uint64_t seed) {
    return PhiloxKey{(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
}

// Ten rounds on counter (c0, c1, c2, c3).
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               PhiloxKey key) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t rk0 = key.k0 + (uint32_t)r * philox_w0();
        const uint32_t rk1 = key.k1 + (uint32_t)r * philox_w1();
        const uint64_t p0 = (uint64_t)philox_m0() * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)philox_m1() * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ rk0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ rk1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

// floor(x * k / 2^32): a uniform index in [0, k) from one 32-bit word.
__device__ __forceinline__ uint32_t pick32(uint32_t x, uint32_t k) {
    return __umulhi(x, k);
}
__device__ __forceinline__ uint64_t pick64(uint32_t x, uint64_t k) {
    // x * k < 2^96; high 64 bits of the 96-bit product
    const uint64_t lo = (uint64_t)x * (uint32_t)k;
    const uint64_t hi = (uint64_t)x * (uint32_t)(k >> 32);
    return hi + (lo >> 32);
}

// Counter domains.
enum : uint32_t { DOM_WALK = 0u, DOM_SEGMENT = 1u, DOM_ENTRY = 2u, DOM_SUCC = 3u };

}  // namespace srk
