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

// a ^ b ^ k in one VALU instruction: gfx950's three-input v_bitop3_b32 with
// truth table 0x96 (XOR of all three inputs).  k must be uniform across the
// wave (a round key): it is read from a scalar register.  The compiler emits
// two v_xor_b32 for the same expression.
__device__ __forceinline__ uint32_t xor_key(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// One round with round key (rk0, rk1).
__device__ __forceinline__ void philox_round(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                             uint32_t &c3, uint32_t rk0, uint32_t rk1) {
    const uint64_t p0 = (uint64_t)philox_m0() * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)philox_m1() * (uint64_t)c2;
    const uint32_t n0 = xor_key((uint32_t)(p1 >> 32), c1, rk0);
    const uint32_t n2 = xor_key((uint32_t)(p0 >> 32), c3, rk1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

__device__ __forceinline__ uint32_t round_key0(PhiloxKey key, int r) {
    return key.k0 + (uint32_t)r * philox_w0();
}
__device__ __forceinline__ uint32_t round_key1(PhiloxKey key, int r) {
    return key.k1 + (uint32_t)r * philox_w1();
}

// Ten rounds on counter (c0, c1, c2, c3).
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               PhiloxKey key) {
#pragma unroll
    for (int r = 0; r < 10; ++r) philox_round(c0, c1, c2, c3, round_key0(key, r), round_key1(key, r));
    return make_uint4(c0, c1, c2, c3);
}

// The draws of one walk, counters (v, j, t, dom) for t = 1, 2, ...: the same
// values as philox4x32_10(v, j, t, dom, key), with the work that does not depend
// on t done once per walk.  In round 1 only the product with t changes from
// step to step (and it grows by M1 per step); round 2 multiplies one word that
// depends on (v, key) alone.  Only words 0 and 1 of the output are formed.
struct WalkDraws {
    uint32_t j;        // walk index (counter word 1)
    uint32_t a, b, cc; // per-walk constants of round 2
    uint64_t mt;       // M1 * t of the last draw
};

__device__ __forceinline__ WalkDraws walk_draws_begin(uint32_t v, uint32_t j, PhiloxKey key,
                                                      uint32_t dom = 0u) {
    WalkDraws w;
    const uint64_t p0 = (uint64_t)philox_m0() * (uint64_t)v;          // round 1, word 0 (fixed)
    const uint32_t c2 = (uint32_t)(p0 >> 32) ^ dom ^ round_key1(key, 0); // round-1 word 2
    const uint64_t q1 = (uint64_t)philox_m1() * (uint64_t)c2;         // round 2's product of word 2
    w.j = j;
    w.a = (uint32_t)(q1 >> 32) ^ round_key0(key, 1);   // round-2 word 0 = a ^ (round-1 word 1)
    w.b = (uint32_t)q1;                                // round-2 word 1
    w.cc = (uint32_t)p0 ^ round_key1(key, 1);          // round-2 word 2 = hi(M0 * w0') ^ cc
    w.mt = 0;
    return w;
}

// Draw for the next step t (the first call gives t = 1): returns (x0, x1).
__device__ __forceinline__ uint2 walk_draw_next(WalkDraws &w, PhiloxKey key) {
    w.mt += (uint64_t)philox_m1();
    // round 1: word 0 = hi(M1 t) ^ j ^ k0, word 1 = lo(M1 t); words 2, 3 fixed
    const uint32_t r1w0 = xor_key((uint32_t)(w.mt >> 32), w.j, round_key0(key, 0));
    const uint32_t r1w1 = (uint32_t)w.mt;
    // round 2
    const uint64_t p0 = (uint64_t)philox_m0() * (uint64_t)r1w0;
    uint32_t c0 = w.a ^ r1w1;
    uint32_t c1 = w.b;
    uint32_t c2 = (uint32_t)(p0 >> 32) ^ w.cc;
    uint32_t c3 = (uint32_t)p0;
#pragma unroll
    for (int r = 2; r < 9; ++r) philox_round(c0, c1, c2, c3, round_key0(key, r), round_key1(key, r));
    // round 10: words 0 and 1 only
    const uint64_t p1 = (uint64_t)philox_m1() * (uint64_t)c2;
    return make_uint2(xor_key((uint32_t)(p1 >> 32), c1, round_key0(key, 9)), (uint32_t)p1);
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

// Counter domains: plain walk steps, pool segment steps, entry-slot picks,
// successor picks, steps of the fixed-length walks of the length-stratified
// estimator, round keys of a node's walk shuffle.
enum : uint32_t {
    DOM_WALK = 0u, DOM_SEGMENT = 1u, DOM_ENTRY = 2u, DOM_SUCC = 3u, DOM_STRAT = 4u, DOM_SHUFFLE = 5u
};

}  // namespace srk
