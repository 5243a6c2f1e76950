// Device helpers shared by the query kernels (single queries and groups).
#pragma once

#include "common.hpp"
#include "philox.hpp"

namespace srk {

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Slot entered by walk (v, j) whose private head ended at node y
// (counter (v, j, 0, 2)).
__device__ __forceinline__ uint32_t entry_slot(const IndexView &ix, PhiloxKey key, uint32_t v,
                                               uint32_t j, uint32_t y) {
    const int64_t b = ix.pool_off[y];
    const int64_t P = ix.pool_off[y + 1] - b;
    const uint4 x = philox4x32_10(v, j, 0u, DOM_ENTRY, key);
    return (uint32_t)(b + (int64_t)pick64(x.x, (uint64_t)P));
}

template <typename T>
__device__ __forceinline__ T block_excl_sum(T x, T *total) {
    __shared__ T part[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T inc = x;
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) part[wave] = inc;
    __syncthreads();
    T before = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) before += part[w];
        tot += part[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

// Cuts entries [0, E1), entry e holding words [joff[e], joff[e + 1]), into
// tiles from the front, each the longest run [a, b) with b - a <= TJ and
// joff[b] - joff[a] <= TN; writes the starts to tiles[0 .. count) and returns
// the count.  Every tile but the last is full in walks (TJ) or holds more than
// TN - w words, w the largest entry, so the count stays within 1 + E1 / TJ +
// joff[E1] / (TN - w).  Called by all 64 lanes of one wave (results uniform);
// needs w <= TN.  Each run's end is found by a 64-way search: the lanes probe
// 64 points of the open range at once, so a range of up to 64^2 entries takes
// two rounds of loads.
__device__ inline uint32_t cut_tiles(const uint32_t *joff, uint32_t E1, uint32_t TJ, uint32_t TN,
                                     uint32_t *tiles, int lane) {
    uint32_t a = 0, nt = 0;
    while (a < E1) {
        if (lane == 0) tiles[nt] = a;
        ++nt;
        const uint32_t base = joff[a];
        // the run ends at the largest b in [lo, hi] with joff[b] - base <= TN;
        // lo = a + 1 always qualifies (one entry fits)
        uint32_t lo = a + 1, hi = min(a + TJ, E1);
        while (lo < hi) {
            const uint32_t span = hi - lo;
            const uint32_t p = lo + (uint32_t)(((uint64_t)span * (uint32_t)(lane + 1)) >> 6);
            const bool fits = joff[p] - base <= TN;
            const uint64_t m = __ballot(fits);   // fits holds for a prefix of the lanes
            const uint32_t k = (uint32_t)__popcll(m);
            const uint32_t p_last = uni(__shfl(p, (int)(k ? k - 1 : 0), 64));
            const uint32_t p_next = uni(__shfl(p, (int)(k < 64 ? k : 63), 64));
            if (k == 64) lo = hi;
            else {
                if (k) lo = p_last;
                hi = p_next - 1;
            }
        }
        a = lo;
    }
    return nt;
}

// The walk's gather of an edge slot.  SRK_EDGE_LOAD selects the cache policy
// (0: default, 1: non-temporal).
#ifndef SRK_EDGE_LOAD
#define SRK_EDGE_LOAD 0
#endif
__device__ __forceinline__ uint2 load_edge(const uint2 *p) {
#if SRK_EDGE_LOAD == 1
    const uint64_t v = __builtin_nontemporal_load((const uint64_t *)p);
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
#else
    return *p;
#endif
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// One pair in flight on a lane.  The six unused words keep the layout the
// plain kind's hot loop was measured with: the compiler's register assignment
// follows the struct, and without them the plain kernel takes 3% longer at
// n = 2^24 (74 instead of 68 VGPRs, extra register moves).
struct Slot {
    uint32_t pos;    // packed: LDS offset of walk (s, j) (16 bits) | its length << 16 | node index << 24
    uint32_t t;      // steps taken
    uint32_t o, d;   // current node: slot offset in E and in-degree
    WalkDraws rng;
    bool busy;
    uint32_t unused[6];
    uint32_t aux;    // stratified: class of walk (s, j) << 8 | class of walk (v, j);
                     // stitched: the tile entry of walk (s, j)
};

constexpr uint32_t ITEM_CHUNK = 64;
// Pairs waiting for their stitched tails, per wave: a ring, a power of two
// above 63 + 64 (a wave drains 64 as soon as 64 wait, after each slot's push).
constexpr uint32_t TAIL_Q = 128;

// ------------------------------------------------- walk shuffle (stratified)
//
// Node v's N fixed-length walks are generated class by class (slots
// [ccum[l], ccum[l+1]) hold the walks of length l) and then shuffled: walk j
// is the walk generated in slot pi_v(j).  pi_v is a four-round Feistel
// network over the grid [0, A) x [0, 2^b) (A 2^b >= N, 2^b about sqrt(N)),
// restricted to [0, N) by cycle walking (Black and Rogaway, CT-RSA 2002); its
// round keys are the four words of Philox(v, 0, 0, DOM_SHUFFLE).  Fewer than
// 2/sqrt(N) of the grid's points lie beyond N, so a lane almost never walks a
// second time.

// MurmurHash3's 32-bit finalizer (A. Appleby, public domain), the round function.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Bijection of the grid, point (hi, lo) = hi 2^b + lo: rounds alternately add
// a round-function value scaled into [0, A) to hi modulo A, and XOR lo with
// its low b bits (a mixed-radix Feistel network, as in NIST SP 800-38G FF1).
__device__ __forceinline__ uint32_t feistel4(uint32_t x, uint32_t A, uint32_t b, uint4 k) {
    const uint32_t mb = (1u << b) - 1u;
    uint32_t hi = x >> b, lo = x & mb;
    hi += __umulhi(fmix32(lo ^ k.x), A);
    hi = hi >= A ? hi - A : hi;
    lo ^= fmix32(hi ^ k.y) & mb;
    hi += __umulhi(fmix32(lo ^ k.z), A);
    hi = hi >= A ? hi - A : hi;
    lo ^= fmix32(hi ^ k.w) & mb;
    return (hi << b) | lo;
}

// pi_v(j) for j < N.  The orbit of j under the bijection is a cycle through
// j, so a value below N comes back within A 2^b applications; the loop is
// bounded by that.
__device__ __forceinline__ uint32_t shuffle_slot(uint32_t j, uint32_t N, uint32_t A, uint32_t b,
                                                 uint4 k) {
    uint32_t y = feistel4(j, A, b, k);
    const uint32_t cap = A << b;
    for (uint32_t it = 1; y >= N && it < cap; ++it) y = feistel4(y, A, b, k);
    return y;
}

// Length class of slot r: the largest l <= phi with ccum[l] <= r.
__device__ __forceinline__ uint32_t slot_class(uint32_t r, const uint32_t *ccum, int32_t phi) {
    int32_t lo = 0, hi = phi + 1;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (ccum[mid] <= r) lo = mid; else hi = mid;
    }
    return (uint32_t)lo;
}

// Meet weight of classes (l1, l2) in units of 2^-40 (Lemma 5's ratio
// Z_l1 Z_l2 / (Zhat_l1 Zhat_l2), truncated).
__device__ __forceinline__ unsigned long long strat_weight(const double *a, uint32_t l1, uint32_t l2) {
    return (unsigned long long)((a[l1] * a[l2]) * 1099511627776.0);
}


}  // namespace srk
