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

// One pair in flight on a lane.
struct Slot {
    uint32_t pos;    // packed: LDS offset of walk (s, j) (16 bits) | its length << 16 | node index << 24
    uint32_t t;      // steps taken
    uint32_t o, d;   // current node: slot offset in E and in-degree
    WalkDraws rng;
    bool busy;
    bool in_tail;    // stitched: the private head is complete
    uint32_t tsig, tm, tu, tseg, tsl;   // stitched tail: entry slot, chain index, position, segment, its length
};

constexpr uint32_t ITEM_CHUNK = 64;


}  // namespace srk
