// Query groups: queries of one batch (or of the server's waiting requests)
// that share a graph, a kind of walks, a walk key and the walks' parameters.
//
// The estimator of Section 3 pairs walk j of the source s with walk j of every
// node v.  The walk (v, j) draws its steps from counters (v, j, t, 0) under the
// query's key, so queries that share the key, the decay and the cap have the
// same walk (v, j) for every v and differ only in their source walks.  A group
// follows each walk (v, j) once and, at every step, compares its position with
// the same step of walk j of each member's source; a member drops out of the
// pair once it has met (counted once, as for a lone query) or its source walk
// has no further step.  The pair ends when the walk stops, reaches a node
// without in-neighbours, or no member is left.  Each member's counts are
// therefore exactly those of its lone run; the walks from the nodes are paid
// for once per group instead of once per query.  The same holds for stitched
// walks (their tails come from the shared index, entered by a draw keyed
// (v, j)) and for the stratified estimator's walks (walk j of v is the walk in
// slot pi_v(j), a function of v and the key; a meet adds Lemma 5's weight of
// the two walks' classes).
#include <algorithm>

#include "common.hpp"
#include "device_common.hpp"

namespace srk {
namespace {

// Tile shapes of the group meet kernel (walks and member positions per tile)
// for groups of up to 8 members and of up to 32; stratified walks keep 64-bit
// weighted sums in LDS, which take room from the tile (and, beyond 8 members,
// from the nodes per work unit).
#ifndef SRK_GROUP_TILE_J
#define SRK_GROUP_TILE_J 1280
#endif
#ifndef SRK_GROUP_TILE_NODES
#define SRK_GROUP_TILE_NODES 32768
#endif
#ifndef SRK_GROUP32_TILE_J
#define SRK_GROUP32_TILE_J 512
#endif
#ifndef SRK_GROUP32_TILE_NODES
#define SRK_GROUP32_TILE_NODES 28672
#endif
#ifndef SRK_GROUP32_STRAT_TILE_NODES
#define SRK_GROUP32_STRAT_TILE_NODES 20480
#endif
#ifndef SRK_GROUP_STRAT_TILE_J
#define SRK_GROUP_STRAT_TILE_J 1024
#endif
#ifndef SRK_GROUP_STRAT_TILE_NODES
#define SRK_GROUP_STRAT_TILE_NODES 24576
#endif
#ifndef SRK_GROUP_SLOTS
#define SRK_GROUP_SLOTS 2
#endif
constexpr int GROUP_BLOCK = 1024;
// GW: the instance's member capacity in words of four (2: up to 8 members, 8:
// up to 32; it sizes the per-member LDS counters and picks the tile shape);
// WK: walks (0 plain, 1 stitched, 2 stratified).
__host__ __device__ constexpr int group_tile_j(int GW, int WK) {
    return GW > 2 ? SRK_GROUP32_TILE_J : WK == 2 ? SRK_GROUP_STRAT_TILE_J : SRK_GROUP_TILE_J;
}
__host__ __device__ constexpr int group_tile_nodes(int GW, int WK) {   // < 2^16
    return GW > 2 ? (WK == 2 ? SRK_GROUP32_STRAT_TILE_NODES : SRK_GROUP32_TILE_NODES)
                  : WK == 2 ? SRK_GROUP_STRAT_TILE_NODES : SRK_GROUP_TILE_NODES;
}
// Nodes per work unit whose sums a stratified instance keeps in LDS.
__host__ __device__ constexpr int group_strat_vb(int GW) { return GW > 2 ? GROUP_STRAT32_VB : MEET_VB; }
// a tile holds at least one entry of the longest form ((G + 1) L words)
static_assert(group_tile_nodes(2, 0) < 65536 && group_tile_nodes(2, 0) > 9 * MAX_CAP, "tile shape");
static_assert(group_tile_nodes(8, 0) < 65536 && group_tile_nodes(8, 0) > 33 * MAX_CAP, "tile shape");
static_assert(group_tile_nodes(2, 2) < 65536 && group_tile_nodes(2, 2) > 9 * MAX_CAP, "tile shape");
static_assert(group_tile_nodes(8, 2) < 65536 && group_tile_nodes(8, 2) > 33 * MAX_CAP, "tile shape");
static_assert(GROUP_MAX == 32, "length words");

// The kernel instance (its GW) for groups of G members.
__host__ __device__ inline int group_gw(int32_t G) { return G <= 8 ? 2 : 8; }

// Length of member q in an entry's length words (byte q).
__device__ __forceinline__ uint32_t byte_of(uint32_t w, int q) { return (w >> (8 * (q & 3))) & 0xffu; }

// ------------------------------------------------------------ compaction
// One block per group.  Keeps the walk indices j for which at least one
// member's walk j has a step and packs the members' positions of walk j step
// by step: for each step t up to the longest member walk, the word of members
// with a position at t, then their positions at t in member order.  Cuts the
// entries into tiles of at most TJ entries and TN words, each the longest run
// from the previous one's end (cut_tiles; an entry holds at most (G + 1) L
// words).  (TJ, TN) is the shape of the kernel instance that runs the group.
__global__ __launch_bounds__(1024) void k_group_compact(const GroupDesc *__restrict__ gd) {
    const GroupDesc &d = gd[blockIdx.x];
    const int32_t Rmax = d.Rmax, L = d.L, G = d.G, gw = d.gw;
    const uint32_t TJ = (uint32_t)group_tile_j(group_gw(G), d.wk);
    const uint32_t TN = (uint32_t)group_tile_nodes(group_gw(G), d.wk);
    const int32_t per = (Rmax + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x;
    const int32_t j0 = min(Rmax, (int32_t)threadIdx.x * per), j1 = min(Rmax, j0 + per);
    uint32_t cnt = 0, nodes = 0;
    for (int32_t j = j0; j < j1; ++j) {
        uint32_t tot = 0, mx = 0;
        for (int32_t q = 0; q < G; ++q) {
            const uint32_t l = j < d.R[q] ? (uint32_t)d.slen[q][j] : 0u;
            tot += l;
            mx = max(mx, l);
        }
        cnt += tot > 0;
        nodes += tot + mx;
    }
    uint32_t E1, total;
    const uint32_t kb = block_excl_sum(cnt, &E1);
    const uint32_t nb = block_excl_sum(nodes, &total);
    uint32_t k = kb, off = nb;
    for (int32_t j = j0; j < j1; ++j) {
        uint32_t tot = 0, mx = 0;
        for (int32_t q = 0; q < G; ++q) {
            const uint32_t l = j < d.R[q] ? (uint32_t)d.slen[q][j] : 0u;
            tot += l;
            mx = max(mx, l);
        }
        if (!tot) continue;
        d.jj[k] = (uint32_t)j;
        d.joff[k] = off;
        for (int32_t wd = 0; wd < gw; ++wd) {
            uint32_t w = 0;
            for (int32_t b = 0; b < 4; ++b) {
                const int32_t q = 4 * wd + b;
                const uint32_t l = (q < G && j < d.R[q]) ? (uint32_t)d.slen[q][j] : 0u;
                w |= l << (8 * b);
            }
            d.glen[(size_t)k * gw + wd] = w;
        }
        // the lengths again from the words just written (registers), not
        // from the members' length arrays at every step
        uint32_t lw[GROUP_MAX / 4];
#pragma unroll
        for (int wd = 0; wd < GROUP_MAX / 4; ++wd)
            lw[wd] = wd < gw ? d.glen[(size_t)k * gw + wd] : 0u;
        for (uint32_t t = 0; t < mx; ++t) {
            const uint32_t at = off++;
            uint32_t am = 0;
#pragma unroll
            for (int wd = 0; wd < GROUP_MAX / 4; ++wd) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int q = 4 * wd + b;
                    if (t < byte_of(lw[wd], b)) {
                        am |= 1u << q;
                        d.pos[off++] = d.sw[q][(size_t)j * L + t];
                    }
                }
            }
            d.pos[at] = am;
        }
        ++k;
    }
    if (threadIdx.x == 0) d.joff[E1] = total;
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t n_tiles = cut_tiles(d.joff, E1, TJ, TN, d.tiles, (int)threadIdx.x);
        if (threadIdx.x == 0) {
            d.tiles[n_tiles] = E1;
            d.meta[0] = E1;
            d.meta[1] = total;
            d.meta[2] = n_tiles;
        }
    }
}

// Work-unit offsets of the groups (one block), one list per kernel instance
// (group_list: the walks, up to 8 members or more): ng + 1
// offsets each, then one cursor each.
__global__ __launch_bounds__(1024) void k_group_units(const GroupDesc *__restrict__ gd, int32_t ng,
                                                      uint32_t *__restrict__ units) {
    const int32_t per = (ng + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x;
    const int32_t g0 = min(ng, (int32_t)threadIdx.x * per), g1 = min(ng, g0 + per);
    for (int list = 0; list < GROUP_LISTS; ++list) {
        uint32_t sum = 0;
        for (int32_t g = g0; g < g1; ++g)
            if (group_list(gd[g].G, gd[g].wk) == list) sum += gd[g].meta[2] * (uint32_t)gd[g].n_chunks;
        uint32_t total;
        uint32_t run = block_excl_sum(sum, &total);
        uint32_t *u = units + list * (ng + 1);
        for (int32_t g = g0; g < g1; ++g) {
            u[g] = run;
            if (group_list(gd[g].G, gd[g].wk) == list) run += gd[g].meta[2] * (uint32_t)gd[g].n_chunks;
        }
        if (threadIdx.x == 0) {
            u[ng] = total;
            units[GROUP_LISTS * (ng + 1) + list] = 0u;
        }
    }
}

// ------------------------------------------------------------ meet kernel
// The single-query meet kernel's scheme with a group in place of a query:
// persistent blocks take units (group, tile of its compacted walks, chunk of
// vb nodes with in-edges) from a device cursor, stage the tile's positions in
// LDS, and hand the pairs (v, entry) of a unit, v-major, to the waves in chunks
// of 64.  A lane keeps NS pairs in flight; a pair carries the LDS offset of
// its entry's block for the next step and the mask of members still tested.
// A step reads the positions of the members present at that step, then
// compares.  Counts go to 16-bit LDS counters per (member, node) (a unit
// holds at most TJ < 2^16 walks), flushed to the members' counts once per
// unit.  WK = 1 (stitched): the walk's first 2^k
// steps are its own draws, the rest is read from the segment index, one load
// per iteration, as in the single-query kernel.  WK = 2 (stratified): walk j
// of v is the fixed-length walk of slot pi_v(j) (the shuffle and the class
// search are done when the pair starts), it takes no stop draws, and a meet of
// member q adds Lemma 5's weight of the classes of walk j of s_q and of v to a
// 64-bit LDS sum per (member, node).

template <int GW>
struct GSlot {
    uint32_t pos;      // LDS offset of the entry's positions (16 bits) | its longest
                       // member walk << 16 | node index << 24
    uint32_t live;     // members still tested (bit q)
    uint32_t b;        // LDS offset of the entry's block for the next step
    uint32_t t;        // steps taken
    uint32_t o, d;     // current node: slot offset in E and in-degree
    WalkDraws rng;
    bool busy;
    uint32_t ph;       // stitched: 0 head; 1 node id, 2 pool offsets, 3 segment length,
                       // 4 tail step; 5 chain, 6 next segment's length
    uint32_t tsig, tm, tu, tseg, tsl;   // stitched tail: entry slot, chain index, position,
                                        // segment, its length
    uint32_t cv, jw;   // stratified: class (and last step) of walk (v, j), and j
};

// Compares the pair's position at step t with the members' positions at step
// t.  The entry's block for step t is the word of members with a position at
// t, then those positions in member order; the slot's offset b moves on to the
// next step's block (every step is compared once, in order).  A hit sends the
// lane to an exact pass that names the members; meets are rare, so the common
// step reads and compares only the positions of the members still walking.
// Returns the members still tested that meet at this step.
template <int GW>
__device__ __forceinline__ uint32_t group_compare(GSlot<GW> &w, const uint32_t *s_nodes) {
    const uint32_t B = w.b;
    const uint32_t am = s_nodes[B];
    const uint32_t c = (uint32_t)__popc(am);
    w.b = B + 1u + c;
    bool hit = false;
    // four positions per round; a read past the block takes word B instead,
    // and a false hit from it is cleared by the exact pass
    for (uint32_t i = 0; i < c; i += 4u) {
        uint32_t pv[4];
#pragma unroll
        for (uint32_t u = 0; u < 4u; ++u) pv[u] = s_nodes[i + u < c ? B + 1u + i + u : B];
#pragma unroll
        for (int u = 0; u < 4; ++u) hit |= pv[u] == w.o;
    }
    if (!hit) return 0u;
    uint32_t met = 0, m = am;
    for (uint32_t i = 0; i < c; ++i) {
        const uint32_t q = (uint32_t)__builtin_ctz(m);
        m &= m - 1u;
        if (s_nodes[B + 1u + i] == w.o) met |= 1u << q;
    }
    return met & w.live;
}

template <int NS, int GW, int WK>
__global__ __launch_bounds__(GROUP_BLOCK) void k_meet_group(const GroupDesc *__restrict__ gd, int32_t ng,
                                                            const uint32_t *__restrict__ ustart,
                                                            uint32_t *__restrict__ cursor,
                                                            unsigned long long *__restrict__ counters) {
    constexpr bool STITCHED = WK == 1, STRAT = WK == 2;
    constexpr int TJ = group_tile_j(GW, WK), TN = group_tile_nodes(GW, WK), GM = 4 * GW;
    __shared__ uint32_t s_nodes[TN];
    __shared__ uint32_t s_j[TJ];
    __shared__ uint16_t s_off[TJ];
    __shared__ uint32_t s_cnt[STRAT ? 1 : GM / 2 * MEET_VB];   // members 2i, 2i+1 in the low, high half
    // stratified: weighted sums per (member, node), the nodes' shuffle keys,
    // the class starts
    constexpr int VBW = group_strat_vb(GW);
    __shared__ unsigned long long s_w[STRAT ? GM * VBW : 1];
    __shared__ uint4 s_fk[STRAT ? MEET_VB : 1];
    __shared__ uint32_t s_ccum[STRAT ? MAX_CAP + 2 : 1];
    __shared__ uint32_t s_vid[MEET_VB];
    __shared__ uint2 s_vrow[MEET_VB];
    __shared__ uint32_t s_srcm[MEET_VB];   // members whose source is the node
    __shared__ uint8_t s_maxl[TJ];         // longest member walk of the entry
    __shared__ uint32_t s_unit, s_item;

    const int lane = threadIdx.x & 63;
    const uint32_t n_units = ustart[ng];
    uint32_t cur_g = 0xffffffffu, cur_tile = 0xffffffffu;
    uint32_t K = 0;
    uint32_t st_moves = 0, st_draws = 0, st_meets = 0, st_pairs = 0, st_tail = 0;

    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(cursor, 1u);
        __syncthreads();
        const uint32_t unit = s_unit;
        if (unit >= n_units) break;
        int32_t lo = 0, hi = ng;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (ustart[mid] <= unit) lo = mid; else hi = mid;
        }
        const int32_t gi = lo;
        const GroupDesc &d = gd[gi];
        const int32_t n_chunks = (int32_t)uni((uint32_t)d.n_chunks);
        const int32_t vb = (int32_t)uni((uint32_t)d.vb);
        const int32_t G = (int32_t)uni((uint32_t)d.G);
        const int32_t gw = (int32_t)uni((uint32_t)d.gw);
        const uint32_t local = unit - ustart[gi];
        const uint32_t tile = local / (uint32_t)n_chunks;
        const uint32_t chunk = local - tile * (uint32_t)n_chunks;
        const PhiloxKey key{uni(d.k0), uni(d.k1)};
        const uint32_t T = uni(d.T);
        const uint32_t gmask = G >= 32 ? 0xffffffffu : (1u << G) - 1u;
        const uint32_t NN = uni((uint32_t)d.Rmax), sa = uni((uint32_t)d.sa), sb = uni((uint32_t)d.sb);
        const int32_t phi = (int32_t)uni((uint32_t)d.L);
        if ((uint32_t)gi != cur_g || tile != cur_tile) {
            const uint32_t k0 = d.tiles[tile], k1 = d.tiles[tile + 1];
            const uint32_t nb = d.joff[k0], ne = d.joff[k1];
            K = k1 - k0;
            for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
                s_j[i] = d.jj[k0 + i];
                s_off[i] = (uint16_t)(d.joff[k0 + i] - nb);
                uint32_t mx = 0;
                for (int32_t wd = 0; wd < gw; ++wd) {
                    const uint32_t lw = d.glen[(size_t)(k0 + i) * gw + wd];
                    mx = max(mx, max(max(byte_of(lw, 0), byte_of(lw, 1)), max(byte_of(lw, 2), byte_of(lw, 3))));
                }
                s_maxl[i] = (uint8_t)mx;
            }
            for (uint32_t i = threadIdx.x; i < ne - nb; i += blockDim.x) s_nodes[i] = d.pos[nb + i];
            if (STRAT)
                for (uint32_t i = threadIdx.x; i < (uint32_t)phi + 2; i += blockDim.x)
                    s_ccum[i] = d.tab->ccum[i];
            cur_g = (uint32_t)gi;
            cur_tile = tile;
        }
        const int32_t vbase = (int32_t)chunk * vb;
        const uint32_t nv = (uint32_t)min(vb, d.n_active - vbase);
        if (STRAT)
            for (uint32_t i = threadIdx.x; i < GM * VBW; i += blockDim.x) s_w[i] = 0ull;
        else
            for (uint32_t i = threadIdx.x; i < GM / 2 * MEET_VB; i += blockDim.x) s_cnt[i] = 0u;
        for (uint32_t i = threadIdx.x; i < nv; i += blockDim.x) {
            const uint32_t id = (uint32_t)d.active[vbase + (int32_t)i];
            s_vid[i] = id;
            s_vrow[i] = d.nodes[id];
            uint32_t m = 0;
            for (int32_t q = 0; q < G; ++q) m |= (uint32_t)((uint32_t)d.s[q] == id) << q;
            s_srcm[i] = m;
            if (STRAT) s_fk[i] = philox4x32_10(id, 0u, 0u, DOM_SHUFFLE, key);
        }
        if (threadIdx.x == 0) s_item = 0u;
        __syncthreads();

        // item i = vl * K + k for node vl < nv and entry k < K
        const uint32_t total = nv * K;
        uint32_t ci = 0, ce = 0, cvl = 0, ck = 0;
        bool drained = false;
        GSlot<GW> sl[NS];
#pragma unroll
        for (int qq = 0; qq < NS; ++qq) {
            sl[qq].busy = false;
            sl[qq].ph = 0;
        }

        for (;;) {
            // ---- refill idle slots; a pair with no member to test (each
            // member's source is v), or a stratified walk of class 0, is skipped
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) {
                uint64_t need = __ballot(!sl[qq].busy);
                while (need != 0ull) {
                    if (ci == ce) {
                        if (drained) break;
                        uint32_t x = 0;
                        if (lane == 0) x = atomicAdd(&s_item, ITEM_CHUNK);
                        x = __builtin_amdgcn_readfirstlane(x);
                        if (x >= total) {
                            drained = true;
                            break;
                        }
                        ci = x;
                        ce = min(x + ITEM_CHUNK, total);
                        cvl = x / K;
                        ck = x - cvl * K;
                    }
                    const uint32_t want = (uint32_t)__popcll(need);
                    const uint32_t avail = ce - ci;
                    const uint32_t take = avail < want ? avail : want;
                    const uint32_t rank = lane_rank(need);
                    const bool mine = ((need >> lane) & 1ull) && rank < take;
                    bool filled = false;
                    if (mine) {
                        uint32_t k = ck + rank, vl = cvl;
                        while (k >= K) {
                            k -= K;
                            ++vl;
                        }
                        // members tested: all but those whose source is v (a
                        // member whose walk j is empty never reads a position)
                        const uint32_t live = gmask & ~s_srcm[vl];
                        uint32_t r = 0, cv = 0;
                        if (STRAT && live) {
                            r = shuffle_slot(s_j[k], NN, sa, sb, s_fk[vl]);
                            cv = slot_class(r, s_ccum, phi);
                        }
                        if (live && (!STRAT || cv > 0u)) {
                            const uint2 row = s_vrow[vl];
                            GSlot<GW> &w = sl[qq];
                            if (STRAT) {
                                w.rng = walk_draws_begin(s_vid[vl], r, key, DOM_STRAT);
                                w.cv = cv;
                                w.jw = s_j[k];
                            } else {
                                w.rng = walk_draws_begin(s_vid[vl], s_j[k], key);
                            }
                            w.pos = (uint32_t)s_off[k] | ((uint32_t)s_maxl[k] << 16) | (vl << 24);
                            w.live = live;
                            w.b = s_off[k];
                            w.t = 0;
                            w.o = row.x;
                            w.d = row.y;
                            w.busy = true;
                            w.ph = 0;
                            filled = true;
                            ++st_pairs;
                        }
                    }
                    need &= ~__ballot(filled);
                    ci += take;
                    ck += take;
                    while (ck >= K && K > 0) {
                        ck -= K;
                        ++cvl;
                    }
                }
            }
            bool any = false;
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) any |= sl[qq].busy;
            if (__ballot(any) == 0ull) {
                if (drained) break;
                continue;
            }

            // ---- head steps: draws, then one load per slot (a head step's
            // gather or the load its stitched tail phase needs), then compares
            bool go[NS];
            uint32_t at[NS];
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) {
                go[qq] = false;
                at[qq] = 0;
                if (sl[qq].busy && !(STITCHED && sl[qq].ph)) {
                    ++sl[qq].t;
                    const uint2 x = walk_draw_next(sl[qq].rng, key);
                    ++st_draws;
                    if (!STRAT && x.x >= T) {
                        sl[qq].busy = false;
                    } else {
                        go[qq] = true;
                        at[qq] = sl[qq].o + pick32(x.y, sl[qq].d);
                    }
                }
            }
            uint2 e[NS];
            uint32_t tv[NS];
            int64_t tb[NS], te[NS];
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) {
                if (go[qq]) e[qq] = load_edge(d.E + at[qq]);
                if (STITCHED && sl[qq].busy && sl[qq].ph) {
                    const GSlot<GW> &w = sl[qq];
                    switch (w.ph) {
                    case 1: tv[qq] = d.ix.node_of[w.o]; break;
                    case 2: tb[qq] = d.ix.pool_off[w.tsig]; te[qq] = d.ix.pool_off[w.tsig + 1]; break;
                    case 3:
                    case 6: tv[qq] = d.ix.seg_lens[w.tseg]; break;
                    case 4: tv[qq] = d.ix.seg[(size_t)w.tseg * d.ix.seg_len + w.tu]; break;
                    default: tv[qq] = d.ix.chain[(size_t)w.tsig * d.ix.width + w.tm + 1]; break;
                    }
                }
            }
            // ---- one compare per slot that reached a new position (a head
            // step's node, or a stitched tail step read from the index), then
            // the end tests of its phase; the other tail phases only advance
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) {
                GSlot<GW> &w = sl[qq];
                const bool tail_step = STITCHED && !go[qq] && w.busy && w.ph == 4u;
                if (go[qq]) {
                    ++st_moves;
                    w.o = e[qq].x;
                    w.d = e[qq].y;
                } else if (tail_step) {
                    ++w.t;
                    ++st_tail;
                    w.o = tv[qq];
                    ++w.tu;
                }
                if (go[qq] || tail_step) {
                    const uint32_t met = group_compare(w, s_nodes);
                    if (met) {
                        const uint32_t vl = w.pos >> 24;
                        st_meets += (uint32_t)__popc(met);
                        w.live &= ~met;
                        for (uint32_t m = met; m; m &= m - 1u) {
                            const uint32_t q = (uint32_t)__builtin_ctz(m);
                            if (STRAT)
                                atomicAdd(&s_w[q * VBW + vl],
                                          strat_weight(d.tab->a, d.scls[q][w.jw], w.cv));
                            else
                                atomicAdd(&s_cnt[(q >> 1) * MEET_VB + vl], 1u << (16 * (q & 1u)));
                        }
                    }
                }
                if (go[qq]) {
                    // the pair ends with its last member walk (or, stratified,
                    // the class of walk (v, j)), when every member tested has
                    // met, or at a node without in-neighbours
                    if (w.live == 0u || w.d == 0u || w.t == ((w.pos >> 16) & 0xffu) ||
                        (STRAT && w.t == w.cv))
                        w.busy = false;
                    else if (STITCHED && w.t == (uint32_t)d.ix.seg_len)
                        w.ph = 1;   // the head made all its moves: enter a pool slot of this node
                    continue;
                }
                if (!(STITCHED && w.busy && w.ph)) continue;
                switch (w.ph) {
                case 1:   // the end node's id
                    w.tsig = tv[qq];
                    w.ph = 2;
                    break;
                case 2: { // its pool: slot picked by draw (v, j, 0, DOM_ENTRY)
                    const uint4 x = philox4x32_10(s_vid[w.pos >> 24], w.rng.j, 0u, DOM_ENTRY, key);
                    w.tsig = (uint32_t)(tb[qq] + (int64_t)pick64(x.x, (uint64_t)(te[qq] - tb[qq])));
                    w.tseg = w.tsig;
                    w.tm = 0;
                    w.ph = 3;
                    break;
                }
                case 3:
                case 6:   // a segment's length
                    w.tsl = tv[qq];
                    w.tu = 0;
                    w.ph = 4;
                    if (w.tsl == 0u) w.busy = false;
                    break;
                case 4:   // after a tail step
                    if (w.live == 0u || w.t == ((w.pos >> 16) & 0xffu)) {
                        w.busy = false;
                    } else if (w.tu == w.tsl) {
                        if (w.tsl < (uint32_t)d.ix.seg_len || w.tm + 1 >= (uint32_t)d.ix.width)
                            w.busy = false;
                        else
                            w.ph = 5;
                    }
                    break;
                default:  // the chain's next segment
                    ++w.tm;
                    w.tseg = tv[qq];
                    if (w.tseg == NIL) w.busy = false;
                    else w.ph = 6;
                    break;
                }
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < (uint32_t)G * nv; i += blockDim.x) {
            const uint32_t q = i / nv, vi = i - q * nv;
            if (STRAT) {
                const unsigned long long c = s_w[q * VBW + vi];
                if (c) atomicAdd(&d.wsum[q][s_vid[vi]], c);
            } else {
                const uint32_t c = (s_cnt[(q >> 1) * MEET_VB + vi] >> (16 * (q & 1u))) & 0xffffu;
                if (c) atomicAdd(&d.cnt[q][s_vid[vi]], c);
            }
        }
    }

    unsigned long long v0 = st_moves, v1 = st_draws, v2 = st_meets, v3 = st_tail, v4 = st_pairs;
    for (int dd = 32; dd > 0; dd >>= 1) {
        v0 += __shfl_xor(v0, dd, 64);
        v1 += __shfl_xor(v1, dd, 64);
        v2 += __shfl_xor(v2, dd, 64);
        v3 += __shfl_xor(v3, dd, 64);
        v4 += __shfl_xor(v4, dd, 64);
    }
    if (lane == 0) {
        atomicAdd(&counters[C_MOVES], v0);
        atomicAdd(&counters[C_DRAWS], v1);
        atomicAdd(&counters[C_MEETS], v2);
        atomicAdd(&counters[C_TAIL], v3);
        atomicAdd(&counters[C_PAIRS], v4);
    }
}

#ifndef SRK_GROUP_SLOTS_STITCHED
#define SRK_GROUP_SLOTS_STITCHED 2
#endif

template <int NS, int GW, int WK>
int group_grid_blocks() {
    static const int blocks = [] {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_meet_group<NS, GW, WK>,
                                                           GROUP_BLOCK, 0);
        if (cus <= 0) cus = 256;
        if (per <= 0) per = 1;
        return cus * per;
    }();
    return blocks;
}

template <int NS, int GW, int WK>
void launch_group_list(const GroupSet &gs, int list, unsigned long long *counters, hipStream_t st) {
    if (gs.units_bound[list] <= 0) return;
    const int blocks = (int)std::min<int64_t>(gs.units_bound[list], group_grid_blocks<NS, GW, WK>());
    k_meet_group<NS, GW, WK><<<blocks, GROUP_BLOCK, 0, st>>>(
        gs.desc, gs.ng, gs.units + (size_t)list * (gs.ng + 1),
        gs.units + GROUP_LISTS * ((size_t)gs.ng + 1) + list, counters);
}

}  // namespace

int32_t group_max_tiles(int64_t Rmax, int64_t sum_RL, int32_t L, int32_t G, int32_t wk) {
    const int GW = group_gw(G);
    const int64_t NW = group_tile_nodes(GW, wk) - (int64_t)(G + 1) * L;
    return (int32_t)(2 + Rmax / group_tile_j(GW, wk) + group_pos_words(Rmax, sum_RL, L) / NW);
}

// A unit's pairs are (its vb nodes) x (the tile's entries); each unit has
// fixed work (the claim, three barriers, staging its nodes, flushing its
// counters, the wait for its longest pair).  A group's tile holds few entries
// (every entry carries all members' positions), so small units pay that work
// over few pairs: on the n = 2^22 graph a 32-member group took 855 ms with 256
// nodes per unit, 894 with 128, 971 with 64 and 1121 with 32 (stitched: 994 /
// 1049 / 1161 / 1366).  Groups therefore take the largest unit that still
// leaves 64 chunks of nodes, whatever the lone queries were tuned to.
int32_t group_unit_nodes(int32_t n_active, int32_t G, int32_t wk) {
    int32_t vb = MEET_VB;
    while (vb > 32 && (n_active + vb - 1) / vb < 64) vb >>= 1;
    if (wk == 2 && G > 8) vb = std::min(vb, GROUP_STRAT32_VB);   // the LDS sums' node limit
    return vb;
}

void describe_group(const QueryDesc *const *members, int32_t G, GroupDesc *gd) {
    const QueryDesc &d0 = *members[0];
    *gd = GroupDesc{};
    gd->nodes = d0.nodes;
    gd->E = d0.E;
    gd->active = d0.active;
    gd->n_active = d0.n_active;
    gd->G = G;
    gd->gw = (G + 3) / 4;
    gd->wk = d0.kind == K_GROUPED_STITCHED ? 1 : d0.kind == K_GROUPED_STRAT ? 2 : 0;
    gd->vb = group_unit_nodes(d0.n_active, G, gd->wk);
    gd->n_chunks = (gd->n_active + gd->vb - 1) / gd->vb;
    gd->ix = d0.ix;
    gd->tab = d0.tab;
    gd->sa = d0.sa;
    gd->sb = d0.sb;
    gd->L = d0.L;
    gd->k0 = d0.k0;
    gd->k1 = d0.k1;
    gd->T = d0.T;
    for (int32_t q = 0; q < G; ++q) {
        const QueryDesc &dq = *members[q];
        gd->s[q] = dq.s;
        gd->R[q] = dq.R;
        gd->sw[q] = dq.sw;
        gd->slen[q] = dq.slen;
        gd->cnt[q] = dq.cnt;
        gd->wsum[q] = dq.wsum;
        gd->scls[q] = dq.scls;
        gd->Rmax = std::max(gd->Rmax, dq.R);
    }
}

size_t group_buffers(GroupDesc *gd, int64_t sum_RL, char *base) {
    size_t at = 0;
    auto take = [&](size_t b) {
        char *r = base ? base + at : nullptr;
        at += (b + 255) & ~(size_t)255;
        return r;
    };
    const int32_t mt = group_max_tiles(gd->Rmax, sum_RL, gd->L, gd->G, gd->wk);
    gd->jj = (uint32_t *)take(4 * (size_t)gd->Rmax);
    gd->joff = (uint32_t *)take(4 * ((size_t)gd->Rmax + 1));
    gd->glen = (uint32_t *)take(4 * (size_t)gd->Rmax * (size_t)gd->gw);
    gd->pos = (uint32_t *)take(4 * (size_t)group_pos_words(gd->Rmax, sum_RL, gd->L));
    gd->tiles = (uint32_t *)take(4 * ((size_t)mt + 1));
    gd->meta = (uint32_t *)take(32);
    return at;
}

static_assert(GROUP_LISTS == 6, "one launch below per group kernel instance");

int launch_groups(const GroupSet &gs, unsigned long long *counters, hipStream_t st) {
    if (gs.ng <= 0) return SIMRANK_OK;
    k_group_compact<<<gs.ng, 1024, 0, st>>>(gs.desc);
    k_group_units<<<1, 1024, 0, st>>>(gs.desc, gs.ng, gs.units);
    launch_group_list<SRK_GROUP_SLOTS, 2, 0>(gs, 0, counters, st);
    launch_group_list<SRK_GROUP_SLOTS, 8, 0>(gs, 1, counters, st);
    launch_group_list<SRK_GROUP_SLOTS_STITCHED, 2, 1>(gs, 2, counters, st);
    launch_group_list<SRK_GROUP_SLOTS_STITCHED, 8, 1>(gs, 3, counters, st);
    launch_group_list<SRK_GROUP_SLOTS, 2, 2>(gs, 4, counters, st);
    launch_group_list<SRK_GROUP_SLOTS, 8, 2>(gs, 5, counters, st);
    SRK_HIP(hipGetLastError());
    return SIMRANK_OK;
}

}  // namespace srk
